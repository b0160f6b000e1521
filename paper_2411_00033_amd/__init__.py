"""MI355X (gfx950) Legendre <-> Chebyshev coefficient transforms.

The modal fast multipole method of Mortensen (arXiv 2411.00033, Alg. 4) behind the
C ABI of ``include/leg2cheb.h``; this package is the thin Python side of it.
PyTorch supplies device memory and streams; all arithmetic runs in the HIP
library ``libleg2cheb.so``.

    import torch, paper_2411_00033_amd as l2c
    plan = l2c.Plan(1_000_000, l2c.LEG2CHEB, leaf_size=64, rank=18)
    z = plan.execute(x)            # x: float64 CUDA tensor, shape (n,) or (batch, n)
"""
from __future__ import annotations

import numpy as np

from . import _lib
from ._lib import (  # noqa: F401  (re-exported ABI names)
    L2C_BF16X2, L2C_FP16X2, L2C_CHEB2LEG, L2C_EHIP, L2C_EINVAL, L2C_ENOMEM, L2C_EUNSUPPORTED, L2C_FP32, L2C_FP64,
    L2C_LEG2CHEB, L2C_OK, L2C_OPT_DIRECT, L2C_OPT_EXCHANGE_TIMEOUT_US, L2C_OPT_SINGLE_LAUNCH,
    L2C_STATUS_EXCHANGE, L2C_STATUS_STREAM, L2C_STATUS_WORKERS, L2C_PATH_DIRECT, L2C_PATH_SINGLE, L2C_PATH_BATCHED, L2C_PATH_DENSE, L2C_PATH_THREE,
    L2C_PATH_REGEN, L2C_TABLES_STORED, L2C_TABLES_REGEN, L2CError,
    TABLE_AHAT, TABLE_B, TABLE_T, TABLE_W, leg2cheb_destroy, leg2cheb_execute, leg2cheb_execute_noalloc, leg2cheb_plan, leg2cheb_plan_ex,
    leg2cheb_plan_export, leg2cheb_plan_info, leg2cheb_plan_set_option, leg2cheb_plan_status,
    leg2cheb_rank_supported, leg2cheb_debug_alloc_hook, leg2cheb_set_timing_events, leg2cheb_batch_plan, leg2cheb_batch_execute,
    leg2cheb_batch_info, leg2cheb_batch_destroy, leg2cheb_batch_tuning,
    L2C_LEG2GRID, L2C_GRID2LEG, L2C_MODAL, L2C_NODAL, leg2cheb_plan_basis, leg2cheb_plan_tables, leg2cheb_plan_cached,
    leg2cheb_plan_cache_size, leg2cheb_dct_plan, leg2cheb_dct_execute, leg2cheb_dct_destroy, leg2cheb_grid_plan,
    leg2cheb_grid_execute, leg2cheb_grid_destroy, leg2cheb_grid_fmm, leg2cheb_grid_dct,
)

LEG2CHEB, CHEB2LEG = L2C_LEG2CHEB, L2C_CHEB2LEG
LEG2GRID, GRID2LEG = L2C_LEG2GRID, L2C_GRID2LEG


def _torch():
    import torch
    return torch


class Plan:
    """Owns one library plan (device tables + workspace) for transforms of length n."""

    def __init__(self, n: int, direction: int = LEG2CHEB, leaf_size: int = 64, rank: int = 18,
                 precision: int = L2C_FP64, max_batch: int = 1, stream=None, basis: int = L2C_MODAL,
                 cached: bool = False, tables: int = L2C_TABLES_STORED):
        torch = _torch()
        st = stream if stream is not None else torch.cuda.current_stream()
        self.device = torch.cuda.current_device()
        if tables != L2C_TABLES_STORED:   # FP64, modal: far-field blocks regenerated per execute
            if precision != L2C_FP64 or basis != L2C_MODAL or cached:
                raise ValueError("tables=L2C_TABLES_REGEN takes an FP64 plan in the modal basis, not cached")
            self.handle = leg2cheb_plan_tables(n, direction, leaf_size, rank, max_batch, tables, st.cuda_stream)
        elif cached:   # a reference to the shared plan of the plan cache (close releases it)
            self.handle = leg2cheb_plan_cached(n, direction, leaf_size, rank, precision, max_batch, basis,
                                               st.cuda_stream)
        elif basis == L2C_MODAL:
            self.handle = leg2cheb_plan_ex(n, direction, leaf_size, rank, precision, max_batch, st.cuda_stream)
        else:
            self.handle = leg2cheb_plan_basis(n, direction, leaf_size, rank, precision, max_batch, basis,
                                              st.cuda_stream)
        self.n, self.direction, self.leaf_size, self.rank = int(n), int(direction), int(leaf_size), int(rank)

    @property
    def info(self) -> dict:
        return leg2cheb_plan_info(self.handle)

    def execute(self, x, out=None, stream=None):
        """Transform x (float64 CUDA tensor, (n,) or (batch, n), contiguous) into out."""
        torch = _torch()
        if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous float64 CUDA tensor")
        if x.shape[-1] != self.n or x.dim() not in (1, 2):
            raise ValueError("x must have shape (n,) or (batch, n) with n = %d" % self.n)
        if x.device.index != self.device:
            raise ValueError("x is on cuda:%d but the plan was made on cuda:%d" % (x.device.index, self.device))
        if out is None:
            out = torch.empty_like(x)
        elif out.shape != x.shape or out.dtype != torch.float64 or not out.is_contiguous() or out.device != x.device:
            raise ValueError("out must match x in shape, dtype, device and be contiguous")
        batch = 1 if x.dim() == 1 else x.shape[0]
        st = stream if stream is not None else torch.cuda.current_stream()
        leg2cheb_execute(self.handle, x.data_ptr(), out.data_ptr(), batch, st.cuda_stream)
        return out

    __call__ = execute

    def export(self, table: int) -> np.ndarray:
        """A plan table in the canonical layout documented in include/leg2cheb.h (host copy)."""
        need = leg2cheb_plan_export(self.handle, table)
        buf = np.empty(need // 8, dtype=np.float64)
        leg2cheb_plan_export(self.handle, table, buf.ctypes.data, need)
        return buf

    def set_direct(self, on: bool) -> None:
        """Alg. 1 directly for short FP64 transforms (default where allowed) or Alg. 4."""
        leg2cheb_plan_set_option(self.handle, L2C_OPT_DIRECT, 1 if on else 0)

    def set_single_launch(self, on: bool) -> None:
        """Choose the single-launch path (default when the plan allows it) or three launches."""
        leg2cheb_plan_set_option(self.handle, L2C_OPT_SINGLE_LAUNCH, 1 if on else 0)

    def set_exchange_timeout_us(self, us: int) -> None:
        """Bound of the single-launch kernel's waits for other workgroups (default 10^6 us)."""
        leg2cheb_plan_set_option(self.handle, L2C_OPT_EXCHANGE_TIMEOUT_US, int(us))

    @property
    def status(self) -> int:
        """Status bits of the single-launch path since the last query (0 = every wait
        completed); synchronizes the device and clears the bits."""
        return leg2cheb_plan_status(self.handle)

    def set_timing_events(self, before, after) -> None:
        """Record torch.cuda.Event pair around the far-field kernel of each execute (None: off)."""
        leg2cheb_set_timing_events(self.handle, before.cuda_event if before is not None else 0,
                                   after.cuda_event if after is not None else 0)

    def close(self) -> None:
        if getattr(self, "handle", None):
            leg2cheb_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _rows(x, n: int, device: int, out):
    """Check x (and out) as (n,) or (batch, n) contiguous float64 CUDA tensors; return out, batch."""
    torch = _torch()
    if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous float64 CUDA tensor")
    if x.shape[-1] != n or x.dim() not in (1, 2):
        raise ValueError("x must have shape (n,) or (batch, n) with n = %d" % n)
    if x.device.index != device:
        raise ValueError("x is on cuda:%d but the plan was made on cuda:%d" % (x.device.index, device))
    if out is None:
        out = torch.empty_like(x)
    elif out.shape != x.shape or out.dtype != torch.float64 or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must match x in shape, dtype, device and be contiguous")
    return out, 1 if x.dim() == 1 else x.shape[0]


class _Handle:
    _destroy = None

    def close(self) -> None:
        if getattr(self, "handle", None):
            type(self)._destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Dct(_Handle):
    """DCT of kind 2 (y_k = sum_j x_j cos(pi k (j + 1/2) / n)) or kind 3 (y_j = sum_k x_k
    cos(pi k (j + 1/2) / n)) on the library's FFT; n with prime factors 2, 3, 5, 7 only."""
    _destroy = staticmethod(leg2cheb_dct_destroy)

    def __init__(self, n: int, kind: int = 2, max_batch: int = 1, stream=None):
        torch = _torch()
        st = stream if stream is not None else torch.cuda.current_stream()
        self.device = torch.cuda.current_device()
        self.handle = leg2cheb_dct_plan(n, kind, max_batch, st.cuda_stream)
        self.n, self.kind = int(n), int(kind)

    def execute(self, x, out=None, stream=None):
        torch = _torch()
        out, batch = _rows(x, self.n, self.device, out)
        st = stream if stream is not None else torch.cuda.current_stream()
        leg2cheb_dct_execute(self.handle, x.data_ptr(), out.data_ptr(), batch, st.cuda_stream)
        return out

    __call__ = execute


class GridPlan(_Handle):
    """Legendre series on the n Chebyshev-Gauss points x_j = cos((j + 1/2) pi / n)
    (LEG2GRID: values sum_k f_k P_k(x_j)) and back (GRID2LEG: Legendre coefficients of
    the interpolant): the FMM plus the DCT of kind 3, or the DCT of kind 2 plus the FMM."""
    _destroy = staticmethod(leg2cheb_grid_destroy)

    def __init__(self, n: int, direction: int = L2C_LEG2GRID, leaf_size: int = 64, rank: int = 18,
                 max_batch: int = 1, stream=None):
        torch = _torch()
        st = stream if stream is not None else torch.cuda.current_stream()
        self.device = torch.cuda.current_device()
        self.handle = leg2cheb_grid_plan(n, direction, leaf_size, rank, max_batch, st.cuda_stream)
        self.n, self.direction = int(n), int(direction)

    @property
    def fmm_info(self) -> dict:
        return leg2cheb_plan_info(leg2cheb_grid_fmm(self.handle))

    def execute(self, x, out=None, stream=None):
        torch = _torch()
        out, batch = _rows(x, self.n, self.device, out)
        st = stream if stream is not None else torch.cuda.current_stream()
        leg2cheb_grid_execute(self.handle, x.data_ptr(), out.data_ptr(), batch, st.cuda_stream)
        return out

    __call__ = execute


class BatchPlan:
    """A ragged batch: transforms of lengths n[i] and directions direction[i], planned together
    (one table set per group of equal levels, half-leaf and direction)."""

    def __init__(self, n, direction, leaf_size=None, rank=None, precision: int = L2C_FP64, tuning=None,
                 stream=None):
        """tuning: a list of (n_max, leaf_size, rank) size buckets; leaf_size and rank alone
        make one bucket for every length; with neither, the library's own table is used."""
        torch = _torch()
        if len(n) != len(direction) or len(n) == 0:
            raise ValueError("n and direction must be non-empty and of equal length")
        if tuning is None and (leaf_size is not None or rank is not None):
            default = 18 if precision == L2C_FP64 else 16
            tuning = [(1 << 62, 64 if leaf_size is None else leaf_size, default if rank is None else rank)]
        st = stream if stream is not None else torch.cuda.current_stream()
        self.device = torch.cuda.current_device()
        self.n = [int(v) for v in n]
        self.direction = [int(v) for v in direction]
        self.handle = leg2cheb_batch_plan(self.n, self.direction, precision, tuning, st.cuda_stream)

    @property
    def info(self) -> dict:
        return leg2cheb_batch_info(self.handle)

    def execute(self, xs, outs=None, stream=None):
        """Transform every xs[i] (float64 CUDA tensor of n[i] values) into outs[i]."""
        torch = _torch()
        if len(xs) != len(self.n):
            raise ValueError("expected %d input tensors" % len(self.n))
        for x, n in zip(xs, self.n):
            if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != n:
                raise ValueError("each input must be a contiguous float64 CUDA tensor of its length")
            if x.device.index != self.device:
                raise ValueError("inputs must be on cuda:%d" % self.device)
        if outs is None:
            outs = [torch.empty_like(x) for x in xs]
        for o, n in zip(outs, self.n):
            if o.dtype != torch.float64 or not o.is_cuda or not o.is_contiguous() or o.numel() != n:
                raise ValueError("each output must be a contiguous float64 CUDA tensor of its length")
        st = stream if stream is not None else torch.cuda.current_stream()
        leg2cheb_batch_execute(self.handle, [x.data_ptr() for x in xs], [o.data_ptr() for o in outs],
                               st.cuda_stream)
        return outs

    __call__ = execute

    def execute_ptrs(self, in_ptrs, out_ptrs, stream=None) -> None:
        """As execute, for callers that hold the device pointers (ints, FP64, n[i] values each)
        already: no per-tensor checks here; the library still rejects null pointers and
        overlapping outputs."""
        torch = _torch()
        if len(in_ptrs) != len(self.n) or len(out_ptrs) != len(self.n):
            raise ValueError("expected %d input and output pointers" % len(self.n))
        st = stream if stream is not None else torch.cuda.current_stream()
        leg2cheb_batch_execute(self.handle, in_ptrs, out_ptrs, st.cuda_stream)

    def close(self) -> None:
        if getattr(self, "handle", None):
            leg2cheb_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def transform(x, direction: int = LEG2CHEB, leaf_size: int = 64, rank: int = 18):
    """One-shot transform (builds and frees a plan)."""
    batch = 1 if x.dim() == 1 else x.shape[0]
    with Plan(x.shape[-1], direction, leaf_size, rank, max_batch=batch) as p:
        out = p.execute(x)
        _torch().cuda.current_stream().synchronize()
        return out
