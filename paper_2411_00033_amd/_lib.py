"""ctypes binding of libleg2cheb.so (include/leg2cheb.h).

Argument marshalling only: every step of the transform runs in the HIP library.
If the library is missing or cannot be loaded, every call raises; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libleg2cheb.so")

L2C_LEG2CHEB, L2C_CHEB2LEG = 0, 1
L2C_FP64, L2C_FP32, L2C_BF16X2, L2C_FP16X2 = 0, 1, 2, 3
L2C_OK, L2C_EINVAL, L2C_ENOMEM, L2C_EHIP, L2C_EUNSUPPORTED = 0, -1, -2, -3, -4
TABLE_AHAT, TABLE_T, TABLE_B, TABLE_W = 0, 1, 2, 3
L2C_PATH_DIRECT, L2C_PATH_THREE, L2C_PATH_SINGLE, L2C_PATH_BATCHED, L2C_PATH_DENSE, L2C_PATH_REGEN = 0, 1, 2, 3, 4, 5
L2C_OPT_SINGLE_LAUNCH, L2C_OPT_DIRECT, L2C_OPT_EXCHANGE_TIMEOUT_US = 1, 2, 3
L2C_STATUS_EXCHANGE, L2C_STATUS_WORKERS, L2C_STATUS_STREAM = 1, 2, 4
L2C_LEG2GRID, L2C_GRID2LEG = 0, 1
L2C_MODAL, L2C_NODAL = 0, 1
L2C_TABLES_STORED, L2C_TABLES_REGEN = 0, 1

EXPORTED = (
    "leg2cheb_plan", "leg2cheb_plan_ex", "leg2cheb_plan_basis", "leg2cheb_plan_tables", "leg2cheb_plan_cached",
    "leg2cheb_plan_cache_size",
    "leg2cheb_execute", "leg2cheb_execute_noalloc", "leg2cheb_destroy",
    "leg2cheb_plan_info",
    "leg2cheb_plan_export", "leg2cheb_plan_set_option", "leg2cheb_plan_status", "leg2cheb_set_timing_events",
    "leg2cheb_rank_supported", "leg2cheb_strerror",
    "leg2cheb_batch_plan", "leg2cheb_batch_execute", "leg2cheb_batch_info", "leg2cheb_batch_destroy",
    "leg2cheb_batch_tuning", "leg2cheb_debug_alloc_hook", "leg2cheb_debug_check_geometry",
    "leg2cheb_dct_plan", "leg2cheb_dct_execute", "leg2cheb_dct_destroy",
    "leg2cheb_grid_plan", "leg2cheb_grid_execute", "leg2cheb_grid_destroy", "leg2cheb_grid_fmm", "leg2cheb_grid_dct",
)


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("n_pad", ctypes.c_int64),
        ("levels", ctypes.c_int32), ("s", ctypes.c_int32), ("rank", ctypes.c_int32),
        ("direction", ctypes.c_int32), ("precision", ctypes.c_int32), ("path", ctypes.c_int32),
        ("n_blocks", ctypes.c_int64), ("n_submatrices", ctypes.c_int64),
        ("table_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64), ("ahat_bytes", ctypes.c_int64),
        ("basis", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TuningBucket(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int64), ("leaf_size", ctypes.c_int32), ("rank", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("buckets", ctypes.POINTER(TuningBucket))]


class L2CError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (what, strerror(code), code))


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libleg2cheb.so not found at %s; build it with "
                          "`python -m paper_2411_00033_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.leg2cheb_plan.argtypes = [ctypes.POINTER(vp), i64, ci, ci, ci]
    lib.leg2cheb_plan_ex.argtypes = [ctypes.POINTER(vp), i64, ci, ci, ci, ci, i64, vp]
    lib.leg2cheb_plan_basis.argtypes = [ctypes.POINTER(vp), i64, ci, ci, ci, ci, i64, ci, vp]
    lib.leg2cheb_plan_cached.argtypes = [ctypes.POINTER(vp), i64, ci, ci, ci, ci, i64, ci, vp]
    lib.leg2cheb_plan_tables.argtypes = [ctypes.POINTER(vp), i64, ci, ci, ci, i64, ci, vp]
    lib.leg2cheb_plan_cache_size.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.leg2cheb_execute.argtypes = [vp, vp, vp, i64, vp]
    lib.leg2cheb_execute_noalloc.argtypes = [vp, vp, vp, i64, vp]
    lib.leg2cheb_destroy.argtypes = [vp]
    lib.leg2cheb_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.leg2cheb_plan_export.argtypes = [vp, ci, vp, i64, ctypes.POINTER(i64)]
    lib.leg2cheb_plan_set_option.argtypes = [vp, ci, i64]
    lib.leg2cheb_plan_status.argtypes = [vp, ctypes.POINTER(ci)]
    lib.leg2cheb_set_timing_events.argtypes = [vp, vp, vp]
    lib.leg2cheb_rank_supported.argtypes = [ci]
    lib.leg2cheb_debug_check_geometry.argtypes = [i64, ci, ci]
    lib.leg2cheb_strerror.argtypes = [ci]
    lib.leg2cheb_strerror.restype = ctypes.c_char_p
    lib.leg2cheb_batch_plan.argtypes = [ctypes.POINTER(vp), i64, ctypes.POINTER(i64), ctypes.POINTER(ci), ci,
                                        ctypes.POINTER(Tuning), vp]
    lib.leg2cheb_batch_tuning.argtypes = [ci, ctypes.POINTER(TuningBucket), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)]
    lib.leg2cheb_batch_execute.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.leg2cheb_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.leg2cheb_batch_destroy.argtypes = [vp]
    lib.leg2cheb_debug_alloc_hook.argtypes = [i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.leg2cheb_dct_plan.argtypes = [ctypes.POINTER(vp), i64, ci, i64, vp]
    lib.leg2cheb_dct_execute.argtypes = [vp, vp, vp, i64, vp]
    lib.leg2cheb_dct_destroy.argtypes = [vp]
    lib.leg2cheb_grid_plan.argtypes = [ctypes.POINTER(vp), i64, ci, ci, ci, i64, vp]
    lib.leg2cheb_grid_execute.argtypes = [vp, vp, vp, i64, vp]
    lib.leg2cheb_grid_destroy.argtypes = [vp]
    lib.leg2cheb_grid_fmm.argtypes = [vp]
    lib.leg2cheb_grid_dct.argtypes = [vp]
    for name in EXPORTED:
        if name not in ("leg2cheb_strerror", "leg2cheb_grid_fmm", "leg2cheb_grid_dct"):
            getattr(lib, name).restype = ci
    lib.leg2cheb_grid_fmm.restype = vp
    lib.leg2cheb_grid_dct.restype = vp
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().leg2cheb_strerror(int(code)).decode()


def _check(rc: int, what: str) -> None:
    if rc != L2C_OK:
        raise L2CError(rc, what)


# ----------------------------------------------------------------- ABI-named wrappers
def leg2cheb_plan(n: int, direction: int, leaf_size: int, rank: int) -> int:
    h = ctypes.c_void_p()
    _check(load().leg2cheb_plan(ctypes.byref(h), int(n), int(direction), int(leaf_size), int(rank)), "leg2cheb_plan")
    return h.value


def leg2cheb_plan_ex(n: int, direction: int, leaf_size: int, rank: int, precision: int = L2C_FP64,
                     max_batch: int = 1, stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load().leg2cheb_plan_ex(ctypes.byref(h), int(n), int(direction), int(leaf_size), int(rank),
                                   int(precision), int(max_batch), ctypes.c_void_p(stream or None)),
           "leg2cheb_plan_ex")
    return h.value


def leg2cheb_plan_basis(n: int, direction: int, leaf_size: int, rank: int, precision: int = L2C_FP64,
                        max_batch: int = 1, basis: int = L2C_MODAL, stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load().leg2cheb_plan_basis(ctypes.byref(h), int(n), int(direction), int(leaf_size), int(rank),
                                      int(precision), int(max_batch), int(basis), ctypes.c_void_p(stream or None)),
           "leg2cheb_plan_basis")
    return h.value


def leg2cheb_plan_tables(n: int, direction: int, leaf_size: int, rank: int, max_batch: int = 1,
                         tables: int = L2C_TABLES_STORED, stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load().leg2cheb_plan_tables(ctypes.byref(h), int(n), int(direction), int(leaf_size), int(rank),
                                       int(max_batch), int(tables), ctypes.c_void_p(stream or None)),
           "leg2cheb_plan_tables")
    return h.value


def leg2cheb_plan_cached(n: int, direction: int, leaf_size: int, rank: int, precision: int = L2C_FP64,
                         max_batch: int = 1, basis: int = L2C_MODAL, stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load().leg2cheb_plan_cached(ctypes.byref(h), int(n), int(direction), int(leaf_size), int(rank),
                                       int(precision), int(max_batch), int(basis), ctypes.c_void_p(stream or None)),
           "leg2cheb_plan_cached")
    return h.value


def leg2cheb_plan_cache_size():
    plans, refs = ctypes.c_int64(), ctypes.c_int64()
    _check(load().leg2cheb_plan_cache_size(ctypes.byref(plans), ctypes.byref(refs)), "leg2cheb_plan_cache_size")
    return plans.value, refs.value


def leg2cheb_execute(plan: int, in_ptr: int, out_ptr: int, batch: int, stream: int = 0) -> None:
    _check(load().leg2cheb_execute(ctypes.c_void_p(plan), ctypes.c_void_p(in_ptr or None),
                                   ctypes.c_void_p(out_ptr or None), int(batch), ctypes.c_void_p(stream or None)),
           "leg2cheb_execute")


def leg2cheb_execute_noalloc(plan: int, in_ptr: int, out_ptr: int, batch: int, stream: int = 0) -> None:
    _check(load().leg2cheb_execute_noalloc(ctypes.c_void_p(plan), ctypes.c_void_p(in_ptr or None),
                                           ctypes.c_void_p(out_ptr or None), int(batch),
                                           ctypes.c_void_p(stream or None)), "leg2cheb_execute_noalloc")


def leg2cheb_destroy(plan: int) -> None:
    _check(load().leg2cheb_destroy(ctypes.c_void_p(plan)), "leg2cheb_destroy")


def leg2cheb_plan_info(plan: int) -> dict:
    info = PlanInfo()
    _check(load().leg2cheb_plan_info(ctypes.c_void_p(plan), ctypes.byref(info)), "leg2cheb_plan_info")
    return info.as_dict()


def leg2cheb_plan_export(plan: int, table: int, dst_ptr: int = 0, nbytes: int = 0) -> int:
    """Copy a plan table to host memory at dst_ptr; with dst_ptr = 0 return its size."""
    need = ctypes.c_int64(0)
    _check(load().leg2cheb_plan_export(ctypes.c_void_p(plan), int(table), ctypes.c_void_p(dst_ptr or None),
                                       int(nbytes), ctypes.byref(need)), "leg2cheb_plan_export")
    return need.value


def leg2cheb_plan_set_option(plan: int, option: int, value: int) -> None:
    _check(load().leg2cheb_plan_set_option(ctypes.c_void_p(plan), int(option), int(value)),
           "leg2cheb_plan_set_option")


def leg2cheb_plan_status(plan: int) -> int:
    st = ctypes.c_int(0)
    _check(load().leg2cheb_plan_status(ctypes.c_void_p(plan), ctypes.byref(st)), "leg2cheb_plan_status")
    return st.value


def leg2cheb_set_timing_events(plan: int, before: int, after: int) -> None:
    _check(load().leg2cheb_set_timing_events(ctypes.c_void_p(plan), ctypes.c_void_p(before or None),
                                             ctypes.c_void_p(after or None)), "leg2cheb_set_timing_events")


def leg2cheb_rank_supported(rank: int) -> bool:
    return bool(load().leg2cheb_rank_supported(int(rank)))


def leg2cheb_debug_alloc_hook(fail_at: int = -1):
    """Arm (fail_at >= 1), disarm (0) or only query (-1) the allocation-failure hook.
    Returns (countdown before the call, allocations the library holds)."""
    pend, live = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load().leg2cheb_debug_alloc_hook(int(fail_at), ctypes.byref(pend), ctypes.byref(live)),
           "leg2cheb_debug_alloc_hook")
    return pend.value, live.value


def _tuning(tuning):
    """(n_max, leaf_size, rank) triples -> a Tuning struct (kept alive by the caller)."""
    rows = [(int(a), int(b), int(c)) for a, b, c in tuning]
    arr = (TuningBucket * max(len(rows), 1))(*[TuningBucket(*r) for r in rows])
    return Tuning(len(rows), arr), arr


def leg2cheb_batch_plan(n, direction, precision: int = L2C_FP64, tuning=None, stream: int = 0) -> int:
    """tuning: None (the library's table) or a list of (n_max, leaf_size, rank) size buckets."""
    count = len(n)
    na = (ctypes.c_int64 * count)(*[int(v) for v in n])
    da = (ctypes.c_int * count)(*[int(v) for v in direction])
    h = ctypes.c_void_p()
    tp = None
    if tuning is not None:
        t, keep = _tuning(tuning)
        tp = ctypes.byref(t)
    _check(load().leg2cheb_batch_plan(ctypes.byref(h), count, na, da, int(precision), tp,
                                      ctypes.c_void_p(stream or None)), "leg2cheb_batch_plan")
    return h.value


def leg2cheb_batch_tuning(precision: int = L2C_FP64):
    """The library's size buckets for the precision, as (n_max, leaf_size, rank) triples."""
    cnt = ctypes.c_int32(0)
    _check(load().leg2cheb_batch_tuning(int(precision), None, 0, ctypes.byref(cnt)), "leg2cheb_batch_tuning")
    arr = (TuningBucket * max(cnt.value, 1))()
    _check(load().leg2cheb_batch_tuning(int(precision), arr, cnt.value, ctypes.byref(cnt)), "leg2cheb_batch_tuning")
    return [(arr[k].n_max, arr[k].leaf_size, arr[k].rank) for k in range(cnt.value)]


def leg2cheb_batch_execute(batch: int, in_ptrs, out_ptrs, stream: int = 0) -> None:
    count = len(in_ptrs)
    ia = (ctypes.c_void_p * count)(*[int(p) for p in in_ptrs])
    oa = (ctypes.c_void_p * count)(*[int(p) for p in out_ptrs])
    _check(load().leg2cheb_batch_execute(ctypes.c_void_p(batch), ia, oa, ctypes.c_void_p(stream or None)),
           "leg2cheb_batch_execute")


def leg2cheb_batch_info(batch: int) -> dict:
    g, t = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load().leg2cheb_batch_info(ctypes.c_void_p(batch), ctypes.byref(g), ctypes.byref(t)),
           "leg2cheb_batch_info")
    return {"groups": g.value, "table_bytes": t.value}


def leg2cheb_batch_destroy(batch: int) -> None:
    _check(load().leg2cheb_batch_destroy(ctypes.c_void_p(batch)), "leg2cheb_batch_destroy")


def leg2cheb_dct_plan(n: int, kind: int, max_batch: int = 1, stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load().leg2cheb_dct_plan(ctypes.byref(h), int(n), int(kind), int(max_batch), ctypes.c_void_p(stream or None)),
           "leg2cheb_dct_plan")
    return h.value


def leg2cheb_dct_execute(dct: int, in_ptr: int, out_ptr: int, batch: int, stream: int = 0) -> None:
    _check(load().leg2cheb_dct_execute(ctypes.c_void_p(dct), ctypes.c_void_p(in_ptr or None),
                                       ctypes.c_void_p(out_ptr or None), int(batch), ctypes.c_void_p(stream or None)),
           "leg2cheb_dct_execute")


def leg2cheb_dct_destroy(dct: int) -> None:
    _check(load().leg2cheb_dct_destroy(ctypes.c_void_p(dct)), "leg2cheb_dct_destroy")


def leg2cheb_grid_plan(n: int, direction: int, leaf_size: int = 64, rank: int = 18, max_batch: int = 1,
                       stream: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load().leg2cheb_grid_plan(ctypes.byref(h), int(n), int(direction), int(leaf_size), int(rank),
                                     int(max_batch), ctypes.c_void_p(stream or None)), "leg2cheb_grid_plan")
    return h.value


def leg2cheb_grid_execute(grid: int, in_ptr: int, out_ptr: int, batch: int, stream: int = 0) -> None:
    _check(load().leg2cheb_grid_execute(ctypes.c_void_p(grid), ctypes.c_void_p(in_ptr or None),
                                        ctypes.c_void_p(out_ptr or None), int(batch), ctypes.c_void_p(stream or None)),
           "leg2cheb_grid_execute")


def leg2cheb_grid_destroy(grid: int) -> None:
    _check(load().leg2cheb_grid_destroy(ctypes.c_void_p(grid)), "leg2cheb_grid_destroy")


def leg2cheb_grid_fmm(grid: int) -> int:
    return load().leg2cheb_grid_fmm(ctypes.c_void_p(grid)) or 0


def leg2cheb_grid_dct(grid: int) -> int:
    return load().leg2cheb_grid_dct(ctypes.c_void_p(grid)) or 0
