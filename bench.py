"""Throughput benchmark of the MI355X Legendre <-> Chebyshev transform.

Workload: one leg2cheb transform of N = 10^6 FP64 coefficients (leaf 64, rank 18),
inputs f_j = z_j / sqrt(j+1), z_j iid N(0,1) from a fixed seed, resident in HBM.
A step is one execute of the whole path (all kernels of Alg. 4) over that vector.

Timing protocol
  * W warm-up steps, then exactly K timed steps between device synchronizations.
  * Cold: before every timed step a 1 GiB read evicts the 256 MiB Infinity Cache,
    so the plan tables and the vectors come from HBM; the step itself is timed with
    HIP events on the execute stream (ms_per_step).  The wall time of the K cold steps
    (flushes included) is reported too.
  * Kernel: K more cold steps in which the library brackets the dominant kernel with
    HIP events of its own on the execute stream (k_fused on the single-launch path:
    the whole of Alg. 4; k_main on the three-kernel path); its mean duration gives
    roofline.achieved.  A separate loop, so that those events add nothing to the step.
  * Warm: K further steps back to back, no flush (warm_ms_per_step).
The CPU baseline times the direct oracle on a bounded sample of rows of the same
transform and extrapolates by term count to the full transform, and times the
single-threaded CPU FMM of Alg. 4 on the whole transform (fastest of 2^(26 - log2 N)
executes, the protocol of Sec. 5.2).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcoeff/s for leg→cheb N=10^6 (FP64 vs batched mixed-prec) at stated rel. error"
HBM_PEAK_GBS = 8000.0
N = 10 ** 6
LEAF, RANK = 64, 18
PMC_FILES = {"k_fused": os.path.join(ROOT, "profiles", "k_fused_pmc_leg2cheb_n1e6.txt"),
             "k_main": os.path.join(ROOT, "profiles", "k_main_pmc_leg2cheb_n1e6.txt")}
CSRC = os.path.join(ROOT, "paper_2411_00033_amd", "csrc")


# Sources each timed kernel is compiled from: a PMC summary holds only while these are unchanged.
KERNEL_SOURCES = {"k_fused": ("l2c_fused.hip", "l2c_device.h", "l2c_internal.h", "l2c_math.h"),
                  "k_main": ("l2c_exec.hip", "l2c_device.h", "l2c_internal.h", "l2c_math.h")}


def source_sha256(kernel="k_fused"):
    """Digest of the HIP sources the kernel is built from."""
    h = hashlib.sha256()
    for name in sorted(KERNEL_SOURCES[kernel]):
        h.update(name.encode())
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


class HipEvents:
    """Raw hipEvent_t handles (the library records them on the execute stream)."""

    def __init__(self, count):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.ev = []
        for _ in range(count):
            h = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev.append(h.value)

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(self.ev[a]), ctypes.c_void_p(self.ev[b])) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def close(self):
        for h in self.ev:
            self.hip.hipEventDestroy(ctypes.c_void_p(h))


def pmc_traffic(kernel):
    """HBM bytes per launch of kernel from the committed rocprofv3 PMC summary (calibrated
    FETCH_SIZE + WRITE_SIZE), or None when the summary is missing or was taken on other sources."""
    try:
        rec = {}
        for ln in open(PMC_FILES[kernel]):
            if ":" in ln and not ln.startswith((" ", "#", "|")):
                k, v = ln.split(":", 1)
                rec[k.strip()] = v.strip()
        if rec.get("source_sha256") != source_sha256(kernel):
            return None
        return float(rec["hbm_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline(f, z_gpu, direction):
    """Direct oracle on every 3rd row of the transform; throughput scaled to the full transform."""
    import oracle
    n = f.size
    rows = np.arange(0, n, 3, dtype=np.int64)
    t0 = time.perf_counter()
    ref = oracle.transform(f, direction, rows)
    dt = time.perf_counter() - t0
    terms_sample = float(np.sum((n - rows + 1) // 2))
    terms_full = float(np.sum((n - np.arange(n) + 1) // 2))
    est_full = dt * terms_full / terms_sample
    err = float(np.max(np.abs(z_gpu[rows] - ref)) / np.max(np.abs(ref)))
    base = {"value": n / est_full / 1e9, "unit": "Gcoeff/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "rows i = 0 mod 3 of the N=10^6 %s (%d rows, %.3g of %.3g terms, %.1f s), "
                      "extrapolated by term count" % (("leg2cheb", "cheb2leg")[direction], rows.size, terms_sample,
                                                      terms_full, dt)}
    # the single-threaded CPU FMM of Alg. 4 (FP64, leaf 64, rank 18), fastest of
    # 2^(26 - log2 N) executes as in Sec. 5.2
    from oracle import cpu_fmm
    reps = 2 ** max(0, 26 - int(round(np.log2(n))))
    with cpu_fmm.CpuFmm(n, direction, LEAF, RANK) as p:
        t = p.fastest_seconds(f, reps)
        zc = p.execute(f)
        plan_s = p.plan_s
    base["fmm"] = {"value": n / t / 1e9, "unit": "Gcoeff/s", "cores": 1, "kind": "cpu_fmm",
                   "ms_per_transform": t * 1e3, "plan_s": plan_s,
                   "einf_vs_gpu": float(np.max(np.abs(zc - z_gpu)) / np.max(np.abs(z_gpu))),
                   "sample": "the whole N=10^6 %s, fastest of %d executes on one host core (single-threaded "
                             "C++ Alg. 4, oracle/cpu_fmm.cpp)" % (("leg2cheb", "cheb2leg")[direction], reps)}
    return base, err


BATCH_N, BATCH_B = 65536, 256
FP32_PEAK_TFLOPS = 157.3


def batched_form(l2c, inputs, torch, K, W, flush, flush_sink, with_fp64=True):
    """The batched FP32 form on 256 leg2cheb transforms of N = 65536 (f = z/(j+1)), cold:
    whole-execute time by torch events, the kb_main kernel by the library's events, and the
    FP64 path on the same batch for comparison."""
    stream = torch.cuda.current_stream()
    F = inputs.decaying(BATCH_N, 1.0, inputs.SEED_BASE + 3, batch=BATCH_B)
    x = torch.from_numpy(F).cuda()
    y32 = torch.empty_like(x)
    p32 = l2c.Plan(BATCH_N, l2c.LEG2CHEB, 64, 16, precision=l2c.L2C_FP32, max_batch=BATCH_B)

    def timed(p, y):
        st = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        en = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        for _ in range(W):
            p.execute(x, y)
        torch.cuda.synchronize()
        for i in range(K):
            torch.sum(flush, dim=0, out=flush_sink)
            st[i].record(stream)
            p.execute(x, y)
            en[i].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([st[i].elapsed_time(en[i]) for i in range(K)]))

    ms32 = timed(p32, y32)
    ev = HipEvents(2 * K)
    for i in range(K):
        torch.sum(flush, dim=0, out=flush_sink)
        l2c.leg2cheb_set_timing_events(p32.handle, ev.ev[2 * i], ev.ev[2 * i + 1])
        p32.execute(x, y32)
    torch.cuda.synchronize()
    l2c.leg2cheb_set_timing_events(p32.handle, 0, 0)
    kmain = float(np.mean([ev.elapsed_ms(2 * i, 2 * i + 1) for i in range(K)]))
    ev.close()
    info = p32.info
    coeffs = float(BATCH_B * BATCH_N)
    s, M = info["s"], 16
    flops = (4.5 * s + 4 * M + 8.0 * M * M / s) * info["n_pad"] * BATCH_B   # Eq. (totalnumflopsnew)
    rec = {"workload": "leg2cheb, 256 transforms of N=65536, f_j = z_j/(j+1), rank 16, leaf 64 (s=32, L=9); "
                       "FP32 tables and products, FP64 input and output; cold HBM",
           "ms_per_execute": ms32, "Gcoeff_s": coeffs / (ms32 * 1e-3) / 1e9,
           "kb_main_ms": kmain,
           "alg_flops": flops, "TFLOPs_achieved": flops / (ms32 * 1e-3) / 1e12,
           "mfma_fp32_frac": flops / (ms32 * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
           "io_bytes": 16.0 * coeffs, "io_GBs": 16.0 * coeffs / (ms32 * 1e-3) / 1e9}
    yb = torch.empty_like(x)
    pb = l2c.Plan(BATCH_N, l2c.LEG2CHEB, 64, 16, precision=l2c.L2C_BF16X2, max_batch=BATCH_B)
    msb = timed(pb, yb)
    pb.close()
    rec.update({"bf16x2_ms_per_execute": msb, "bf16x2_Gcoeff_s": coeffs / (msb * 1e-3) / 1e9})
    yh = torch.empty_like(x)
    ph = l2c.Plan(BATCH_N, l2c.LEG2CHEB, 64, 16, precision=l2c.L2C_FP16X2, max_batch=BATCH_B)
    msh = timed(ph, yh)
    ph.close()
    rec.update({"fp16x2_ms_per_execute": msh, "fp16x2_Gcoeff_s": coeffs / (msh * 1e-3) / 1e9})
    if with_fp64:
        y64 = torch.empty_like(x)
        p64 = l2c.Plan(BATCH_N, l2c.LEG2CHEB, 64, 18, max_batch=BATCH_B)
        ms64 = timed(p64, y64)
        d = (y32 - y64).abs().max().item() / y64.abs().max().item()
        db = (yb - y64).abs().max().item() / y64.abs().max().item()
        dh = (yh - y64).abs().max().item() / y64.abs().max().item()
        rec.update({"fp64_path_ms_per_execute": ms64, "fp64_path_Gcoeff_s": coeffs / (ms64 * 1e-3) / 1e9,
                    "einf_fp32_vs_fp64_path": d, "einf_bf16x2_vs_fp64_path": db, "einf_fp16x2_vs_fp64_path": dh})
        p64.close()
        # the FP64 tile form (rank 16, 16 transforms per FP64 matrix-core tile)
        yt = torch.empty_like(x)
        pt = l2c.Plan(BATCH_N, l2c.LEG2CHEB, 64, 16, max_batch=BATCH_B)
        mst = timed(pt, yt)
        ev = HipEvents(2 * K)
        for i in range(K):
            torch.sum(flush, dim=0, out=flush_sink)
            l2c.leg2cheb_set_timing_events(pt.handle, ev.ev[2 * i], ev.ev[2 * i + 1])
            pt.execute(x, yt)
        torch.cuda.synchronize()
        l2c.leg2cheb_set_timing_events(pt.handle, 0, 0)
        kmt = float(np.mean([ev.elapsed_ms(2 * i, 2 * i + 1) for i in range(K)]))
        ev.close()
        flops64 = (4.5 * s + 4 * 16 + 8.0 * 16 * 16 / s) * info["n_pad"] * BATCH_B
        dt = (yt - y64).abs().max().item() / y64.abs().max().item()
        rec["fp64_tile_form"] = {"ms_per_execute": mst, "Gcoeff_s": coeffs / (mst * 1e-3) / 1e9, "rank": 16,
                                 "path": pt.info["path"], "kb_main_ms": kmt,
                                 "TFLOPs_achieved": flops64 / (mst * 1e-3) / 1e12,
                                 "mfma_fp64_frac": flops64 / (mst * 1e-3) / 1e12 / 78.6,
                                 "einf_vs_fp64_path_rank18": dt}
        pt.close()
        # the nodal basis (Eq. (AijLag)) on the same kernels: FP32 form and FP64 tile form
        nod = {}
        for tag, prec in (("fp32", l2c.L2C_FP32), ("fp64_tile", l2c.L2C_FP64)):
            yn = torch.empty_like(x)
            pn = l2c.Plan(BATCH_N, l2c.LEG2CHEB, 64, 16, precision=prec, max_batch=BATCH_B, basis=l2c.L2C_NODAL)
            msn = timed(pn, yn)
            pn.close()
            nod[tag] = {"ms_per_execute": msn, "Gcoeff_s": coeffs / (msn * 1e-3) / 1e9,
                        "einf_vs_fp64_path_rank18": (yn - y64).abs().max().item() / y64.abs().max().item()}
        rec["nodal_basis"] = nod
    p32.close()
    return rec


def lines_form(l2c, inputs, torch, K, W, flush, flush_sink):
    """65536 lines of N = 1024 (a 256 x 256 x 1024 tensor along its last axis), f = z/(k+1):
    leg2cheb, cold, in the FP64 path and the FP32 form; round-trip error through cheb2leg."""
    stream = torch.cuda.current_stream()
    n, lines = 1024, 256 * 256
    x = torch.from_numpy(inputs.decaying(n, 1.0, inputs.SEED_BASE + 5, batch=lines)).cuda()
    z, g = torch.empty_like(x), torch.empty_like(x)
    rec = {"workload": "65536 lines of N=1024 (256 x 256 x 1024 FP64 tensor, last axis), f_k = z_k/(k+1); cold HBM"}
    for tag, prec, rank in (("fp64", l2c.L2C_FP64, 18), ("fp32", l2c.L2C_FP32, 16)):
        pf = l2c.Plan(n, l2c.LEG2CHEB, 64, rank, precision=prec, max_batch=lines)
        pb = l2c.Plan(n, l2c.CHEB2LEG, 64, rank, precision=prec, max_batch=lines)
        for _ in range(W):
            pf.execute(x, z)
        torch.cuda.synchronize()
        st = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        en = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        for i in range(K):
            torch.sum(flush, dim=0, out=flush_sink)
            st[i].record(stream)
            pf.execute(x, z)
            en[i].record(stream)
        pb.execute(z, g)
        torch.cuda.synchronize()
        ms = float(np.mean([st[i].elapsed_time(en[i]) for i in range(K)]))
        rt = ((g - x).abs().amax(dim=1) / x.abs().amax(dim=1)).max().item()
        rec[tag] = {"ms_per_execute": ms, "Gcoeff_s": n * lines / (ms * 1e-3) / 1e9, "round_trip_einf": rt,
                    "path": pf.info["path"]}
        pf.close()
        pb.close()
    return rec


def small_and_ragged(l2c, inputs, torch, K, W, flush, flush_sink, small=True):
    """The n = 1024 single transform (latency, cold) and the 2048-transform ragged batch
    (n log-uniform in [128, 262144], directions 50/50) through BatchPlan.execute_ptrs."""
    stream = torch.cuda.current_stream()

    def timed(fn, k, cold=True):
        st = [torch.cuda.Event(enable_timing=True) for _ in range(k)]
        en = [torch.cuda.Event(enable_timing=True) for _ in range(k)]
        for _ in range(W):
            fn()
        torch.cuda.synchronize()
        for i in range(k):
            if cold:
                torch.sum(flush, dim=0, out=flush_sink)
            st[i].record(stream)
            fn()
            en[i].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([st[i].elapsed_time(en[i]) for i in range(k)]))

    rec = {}
    if small:
        x1 = torch.from_numpy(inputs.decaying(1024, 1.0, inputs.SEED_BASE + 1)).cuda()
        y1 = torch.empty_like(x1)
        with l2c.Plan(1024, l2c.LEG2CHEB, 64, 18) as p1:
            one = {"us_per_execute_cold": timed(lambda: p1.execute(x1, y1), K) * 1e3,
                   "us_per_execute_warm": timed(lambda: p1.execute(x1, y1), K, cold=False) * 1e3,
                   "path": p1.info["path"]}
            p1.set_direct(False)   # the same transform by Alg. 4
            one["multipole"] = {"us_per_execute_cold": timed(lambda: p1.execute(x1, y1), K) * 1e3,
                                "us_per_execute_warm": timed(lambda: p1.execute(x1, y1), K, cold=False) * 1e3,
                                "path": p1.info["path"]}
            rec["n1024_single"] = one
    sizes, dirs = inputs.ragged_sizes(2048, inputs.SEED_BASE + 4)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    x = torch.randn(int(offs[-1]), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    ip = [x.data_ptr() + 8 * int(o) for o in offs[:-1]]
    op = [y.data_ptr() + 8 * int(o) for o in offs[:-1]]
    rg = {"workload": "2048 transforms, n log-uniform in [128, 262144] (%d coefficients), directions 50/50"
                      % int(offs[-1])}
    for tag, prec in (("fp64", l2c.L2C_FP64), ("fp32", l2c.L2C_FP32)):
        # leaf size and rank per size bucket from the library's autotuned table
        with l2c.BatchPlan(sizes.tolist(), dirs.tolist(), precision=prec) as bp:
            ms = timed(lambda: bp.execute_ptrs(ip, op), max(2, K // 4))
            rg[tag] = {"ms_per_execute": ms, "Gcoeff_s": float(offs[-1]) / (ms * 1e-3) / 1e9,
                       "groups": bp.info["groups"], "tuning": l2c.leg2cheb_batch_tuning(prec)}
    rec["ragged_2048"] = rg
    return rec


def grid_form(l2c, inputs, torch, K, W, flush, flush_sink):
    """The grid pipeline at N = 10^6 (Legendre series on the Chebyshev-Gauss grid and back,
    Sec. 1) and the DCTs alone (Sec. 5.2 times the FMM against a DCT of type 2), cold; the
    FMM's time is that of leg2cheb on the same input, so fmm_over_dct2 is the paper's ratio."""
    stream = torch.cuda.current_stream()

    def timed(fn):
        st = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        en = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        for _ in range(W):
            fn()
        torch.cuda.synchronize()
        for i in range(K):
            torch.sum(flush, dim=0, out=flush_sink)
            st[i].record(stream)
            fn()
            en[i].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([st[i].elapsed_time(en[i]) for i in range(K)]))

    n = N
    x = torch.from_numpy(inputs.decaying(n, 0.5, inputs.SEED_BASE + 2)).cuda()
    u = torch.empty_like(x)
    back = torch.empty_like(x)
    rec = {"workload": "N=1000000, f_j = z_j/sqrt(j+1); leg2grid = leg2cheb + DCT-3, grid2leg = DCT-2 + cheb2leg "
                       "(leaf 64, rank 18, FP64); DCTs on the library's FFT (100 x 100 x 100 four-step split); cold HBM"}
    with l2c.GridPlan(n, l2c.LEG2GRID) as fw, l2c.GridPlan(n, l2c.GRID2LEG) as bw, \
            l2c.Dct(n, 2) as d2, l2c.Dct(n, 3) as d3, l2c.Plan(n, l2c.LEG2CHEB, LEAF, RANK) as p:
        rec["leg2grid_ms"] = timed(lambda: fw.execute(x, u))
        rec["grid2leg_ms"] = timed(lambda: bw.execute(u, back))
        rec["dct2_ms"] = timed(lambda: d2.execute(x, back))
        rec["dct3_ms"] = timed(lambda: d3.execute(x, back))
        rec["fmm_leg2cheb_ms"] = timed(lambda: p.execute(x, back))
        bw.execute(fw.execute(x, u), back)
        torch.cuda.synchronize()
        rec["round_trip_einf"] = ((back - x).abs().max() / x.abs().max()).item()
    rec["fmm_over_dct2"] = rec["fmm_leg2cheb_ms"] / rec["dct2_ms"]
    rec["dct2_GBs_io"] = 16.0 * n / (rec["dct2_ms"] * 1e-3) / 1e9
    rec["leg2grid_Gcoeff_s"] = n / (rec["leg2grid_ms"] * 1e-3) / 1e9
    return rec


def regen_form(l2c, inputs, torch, K, W, flush, flush_sink):
    """N = 10^6 on plans that recompute the far-field blocks in every execute
    (L2C_TABLES_REGEN) against the stored-table plans: plan time, table bytes, cold execute
    time per direction, and the largest difference of the outputs relative to max|z|."""
    stream = torch.cuda.current_stream()

    def timed(fn):
        st = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        en = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        for _ in range(W):
            fn()
        torch.cuda.synchronize()
        for i in range(K):
            torch.sum(flush, dim=0, out=flush_sink)
            st[i].record(stream)
            fn()
            en[i].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([st[i].elapsed_time(en[i]) for i in range(K)]))

    n = N
    x = torch.from_numpy(inputs.decaying(n, 0.5, inputs.SEED_BASE + 2)).cuda()
    zr, zs = torch.empty_like(x), torch.empty_like(x)
    rec = {"workload": "N=1000000, f_j = z_j/sqrt(j+1), leaf 64, rank 18, FP64; far-field blocks below the "
                       "subtree roots recomputed from the kernel samples in every execute; cold HBM"}
    for direction, name in ((l2c.LEG2CHEB, "leg2cheb"), (l2c.CHEB2LEG, "cheb2leg")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pr = l2c.Plan(n, direction, LEAF, RANK, tables=l2c.L2C_TABLES_REGEN)
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t0) * 1e3
        with pr, l2c.Plan(n, direction, LEAF, RANK) as ps:
            ms = timed(lambda: pr.execute(x, zr))
            ms_stored = timed(lambda: ps.execute(x, zs))
            torch.cuda.synchronize()
            diff = ((zr - zs).abs().max() / zs.abs().max()).item()
            rec[name] = {"ms_per_execute": ms, "Gcoeff_s": n / (ms * 1e-3) / 1e9, "path": pr.info["path"],
                         "plan_ms": plan_ms, "table_bytes": pr.info["table_bytes"],
                         "stored_table_bytes": ps.info["table_bytes"], "stored_ms_per_execute": ms_stored,
                         "einf_vs_stored_tables": diff}
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (PMC byte-counter calibration)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched-form and line-batch measurements (profiling the N=10^6 kernel alone)")
    ap.add_argument("--workload", default="leg2cheb_1e6",
                    choices=["leg2cheb_1e6", "fp32_batch", "lines_3d", "ragged", "grid", "regen"],
                    help="fp32_batch: only the batched FP32 form (256 x 65536); lines_3d: only the "
                         "65536 lines of n = 1024 (FP64 dense path and FP32 form); grid: the grid pipeline and the "
                         "DCTs at N = 10^6; regen: N = 10^6 with the far-field blocks recomputed per execute; "
                         "e.g. under a profiler")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the transform is a single-GPU kernel path "
              "(multi-GPU sharding is designed but not built); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2411_00033_amd as l2c
    from paper_2411_00033_amd import inputs

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    f = inputs.decaying(N, 0.5, inputs.SEED_BASE + 2)
    x = torch.from_numpy(f).to(dev)
    out = torch.empty_like(x)
    flush = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)   # 1 GiB
    flush_sink = torch.empty((), dtype=torch.float64, device=dev)

    if args.calibrate_copy:
        src = torch.ones(1 << 25, dtype=torch.float64, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        torch.sum(flush, dim=0, out=flush_sink)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload == "fp32_batch":
        rec = batched_form(l2c, inputs, torch, args.steps, args.warmup, flush, flush_sink, with_fp64=False)
        print(json.dumps({"workload": "fp32_batch", "steps": args.steps, "warmup": args.warmup, **rec}), flush=True)
        return
    if args.workload == "ragged":
        rec = small_and_ragged(l2c, inputs, torch, args.steps, args.warmup, flush, flush_sink, small=False)
        print(json.dumps({"steps": args.steps, "warmup": args.warmup, **rec}), flush=True)
        return
    if args.workload == "lines_3d":
        rec = lines_form(l2c, inputs, torch, args.steps, args.warmup, flush, flush_sink)
        print(json.dumps({"steps": args.steps, "warmup": args.warmup, **rec}), flush=True)
        return
    if args.workload == "regen":
        rec = regen_form(l2c, inputs, torch, args.steps, args.warmup, flush, flush_sink)
        print(json.dumps({"steps": args.steps, "warmup": args.warmup, **rec}), flush=True)
        return
    if args.workload == "grid":
        rec = grid_form(l2c, inputs, torch, args.steps, args.warmup, flush, flush_sink)
        print(json.dumps({"steps": args.steps, "warmup": args.warmup, **rec}), flush=True)
        return

    plan = l2c.Plan(N, l2c.LEG2CHEB, LEAF, RANK)
    info = plan.info
    K, W = args.steps, args.warmup
    ev = HipEvents(2 * K)
    start = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    end = [torch.cuda.Event(enable_timing=True) for _ in range(K)]

    for _ in range(W):
        plan.execute(x, out)
    torch.cuda.synchronize()

    # cold timed region
    t0 = time.perf_counter()
    for i in range(K):
        torch.sum(flush, dim=0, out=flush_sink)
        start[i].record(stream)
        plan.execute(x, out)
        end[i].record(stream)
    torch.cuda.synchronize()
    wall_cold = (time.perf_counter() - t0) * 1e3 / K
    step_ms = [start[i].elapsed_time(end[i]) for i in range(K)]
    ms = float(np.mean(step_ms))

    # cold, the dominant kernel alone (library events)
    for i in range(K):
        torch.sum(flush, dim=0, out=flush_sink)
        l2c.leg2cheb_set_timing_events(plan.handle, ev.ev[2 * i], ev.ev[2 * i + 1])
        plan.execute(x, out)
    torch.cuda.synchronize()
    l2c.leg2cheb_set_timing_events(plan.handle, 0, 0)
    far = float(np.mean([ev.elapsed_ms(2 * i, 2 * i + 1) for i in range(K)]))

    # warm timed region
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        plan.execute(x, out)
    torch.cuda.synchronize()
    warm_ms = (time.perf_counter() - t0) * 1e3 / K

    # the other direction at the same size (cold, same protocol); its plan stage (Secs. 3.2,
    # 4.3: lambda, B, T, Ahat) is timed by wall clock including the device sync (the first
    # plan of the process also pays one-time initialisation)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan_c = l2c.Plan(N, l2c.CHEB2LEG, LEAF, RANK)
    plan_ms = (time.perf_counter() - t0) * 1e3
    out_c = torch.empty_like(x)
    for _ in range(W):
        plan_c.execute(x, out_c)
    cs = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ce = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    torch.cuda.synchronize()
    for i in range(K):
        torch.sum(flush, dim=0, out=flush_sink)
        cs[i].record(stream)
        plan_c.execute(x, out_c)
        ce[i].record(stream)
    torch.cuda.synchronize()
    c2l_ms = float(np.mean([cs[i].elapsed_time(ce[i]) for i in range(K)]))
    # round trip at the same size: cheb2leg of the leg2cheb output against the input
    back = torch.empty_like(x)
    plan_c.execute(out, back)
    torch.cuda.synchronize()
    round_trip = ((back - x).abs().max() / x.abs().max()).item()

    # every wait of the single-launch kernel completed in every execute above (a wait that
    # gave up would have made its output wrong)
    for p_, tag in ((plan, "leg2cheb"), (plan_c, "cheb2leg")):
        st_bits = p_.status
        if st_bits != 0:
            print("bench.py: the %s plan reports status bits %#x: a single-launch wait gave up, results invalid"
                  % (tag, st_bits), file=sys.stderr)
            sys.exit(3)
    z = out.cpu().numpy()
    ahat_alg = 8.0 * RANK * RANK * info["n_submatrices"]          # Ahat, one M x M table per submatrix
    main_alg = 16.0 * N + ahat_alg                                 # + FP64 input read and output write
    path_alg = main_alg                                            # compulsory bytes of the whole step
    achieved = main_alg / (far * 1e-3) / 1e9
    kname = "k_fused" if info["path"] == l2c.L2C_PATH_SINGLE else "k_main"
    traffic = pmc_traffic(kname)
    rec = {
        "metric": METRIC,
        "value": N / (ms * 1e-3) / 1e9,
        "unit": "Gcoeff/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "leg2cheb, one transform of N=1000000 FP64 coefficients, f_j = z_j/sqrt(j+1), "
                               "z_j ~ N(0,1) seeded; leaf 64 (s=31, L=13), rank 18; cold HBM",
                   "n": N, "direction": "leg2cheb", "leaf_size": LEAF, "rank": RANK, "batch": 1,
                   "levels": info["levels"], "s": info["s"], "n_pad": info["n_pad"], "precision": "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ("k_fused<18> (all of Alg. 4 in one launch)" if kname == "k_fused" else
                                "k_main<18> (far field + downward pass + leaf evaluation + near field)"),
                     "kernel_ms": far, "alg_bytes_per_launch": main_alg},
        "path_roofline": {"alg_bytes_per_step": path_alg, "achieved_GBs": path_alg / (ms * 1e-3) / 1e9,
                          "frac": path_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "warm_ms_per_step": warm_ms,
        "cold_wall_ms_per_step_incl_flush": wall_cold,
        "cheb2leg_ms_per_step": c2l_ms,
        "round_trip_einf": round_trip,
        "plan": {"table_bytes": info["table_bytes"], "ahat_bytes_padded": info["ahat_bytes"], "plan_ms": plan_ms},
    }
    if not args.no_extra:
        rec["batched_fp32_form"] = batched_form(l2c, inputs, torch, min(K, 20), min(W, 5), flush, flush_sink)
        rec["lines_3d"] = lines_form(l2c, inputs, torch, min(K, 10), min(W, 3), flush, flush_sink)
        rec.update(small_and_ragged(l2c, inputs, torch, min(K, 20), min(W, 3), flush, flush_sink))
        rec["grid_1e6"] = grid_form(l2c, inputs, torch, min(K, 20), min(W, 3), flush, flush_sink)
        rec["regen_tables_1e6"] = regen_form(l2c, inputs, torch, min(K, 20), min(W, 3), flush, flush_sink)
    if not args.no_cpu_baseline:
        base, err = cpu_baseline(f, z, 0)
        rec["cpu_baseline"] = base
        rec["einf_vs_oracle_sampled"] = err
    else:
        rec["cpu_baseline"] = None
    ev.close()
    plan.close()
    plan_c.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
