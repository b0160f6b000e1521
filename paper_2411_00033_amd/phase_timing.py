"""Phase timeline of the single-launch kernel (k_fused) from an instrumented build.

Builds a variant of the library with L2C_PHASE_TIMING (every L2C_TS point of the kernels
records the wall clock), runs cold leg2cheb executes of the N = 10^6 workload through it,
and prints, per phase, the median and maximum over the workgroups ("units") of the time
since the earliest unit start, in microseconds.  The product library is not touched: the
variant is written to paper_2411_00033_amd/_build/.

    python -m paper_2411_00033_amd.phase_timing [--n 1000000] [--reps 10]

Phases of k_fused (kernel 3), in the order the kernel passes them:
"""
from __future__ import annotations

import argparse
import ctypes
import os

import numpy as np

from . import build as hipbuild

PHASES = [
    (0, "start"),
    (1, "input, T, B, P staged (workers' first barrier)"),
    (17, "streamer: first group's loads issued"),
    (16, "workers: step (1) products done (before their barrier)"),
    (2, "step (1) done (finest w)"),
    (12, "step (2) inside the unit done"),
    (3, "unit root and boundary nodes published"),
    (18, "near waves: Q table done"),
    (4, "near field (step (6)) done"),
    (11, "top wave: next unit's nodes and the roots below its ancestors polled"),
    (13, "top wave: its ancestors (step (2) above the units) published"),
    (14, "top wave: tree-top items polled"),
    (9, "top wave: tree-top items in LDS"),
    (15, "streamer: first group multiplied"),
    (8, "streamer: own far-field blocks done (step (3))"),
    (20, "workers: near field and tree-top items both done (worker barrier)"),
    (21, "workers: tree-top reduction rounds done"),
    (22, "workers: ancestor far-field blocks done (worker barrier)"),
    (10, "top wave: tree-top reduction, ancestor blocks, chain to the unit root"),
    (5, "all waves joined"),
    (6, "step (4) inside the unit done"),
    (7, "steps (5), (7) and output done (end)"),
]
__doc__ += "\n".join("  %2d  %s" % p for p in PHASES) + "\n"

KERNELS, UNITS, SLOTS = 4, 4096, 24


def build_variant() -> str:
    os.makedirs(hipbuild.OBJ, exist_ok=True)
    out = os.path.join(hipbuild.OBJ, "libleg2cheb_phase.so")
    cmd = [hipbuild.HIPCC, *hipbuild.FLAGS, "-shared", "-DL2C_PHASE_TIMING", "-I",
           os.path.join(hipbuild.ROOT, "include"), *hipbuild.sources(), "-o", out]
    rc, txt = hipbuild._run(cmd, False)
    if rc != 0:
        raise RuntimeError("hipcc failed:\n" + txt)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=10 ** 6)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--direction", type=int, default=0)
    ap.add_argument("--lib", default="", help="use this instrumented library instead of building one")
    ap.add_argument("--dump", default="", help="also save every unit's times (us, reps x units x phases) to this .npy file")
    args = ap.parse_args()
    path = args.lib or build_variant()
    from . import _lib
    _lib.LIB_PATH = path
    import torch
    from . import Plan, inputs
    lib = _lib.load()
    lib.l2c_debug_phase_ts.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
    lib.l2c_debug_phase_ts.restype = ctypes.c_int
    count = KERNELS * UNITS * SLOTS
    buf = np.zeros(count, dtype=np.uint64)
    hip = ctypes.CDLL("libamdhip64.so")
    khz = ctypes.c_int(0)
    hip.hipDeviceGetAttribute(ctypes.byref(khz), 10017, 0)   # hipDeviceAttributeWallClockRate (ROCm 7 enum)
    if khz.value <= 0:
        raise RuntimeError("hipDeviceGetAttribute(WallClockRate) failed")
    tick_us = 1e3 / khz.value
    x = torch.from_numpy(inputs.decaying(args.n, 0.5, inputs.SEED_BASE + 2)).cuda()
    y = torch.empty_like(x)
    flush = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    sink = torch.empty((), dtype=torch.float64, device="cuda")
    rows = []
    with Plan(args.n, args.direction) as p:
        for rep in range(args.reps + 2):
            torch.sum(flush, dim=0, out=sink)
            torch.cuda.synchronize()
            assert lib.l2c_debug_phase_ts(None, count, 1) == 0
            p.execute(x, y)
            torch.cuda.synchronize()
            assert lib.l2c_debug_phase_ts(buf.ctypes.data, count, 0) == 0
            if rep >= 2:
                t = buf.reshape(KERNELS, UNITS, SLOTS)[3].astype(np.float64)
                used = np.flatnonzero(t[:, 0] > 0)
                rows.append(t[used])
        assert p.status == 0
    t = np.stack(rows)                       # reps x units x slots
    t0 = np.min(np.where(t[:, :, 0:1] > 0, t[:, :, 0:1], np.inf), axis=1, keepdims=True)
    rel = (t - t0) * tick_us
    if args.dump:
        np.save(args.dump, np.where(t > 0, rel, np.nan))
    print("k_fused phase timeline, n = %d, direction %d, %d units, %d cold executes (wall clock %d kHz)"
          % (args.n, args.direction, t.shape[1], args.reps, khz.value))
    print("| phase | what | median over units (us) | max over units (us) |")
    print("|---|---|---|---|")
    for ph, what in PHASES:
        v = rel[:, :, ph]
        ok = t[:, :, ph] > 0
        if not ok.any():
            continue
        med = np.median([np.median(v[r][ok[r]]) for r in range(v.shape[0]) if ok[r].any()])
        mx = np.median([np.max(v[r][ok[r]]) for r in range(v.shape[0]) if ok[r].any()])
        print("| %d | %s | %.1f | %.1f |" % (ph, what, med, mx))


if __name__ == "__main__":
    main()
