"""ctypes side of cpu_fmm.cpp: the single-threaded CPU implementation of Alg. 4.

TEST AND BENCHMARK INFRASTRUCTURE ONLY (see the package docstring): the CPU baseline
that the benchmark times beside the GPU path, pinned against the direct oracle in
tests/test_cpu_fmm.py.  It shares no code with the oracle or the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpu_fmm.cpp")
_LIB = os.path.join(_HERE, "libcpufmm.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile cpu_fmm.cpp into libcpufmm.so next to it: g++ -O3 for x86-64-v3 (AVX2 and
    FMA, which every host of this GPU has; the library may be built on another host than
    the one it runs on), no fast-math; the sums marked omp simd may be vectorized in any
    order."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-march=x86-64-v3", "-fopenmp-simd", "-std=c++17", "-fPIC", "-shared", _SRC,
                               "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.cpu_fmm_plan.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.cpu_fmm_plan.restype = ctypes.c_void_p
        lib.cpu_fmm_execute.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.cpu_fmm_execute.restype = ctypes.c_int
        lib.cpu_fmm_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
        lib.cpu_fmm_info.restype = ctypes.c_int
        lib.cpu_fmm_destroy.argtypes = [ctypes.c_void_p]
        lib.cpu_fmm_destroy.restype = None
        _lib = lib
    return _lib


class CpuFmm:
    """One planned transform of length n (direction 0 leg2cheb, 1 cheb2leg)."""

    def __init__(self, n: int, direction: int = 0, leaf: int = 64, rank: int = 18):
        lib = _load()
        t0 = time.perf_counter()
        self.h = lib.cpu_fmm_plan(int(n), int(direction), int(leaf), int(rank))
        self.plan_s = time.perf_counter() - t0
        if not self.h:
            raise ValueError("cpu_fmm_plan rejected (n=%d, direction=%d, leaf=%d, rank=%d)"
                             % (n, direction, leaf, rank))
        self.n = int(n)
        info = (ctypes.c_int64 * 3)()
        lib.cpu_fmm_info(self.h, info)
        self.L, self.s, self.N = int(info[0]), int(info[1]), int(info[2])

    def execute(self, f, out=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (self.n,):
            raise ValueError("f must have shape (%d,)" % self.n)
        if out is None:
            out = np.empty(self.n, dtype=np.float64)
        if _load().cpu_fmm_execute(self.h, f.ctypes.data, out.ctypes.data) != 0:
            raise RuntimeError("cpu_fmm_execute failed")
        return out

    def fastest_seconds(self, f, reps: int) -> float:
        """The fastest of reps executes (the timing protocol of Sec. 5.2)."""
        out = np.empty(self.n, dtype=np.float64)
        best = float("inf")
        for _ in range(max(1, reps)):
            t0 = time.perf_counter()
            self.execute(f, out)
            best = min(best, time.perf_counter() - t0)
        return best

    def close(self):
        if getattr(self, "h", None):
            _load().cpu_fmm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def transform(f, direction: int, leaf: int = 64, rank: int = 18) -> np.ndarray:
    with CpuFmm(len(f), direction, leaf, rank) as p:
        return p.execute(f)
