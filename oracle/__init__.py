"""CPU oracle for the Legendre <-> Chebyshev transforms of arXiv 2411.00033.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package.  The product library
never links, loads or calls it, and the two share no code.

Contents
--------
* ``oracle.c`` (loaded here through ctypes): the plain O(N^2) direct products
  z = C^{-1} A f (leg2cheb) and z = A^{-1} C f (cheb2leg) from the closed forms
  of Sec. 1, Eqs. (aij)/(hik)/(Lambda), and of the reverse kernel, Eq. (Lxymod);
  plus a back-substitution route for cheb2leg.  See the header of oracle.c.
* ``oracle.c`` also holds the grid pipeline of Sec. 1: the DCTs of kinds 2 and 3 as plain
  cosine sums, and the Legendre series evaluated on the Chebyshev-Gauss points through the
  three-term recurrence (``dct``, ``legval_cg``, ``grid2leg``).
* ``fmm_ref``: the plan tables and the seven steps of Alg. 4 written out in
  numpy in the paper's order and notation (an approximation of the direct
  product; pinned against it in the tests).
* ``cpu_fmm`` (``cpu_fmm.cpp``): a single-threaded C++ implementation of Alg. 4, the
  CPU baseline that the benchmark times beside the GPU path; not an oracle, pinned
  against the direct oracle in ``tests/test_cpu_fmm.py``.

Every function here is pinned in ``tests/test_oracle_*.py`` against exact
rational arithmetic, library routines and invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, OpenMP, libquadmath, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lquadmath", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_lambda.argtypes = [i64, dp]
        for name in ("oracle_leg2cheb", "oracle_cheb2leg"):
            getattr(lib, name).argtypes = [i64, dp, i64, i64p, dp]
        lib.oracle_cheb2leg_backsub.argtypes = [i64, dp, dp]
        lib.oracle_dct.argtypes = [i64, dp, ctypes.c_int, i64, i64p, dp]
        lib.oracle_legval_cg.argtypes = [i64, dp, i64, i64p, dp]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().oracle_num_threads())


def lambda_table(n: int) -> np.ndarray:
    """lambda_k = Gamma(k+1/2)/Gamma(k+1) for k < n (Eq. (Lambda), recursion (Lambdaint))."""
    out = np.empty(n, dtype=np.float64)
    rc = _load().oracle_lambda(n, _dptr(out))
    if rc != 0:
        raise ValueError("oracle_lambda failed (%d)" % rc)
    return out


def _rows_call(fn, f, rows):
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim != 1 or f.size < 1:
        raise ValueError("f must be a non-empty 1-D array")
    if rows is None:
        z = np.empty(f.size, dtype=np.float64)
        rc = fn(f.size, _dptr(f), 0, None, _dptr(z))
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        z = np.empty(r.size, dtype=np.float64)
        rc = fn(f.size, _dptr(f), r.size, r.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(z))
    if rc != 0:
        raise ValueError("oracle call failed (%d)" % rc)
    return z


def leg2cheb(f, rows=None) -> np.ndarray:
    """z = C^{-1} A f (all rows, or only ``rows``)."""
    return _rows_call(_load().oracle_leg2cheb, f, rows)


def cheb2leg(f, rows=None) -> np.ndarray:
    """z = A^{-1} C f through the reverse kernel of Eq. (Lxymod) (all rows, or ``rows``)."""
    return _rows_call(_load().oracle_cheb2leg, f, rows)


def cheb2leg_backsub(f) -> np.ndarray:
    """z = A^{-1} C f by back substitution on A z = C f (independent second route)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    z = np.empty(f.size, dtype=np.float64)
    rc = _load().oracle_cheb2leg_backsub(f.size, _dptr(f), _dptr(z))
    if rc != 0:
        raise ValueError("oracle_cheb2leg_backsub failed (%d)" % rc)
    return z


def transform(f, direction: int, rows=None) -> np.ndarray:
    """direction 0 = leg2cheb, 1 = cheb2leg."""
    return leg2cheb(f, rows) if direction == 0 else cheb2leg(f, rows)


def einf(z, zref) -> float:
    """Relative max-norm error of Eq. (Einf): ||z - z*||_inf / ||z*||_inf."""
    z = np.asarray(z, dtype=np.float64)
    zref = np.asarray(zref, dtype=np.float64)
    den = np.max(np.abs(zref))
    return float(np.max(np.abs(z - zref)) / den) if den > 0 else float(np.max(np.abs(z)))


def _rows_fn(fn, f, rows, *extra):
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim != 1 or f.size < 1:
        raise ValueError("input must be a non-empty 1-D array")
    if rows is None:
        z = np.empty(f.size, dtype=np.float64)
        rc = fn(f.size, _dptr(f), *extra, 0, None, _dptr(z))
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        z = np.empty(r.size, dtype=np.float64)
        rc = fn(f.size, _dptr(f), *extra, r.size, r.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(z))
    if rc != 0:
        raise ValueError("oracle call failed (%d)" % rc)
    return z


def dct(x, kind: int, rows=None) -> np.ndarray:
    """kind 2: y_k = sum_j x_j cos(pi k (2j+1)/(2n)); kind 3: y_j = sum_k x_k cos(pi k (2j+1)/(2n))."""
    return _rows_fn(_load().oracle_dct, x, rows, int(kind))


def legval_cg(f, rows=None) -> np.ndarray:
    """u_j = sum_k f_k P_k(x_j) on the Chebyshev-Gauss points x_j = cos(pi (2j+1)/(2n))."""
    return _rows_fn(_load().oracle_legval_cg, f, rows)


def grid2leg(u) -> np.ndarray:
    """Legendre coefficients of the degree < n interpolant of the values u_j at the
    Chebyshev-Gauss points: Chebyshev coefficients c_k = (2 - delta_k0)/n sum_j u_j
    cos(pi k (2j+1)/(2n)) (Gauss-Chebyshev quadrature), then cheb2leg (Sec. 1)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    c = dct(u, 2) * (2.0 / u.size)
    c[0] *= 0.5
    return cheb2leg(c)


def leg2grid(f, rows=None) -> np.ndarray:
    """Alias of legval_cg: the forward grid transform."""
    return legval_cg(f, rows)
