"""Plain numpy reference of the modal multipole method (arXiv 2411.00033, Secs. 3-4).

TEST INFRASTRUCTURE ONLY (see the package docstring).  It follows the paper's
order and notation, with no blocking, fusion or reordering:

* sizes:           Eqs. (Nb), (Ntot), (numlevels), (total_blocks_and_mats)
* indexing:        Eqs. (cfrompq), (globalij), (fgamma), (zgamma)
* Lambda(z):       Eq. (Lambda), evaluated with mpmath (arbitrary precision gamma)
* kernels:         A(x,y) of Sec. 3.2 and the reverse kernel L(x,y), Eq. (Lxymod)
* Ahat:            the 2-D Chebyshev-Gauss transform of Eq. (aklmore)
* T(sigma):        the Vandermonde matrix of Eqs. (matveczs), (Xs)
* B(l):            W^{-1} V(l) W of App. A3, in exact rational arithmetic
* execute:         steps (1)-(7) of Alg. 4, with step (6) as the direct product over
                   the entries that no far-field submatrix covers; stage_input and
                   upward are its steps (0) and (1)-(2), exposed for phase tests.

It is slow (Python loops over blocks, mpmath for every kernel sample) and meant
for n up to a few thousand.  Alg. 4 is an approximation of the direct product;
the tests pin this module against the direct oracle and against exact values.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import mpmath
import numpy as np

LEG2CHEB, CHEB2LEG = 0, 1


# ----------------------------------------------------------------------------- sizes
def sizes(n: int, leaf: int = 64, rank: int = 18) -> dict:
    """Levels and padded length for an input of length n (Eq. (numlevels)).

    ``leaf`` is the side 2*s_hat of the smallest submatrices, so s_hat = leaf/2.
    L = ceil(log2(n / s_hat)) - 2, s = ceil(n / 2^(L+2)), N = s 2^(L+2).
    L <= 0 means the whole product is done directly (Alg. 1).
    """
    shat = leaf // 2
    p = 0
    while (shat << p) < n:  # smallest p with 2^p * s_hat >= n, i.e. ceil(log2(n/s_hat))
        p += 1
    L = p - 2
    if L <= 0:
        return dict(n=n, L=0, s=n, N=n, M=rank, direct=True, b=[], Nb=0, Nc=0)
    s = -(-n // (1 << (L + 2)))
    N = s << (L + 2)
    b = [(1 << (g + 1)) - 1 for g in range(L)]  # Eq. (Nb)
    Nb = N // (2 * s) - L - 2  # Eq. (total_blocks_and_mats)
    return dict(n=n, L=L, s=s, N=N, M=rank, direct=False, b=b, Nb=Nb, Nc=3 * Nb)


def h(L: int, s: int, g: int) -> int:
    """Half the submatrix side on level g: h_g = s 2^(L-g-1)."""
    return s << (L - g - 1)


def r_of(p: int, q: int) -> int:
    """Eq. (cfrompq)."""
    return p + q * (q + 1) // 2


def corner(L: int, s: int, g: int, b: int, p: int, q: int):
    """Global (i, j) of the upper-left corner of submatrix (g, b, r(p,q)), Eq. (globalij)."""
    hg = h(L, s, g)
    return 2 * hg * (2 * b + p), 2 * hg * (2 * b + q + 2)


# ----------------------------------------------------------------------------- Lambda
mpmath.mp.dps = 30


@lru_cache(maxsize=None)
def Lambda(z: float) -> float:
    """Lambda(z) = Gamma(z+1/2)/Gamma(z+1), Eq. (Lambda)."""
    zz = mpmath.mpf(z)
    return float(mpmath.gammaprod([zz + mpmath.mpf(1) / 2], [zz + 1]))


def kernel_A(x: float, y: float) -> float:
    """A(x,y) = Lambda((y-x)/2) Lambda((y+x)/2), smooth for y > x (Sec. 3.2)."""
    return Lambda((y - x) / 2.0) * Lambda((y + x) / 2.0)


def kernel_L(x: float, y: float) -> float:
    """Reverse-direction kernel, Eq. (Lxymod)."""
    g = 2.0 * (x + 0.5) * y / ((x + y) * (x + y + 1.0) * (x - y + 1.0))
    return g * Lambda((y - x) / 2.0) / Lambda((x + y) / 2.0)


def entry(direction: int, i: int, j: int) -> float:
    """Nonzero entry (i, j), j >= i, j - i even, of A (leg2cheb) or of K = A^{-1} C diag(1/c)."""
    if direction == LEG2CHEB:
        return Lambda((j - i) / 2) * Lambda((j + i) / 2)
    if i == j:
        return math.sqrt(math.pi) / (2.0 * Lambda(i))
    return kernel_L(float(i), float(j))


# ----------------------------------------------------------------------------- tables
def vandermonde(s: int, M: int) -> np.ndarray:
    """T[sigma] = (T_k(X_m^sigma)), X_m^sigma = -1 + (2m+sigma)/s, shape (2, s, M); Eq. (Xs)."""
    T = np.empty((2, s, M))
    for sig in (0, 1):
        X = -1.0 + (2.0 * np.arange(s) + sig) / s
        T[sig] = np.cos(np.outer(np.arccos(np.clip(X, -1.0, 1.0)), np.arange(M)))
    return T


def _binom(n: int, k: int) -> int:
    return math.comb(n, k) if 0 <= k <= n else 0


def b_matrices_exact(M: int):
    """B(0), B(1) = W^{-1} V(l) W in exact rationals (App. A3, Eqs. (xn), (al), (WAW))."""
    c = lambda j: 2 if j == 0 else 1
    W = [[Fraction(0)] * M for _ in range(M)]
    Wi = [[Fraction(0)] * M for _ in range(M)]
    for n in range(M):
        for j in range(n + 1):
            if (n - j) % 2 == 0:
                W[n][j] = Fraction(2 * _binom(n, (n - j) // 2), c(j) * 2 ** n)
                if n == 0:
                    Wi[n][j] = Fraction(1)
                else:
                    Wi[n][j] = Fraction(n * (-1) ** ((n - j) // 2) * 2 ** j * _binom((n + j) // 2, (n - j) // 2), n + j)
    out = []
    for l in (0, 1):
        V = [[Fraction(_binom(n, n - j) * (2 * l - 1) ** (n - j), 2 ** n) if j <= n else Fraction(0)
              for j in range(M)] for n in range(M)]
        VW = [[sum(V[n][k] * W[k][j] for k in range(M)) for j in range(M)] for n in range(M)]
        B = [[sum(Wi[n][k] * VW[k][j] for k in range(M)) for j in range(M)] for n in range(M)]
        out.append(B)
    return out


def b_matrices(M: int) -> np.ndarray:
    """B(0), B(1) as float64, shape (2, M, M)."""
    return np.array([[[float(v) for v in row] for row in B] for B in b_matrices_exact(M)])


def ahat(direction: int, i: int, j: int, hg: int, M: int) -> np.ndarray:
    """Chebyshev coefficients of the kernel on [i, i+2h] x [j, j+2h], Eq. (aklmore)."""
    kern = kernel_A if direction == LEG2CHEB else kernel_L
    XG = np.cos((np.arange(M) + 0.5) * np.pi / M)
    x = i + hg * (XG + 1.0)
    y = j + hg * (XG + 1.0)
    S = np.array([[kern(float(xm), float(yn)) for yn in y] for xm in x])
    Cm = np.cos(np.outer(np.arange(M), (np.arange(M) + 0.5) * np.pi / M))  # cos(k(m+1/2)pi/M)
    ck = np.where(np.arange(M) == 0, 2.0, 1.0)
    out = np.zeros((M, M))
    for k in range(M):
        for l in range(M):
            out[k, l] = 4.0 / (ck[k] * ck[l] * M * M) * np.sum(S * np.outer(Cm[k], Cm[l]))
    return out


def plan(n: int, direction: int = LEG2CHEB, leaf: int = 64, rank: int = 18) -> dict:
    """All tables of the initialization stage (Secs. 3.2, 4.3) for one transform."""
    P = sizes(n, leaf, rank)
    P["direction"] = direction
    if P["direct"]:
        return P
    L, s, M = P["L"], P["s"], P["M"]
    P["T"] = vandermonde(s, M)
    P["B"] = b_matrices(M)
    A = []
    for g in range(L):
        Ag = np.zeros((P["b"][g], 3, M, M))
        for b in range(P["b"][g]):
            for q in (0, 1):
                for p in range(q + 1):
                    i, j = corner(L, s, g, b, p, q)
                    Ag[b, r_of(p, q)] = ahat(direction, i, j, h(L, s, g), M)
        A.append(Ag)
    P["Ahat"] = A
    return P


# ----------------------------------------------------------------------------- coverage
def far_field_mask(P: dict) -> np.ndarray:
    """Boolean N x N mask of the entries covered by far-field submatrices (all levels)."""
    N = P["N"]
    mask = np.zeros((N, N), dtype=np.int32)
    if P["direct"]:
        return mask
    L, s = P["L"], P["s"]
    for g in range(L):
        hg = h(L, s, g)
        for b in range(P["b"][g]):
            for q in (0, 1):
                for p in range(q + 1):
                    i, j = corner(L, s, g, b, p, q)
                    mask[i:i + 2 * hg, j:j + 2 * hg] += 1
    return mask


def near_field_mask(P: dict) -> np.ndarray:
    """Entries handled by step (6): finest row node u x columns [2su, 2s(u+2)), upper triangle."""
    N = P["N"]
    mask = np.zeros((N, N), dtype=np.int32)
    if P["direct"]:
        return np.triu(np.ones((N, N), dtype=np.int32))
    s = P["s"]
    for u in range(N // (2 * s)):
        for i in range(2 * s * u, 2 * s * (u + 1)):
            jhi = min(N, 2 * s * (u + 2))
            mask[i, i:jhi] += 1
    return mask


# ----------------------------------------------------------------------------- execute
def stage_input(P: dict, f: np.ndarray) -> np.ndarray:
    """Step (0): the input zero-padded to N; for Cheb2Leg C is applied first (u = c .* f)."""
    n, N = P["n"], P["N"]
    f = np.asarray(f, dtype=np.float64)
    assert f.shape == (n,)
    u = np.zeros(N)
    u[:n] = f
    if P["direction"] == CHEB2LEG:
        u[0] *= 2.0  # c .* f: C applied first, its pi/2 lives in the kernel
    return u


def upward(P: dict, u: np.ndarray, sig: int) -> list:
    """Steps (1)-(2) of Alg. 4 for parity sig: w[g] of shape (b_g, 2, M), where w[g][b, q]
    is the upward vector of column node 2b + q + 2 of level g (Eq. (globalij))."""
    L, s, M, T, B, bg = P["L"], P["s"], P["M"], P["T"], P["B"], P["b"]
    w = [np.zeros((bg[g], 2, M)) for g in range(L)]
    # step (1): w(L-1) = f^sigma(L-1) T(sigma), f(L-1) = f[4 h_{L-1}:] as (b, 2, 2s)
    fL = u[4 * s:].reshape(bg[L - 1], 2, 2 * s)[:, :, sig::2]
    w[L - 1] = np.einsum("bqm,mk->bqk", fL, T[sig])
    # step (2): upward, Eq. (wtk)
    for g in range(L - 1, 0, -1):
        for b in range(1, bg[g]):
            b0, q0 = divmod(b - 1, 2)
            w[g - 1][b0, q0] = B[0] @ w[g][b, 0] + B[1] @ w[g][b, 1]
    return w


def execute(P: dict, f: np.ndarray) -> np.ndarray:
    """Alg. 4 (Leg2Cheb; the same steps for Cheb2Leg with the reverse kernel)."""
    n, N, direction = P["n"], P["N"], P["direction"]
    u = stage_input(P, f)
    z = np.zeros(N)
    if not P["direct"]:
        L, s, M, T, B, A = P["L"], P["s"], P["M"], P["T"], P["B"], P["Ahat"]
        bg = P["b"]
        for sig in (0, 1):
            w = upward(P, u, sig)
            c = [np.zeros((bg[g], 2, M)) for g in range(L)]
            # step (3): far-field products
            for g in range(L):
                for b in range(bg[g]):
                    for q in (0, 1):
                        for p in range(q + 1):
                            c[g][b, p] += A[g][b, r_of(p, q)] @ w[g][b, q]
            # step (4): downward
            for g in range(L - 1):
                for b in range(bg[g + 1] - 1):
                    b0, q0 = divmod(b, 2)
                    for p in (0, 1):
                        c[g + 1][b, p] += B[p].T @ c[g][b0, q0]
            # step (5): z^sigma(L-1) = c(L-1) T^T(sigma), z(L-1) = z[:N - 4s] as (b, 2, 2s)
            zL = np.einsum("bpk,mk->bpm", c[L - 1], T[sig])
            zv = z[:N - 4 * s].reshape(bg[L - 1], 2, 2 * s)
            zv[:, :, sig::2] += zL
    # step (6): direct product over the near-diagonal entries
    s = P["s"]
    nodes = 1 if P["direct"] else N // (2 * s)
    for unode in range(nodes):
        lo, hi = (0, N) if P["direct"] else (2 * s * unode, 2 * s * (unode + 1))
        for i in range(lo, hi):
            jhi = N if P["direct"] else min(N, 2 * s * (unode + 2))
            for j in range(i, jhi, 2):
                z[i] += entry(direction, i, j) * u[j]
    # step (7)
    if direction == LEG2CHEB:
        cvec = np.where(np.arange(N) == 0, 2.0, 1.0)
        z = z / (cvec * np.pi / 2.0)
    return z[:n]
