"""Pins of the numpy reference of the modal multipole method (oracle/fmm_ref.py).

The plan tables are checked against the values the paper prints (B rows, the
tau coefficients, the block counts of Sec. 3.1), against their defining
identities, and the seven steps of Alg. 4 are checked against the direct
oracle, which the tests in test_oracle_direct.py pin independently.
"""
from fractions import Fraction
import os

import mpmath
import numpy as np
import pytest

import oracle
from oracle import fmm_ref as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


# ----------------------------------------------------------------- B(l)
def test_b_rows_match_printed_eq_appT():
    B = F.b_matrices_exact(18)
    printed = {}
    for name, r, c, num, den in _golden_lines("b_rows_eq_appT.txt"):
        printed[(int(name[1]), int(r), int(c))] = Fraction(int(num), int(den))
    for l in (0, 1):
        for r in range(4):
            for c in range(18):
                assert B[l][r][c] == printed.get((l, r, c), Fraction(0)), (l, r, c)


def test_b_structure_exact_dyadic_and_sign_relation():
    """Lower triangular, dyadic (exact in FP64), B(1)_nk = (-1)^(n-k) B(0)_nk (App. A2, A3)."""
    B = F.b_matrices_exact(18)
    for n in range(18):
        for k in range(18):
            if k > n:
                assert B[0][n][k] == 0 and B[1][n][k] == 0
            assert B[1][n][k] == (-1) ** ((n - k) % 2) * B[0][n][k]
            d = B[0][n][k].denominator
            assert d & (d - 1) == 0  # power of two
            assert float(B[0][n][k]) == B[0][n][k]  # exactly representable


def test_b_defining_identity():
    """T_n((Y+2l-1)/2) = sum_k b^(l)_nk T_k(Y), Eq. (Tky), at random Y (numpy chebval)."""
    M = 18
    B = F.b_matrices(M)
    Y = np.random.default_rng(1).uniform(-1, 1, 200)
    for l in (0, 1):
        for n in range(M):
            e = np.zeros(n + 1)
            e[n] = 1.0
            lhs = np.polynomial.chebyshev.chebval((Y + 2 * l - 1) / 2, e)
            rhs = np.polynomial.chebyshev.chebval(Y, B[l][n])
            assert np.max(np.abs(lhs - rhs)) <= 1e-14


# ----------------------------------------------------------------- sizes and coverage
def test_block_counts_match_sec31_example():
    g = {ln[0]: [int(v) for v in ln[1:]] for ln in _golden_lines("levels_fig3levels.txt")}
    L = g["levels"][0]
    P = F.sizes(32 * 2 ** (L + 2), leaf=64)
    assert P["L"] == L and P["b"] == g["blocks"] and P["Nb"] == g["total_blocks"][0]
    assert P["Nc"] == 3 * g["total_blocks"][0]


@pytest.mark.parametrize("n,leaf", [(1000000, 64), (1024, 64), (65536, 64), (128, 64), (129, 64),
                                    (262144, 64), (100, 16), (5, 64), (1, 64), (300, 8)])
def test_sizes_rules(n, leaf):
    """Eq. (numlevels): s in [s_hat/2, s_hat], N = s 2^(L+2) >= n; Eq. (total_blocks_and_mats)."""
    P = F.sizes(n, leaf)
    if P["direct"]:
        assert n <= 2 * leaf
        return
    shat, L, s, N = leaf // 2, P["L"], P["s"], P["N"]
    assert N == s * 2 ** (L + 2) and N >= n and N - n < 2 ** (L + 2)
    assert shat / 2 <= s <= shat
    assert P["Nb"] == sum(P["b"]) == N // (2 * s) - L - 2


def test_config_sizes():
    """The single-transform sizes at N = 10^6, leaf 64: L = 13, s = 31, N = 1015808."""
    P = F.sizes(10 ** 6, 64)
    assert (P["L"], P["s"], P["N"], P["Nb"], P["Nc"]) == (13, 31, 1015808, 16369, 49107)


@pytest.mark.parametrize("n,leaf", [(256, 8), (200, 8), (96, 4), (512, 16), (1000, 32), (17, 4)])
def test_far_and_near_fields_tile_the_upper_triangle_once(n, leaf):
    P = F.sizes(n, leaf)
    if P["direct"]:
        pytest.skip("direct-only size")
    N = P["N"]
    tot = F.far_field_mask(P) + F.near_field_mask(P)
    assert np.array_equal(tot, np.triu(np.ones((N, N), dtype=np.int32)))


# ----------------------------------------------------------------- Lambda and tau
def test_lambda_reference_matches_binomial_form():
    with mpmath.workdps(40):
        for k in (0, 1, 5, 20, 57):
            ref = mpmath.sqrt(mpmath.pi) * mpmath.binomial(2 * k, k) / mpmath.mpf(4) ** k
            assert abs(F.Lambda(float(k)) - float(ref)) <= np.spacing(float(ref))


def test_tau_series_accuracy_claim():
    """Eq. (tau) truncated to 5/4/3/2 terms stays within one eps (2^-52) of the exact ratio.

    Reading: the printed thresholds bound Lambda's argument z, so the series is
    evaluated at x = z + 1/4 (Lambda(z) = tau(z+1/4)/sqrt(z+1/4)).  Taken at x = z
    the 5-term threshold 19.88 would be 1.13 eps at its low end.
    """
    rows = _golden_lines("tau_eq_tau.txt")
    coef = [(int(p), Fraction(int(a), int(b))) for p, a, b in [r for r in rows if r[0] != "threshold"]]
    thr = {int(t): float(z) for _, t, z in [r for r in rows if r[0] == "threshold"]}
    with mpmath.workdps(40):
        for terms, zmin in thr.items():
            for z in np.linspace(zmin + 0.01, zmin * 4, 23):
                x = mpmath.mpf(z) + mpmath.mpf(1) / 4
                ref = mpmath.sqrt(x) * mpmath.gamma(x + 0.25) / mpmath.gamma(x + 0.75)
                approx = sum(mpmath.mpf(c.numerator) / c.denominator * x ** (-p) for p, c in coef[:terms])
                assert abs(approx / ref - 1) <= 2.0 ** -52, (terms, z)


# ----------------------------------------------------------------- Ahat and T
def test_vandermonde_is_chebyshev():
    T = F.vandermonde(31, 18)
    for sig in (0, 1):
        X = -1.0 + (2.0 * np.arange(31) + sig) / 31
        ref = np.polynomial.chebyshev.chebvander(X, 17)
        assert np.max(np.abs(T[sig] - ref)) <= 1e-14


@pytest.mark.parametrize("direction,tol", [(0, 1e-14), (1, 1e-12)])
def test_ahat_reproduces_kernel(direction, tol):
    """Sum_kl ahat_kl T_k(X) T_l(Y) matches the kernel at samples and at integer entries (Eq. (Aij))."""
    P = F.plan(1024, direction, 64, 18)
    L, s = P["L"], P["s"]
    for g, b, p, q in [(L - 1, 0, 0, 0), (L - 1, 3, 1, 1), (L - 2, 1, 0, 1), (0, 0, 0, 0)]:
        hg = F.h(L, s, g)
        i, j = F.corner(L, s, g, b, p, q)
        A = P["Ahat"][g][b, F.r_of(p, q)]
        XG = np.cos((np.arange(18) + 0.5) * np.pi / 18)
        V = np.polynomial.chebyshev.chebvander(XG, 17)
        S = V @ A @ V.T
        kern = F.kernel_A if direction == 0 else F.kernel_L
        Sref = np.array([[kern(i + hg * (xm + 1), j + hg * (yn + 1)) for yn in XG] for xm in XG])
        assert np.max(np.abs(S - Sref)) <= 1e-14 * np.max(np.abs(Sref))
        # integer grid entries of the same parity
        for sig in (0, 1):
            X = -1.0 + (2.0 * np.arange(hg) + sig) / hg
            Vx = np.polynomial.chebyshev.chebvander(X, 17)
            E = Vx @ A @ Vx.T
            Eref = np.array([[F.entry(direction, i + 2 * m + sig, j + 2 * n_ + sig) for n_ in range(hg)]
                             for m in range(hg)])
            assert np.max(np.abs(E - Eref)) <= tol * np.max(np.abs(Eref))


# ----------------------------------------------------------------- Alg. 4 vs direct
@pytest.mark.parametrize("n,leaf", [(1024, 64), (700, 32), (100, 16), (256, 64), (64, 64), (1, 64)])
@pytest.mark.parametrize("direction", [0, 1])
def test_alg4_matches_direct_oracle(n, leaf, direction):
    f = np.random.default_rng(n + direction).standard_normal(n) / np.arange(1, n + 1)
    P = F.plan(n, direction, leaf, 18)
    z = F.execute(P, f)
    assert oracle.einf(z, oracle.transform(f, direction)) <= 2e-15


@pytest.mark.parametrize("n", [300, 1000, 3000])
@pytest.mark.parametrize("direction", [0, 1])
def test_upward_vectors_are_chebyshev_moments(n, direction):
    """Steps (1)-(2): the upward vector of every column node equals the node's Chebyshev
    moments taken directly, w_k = sum_e T_k(-1 + e/h_g) u[2 h_g t + e] over the node's 2 h_g
    entries e of parity sigma (h_g = s 2^(L-g-1)).  The B(l) re-expansion of Eq. (Tky) is
    exact for degree < M, so the two agree to rounding; a wrong B, child order, parity or
    level offset breaks it."""
    sz = F.sizes(n, 64, 18)
    P = dict(sz, direction=direction, T=F.vandermonde(sz["s"], 18), B=F.b_matrices(18))
    f = np.random.default_rng(n + direction).standard_normal(n)
    u = F.stage_input(P, f)
    L, s = P["L"], P["s"]
    for sig in (0, 1):
        w = F.upward(P, u, sig)
        for g in range(L):
            hg = s << (L - g - 1)
            e = np.arange(sig, 2 * hg, 2)
            V = np.polynomial.chebyshev.chebvander(-1.0 + e / hg, 17)   # [entry][k]
            ref = np.zeros_like(w[g])
            for b in range(P["b"][g]):
                for q in (0, 1):
                    t = 2 * b + q + 2
                    ref[b, q] = u[2 * hg * t + e] @ V
            scale = np.max(np.abs(ref))
            assert np.max(np.abs(w[g] - ref)) <= 1e-13 * scale, (sig, g)
