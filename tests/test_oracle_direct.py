"""Pins of the direct CPU oracle (oracle.c) against values fixed by the paper and by mathematics.

Each test targets a mistake that the oracle could plausibly contain: a wrong
lambda, a dropped c_i, a transposed or shifted index, a wrong sign in the
reverse kernel, or a wrong diagonal.  None of them re-types the oracle's own
formula: the references are exact rational polynomial algebra, mpmath's gamma
function, numpy's Clenshaw evaluation of Legendre and Chebyshev series, the
printed pattern of Eq. (matH), and invariants.
"""
from fractions import Fraction
import math
import os

import mpmath
import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- exact reference
def exact_leg2cheb_matrix(n):
    """Columns j: the Chebyshev coefficients of L_j, in exact rationals.

    Built from Bonnet's recurrence (j+1) L_{j+1} = (2j+1) x L_j - j L_{j-1} and
    x T_k = (T_{k+1} + T_{|k-1|})/2, entirely in the Chebyshev basis.
    """
    def times_x(v):
        out = [Fraction(0)] * (len(v) + 1)
        for k, a in enumerate(v):
            if a == 0:
                continue
            out[k + 1] += a / 2
            out[abs(k - 1)] += a / 2
        return out

    cols = [[Fraction(1)], [Fraction(0), Fraction(1)]]
    for j in range(1, n - 1):
        xl = times_x(cols[j])
        prev = cols[j - 1] + [Fraction(0)] * (len(xl) - len(cols[j - 1]))
        cols.append([(Fraction(2 * j + 1) * a - Fraction(j) * b) / (j + 1) for a, b in zip(xl, prev)])
    M = [[Fraction(0)] * n for _ in range(n)]
    for j in range(n):
        for i, a in enumerate(cols[j][:n]):
            M[i][j] = a
    return M


def exact_upper_inverse(M):
    n = len(M)
    X = [[Fraction(0)] * n for _ in range(n)]
    for col in range(n):
        for i in range(n - 1, -1, -1):
            acc = Fraction(1 if i == col else 0)
            for k in range(i + 1, n):
                if M[i][k] != 0 and X[k][col] != 0:
                    acc -= M[i][k] * X[k][col]
            X[i][col] = acc / M[i][i]
    return X


def dense(fn, n):
    """Matrix whose column j is fn(e_j)."""
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(fn(e))
    return np.array(cols).T


N_EXACT = 40


@pytest.fixture(scope="module")
def exact40():
    M = exact_leg2cheb_matrix(N_EXACT)
    return np.array([[float(v) for v in row] for row in M]), np.array(
        [[float(v) for v in row] for row in exact_upper_inverse(M)])


# ----------------------------------------------------------------- lambda
@pytest.mark.parametrize("k", [0, 1, 2, 3, 10, 19, 20, 21, 100, 1000, 12345, 300007, 1000000, 1015807])
def test_lambda_matches_gamma_ratio(k):
    """lambda_k = Gamma(k+1/2)/Gamma(k+1), Eq. (Lambda); mpmath at 40 digits; <= 1 ulp."""
    lam = oracle.lambda_table(k + 1)[k]
    with mpmath.workdps(40):
        ref = mpmath.gammaprod([k + mpmath.mpf(1) / 2], [k + 1])
    assert abs(lam - float(ref)) <= np.spacing(float(ref))


def test_lambda_small_closed_form():
    """lambda_k = sqrt(pi) binom(2k,k)/4^k for integer k (Eq. (Lambdaint) unrolled); k < 60."""
    lam = oracle.lambda_table(60)
    with mpmath.workdps(40):
        sp = mpmath.sqrt(mpmath.pi)
        for k in range(60):
            ref = float(sp * mpmath.mpf(math.comb(2 * k, k)) / mpmath.mpf(4) ** k)
            assert abs(lam[k] - ref) <= np.spacing(ref), k


# ----------------------------------------------------------------- A and C^{-1}A
def test_leg2cheb_matches_exact_rationals(exact40):
    """Columns of C^{-1}A equal the exact Chebyshev coefficients of L_j (N = 40)."""
    E, _ = exact40
    D = dense(oracle.leg2cheb, N_EXACT)
    assert np.max(np.abs(D - E)) <= 2e-16


def test_worked_polynomials():
    """Textbook expansions: L2 = T0/4 + 3T2/4, L3 = 3T1/8 + 5T3/8, L4 = 9T0/64 + 5T2/16 + 35T4/64."""
    cases = {2: {0: 1 / 4, 2: 3 / 4}, 3: {1: 3 / 8, 3: 5 / 8}, 4: {0: 9 / 64, 2: 5 / 16, 4: 35 / 64},
             5: {1: 15 / 64, 3: 35 / 128, 5: 63 / 128}}
    for j, coef in cases.items():
        e = np.zeros(8)
        e[j] = 1.0
        z = oracle.leg2cheb(e)
        ref = np.zeros(8)
        for i, v in coef.items():
            ref[i] = v
        assert np.max(np.abs(z - ref)) <= 2e-16, j
    # and the reverse: T2 = -L0/3 + 4L2/3, T3 = -3L1/5 + 8L3/5
    for j, coef in {2: {0: -1 / 3, 2: 4 / 3}, 3: {1: -3 / 5, 3: 8 / 5}}.items():
        e = np.zeros(8)
        e[j] = 1.0
        z = oracle.cheb2leg(e)
        ref = np.zeros(8)
        for i, v in coef.items():
            ref[i] = v
        assert np.max(np.abs(z - ref)) <= 4e-16, j


def test_matH_pattern():
    """The printed corner of A, Eq. (matH): A = C * (C^{-1}A) matches lambda_k lambda_m or 0."""
    lam = oracle.lambda_table(8)
    D = dense(oracle.leg2cheb, 8)
    c = np.where(np.arange(8) == 0, 2.0, 1.0) * np.pi / 2
    A = D * c[:, None]
    with open(os.path.join(GOLDEN, "matH_pattern.txt")) as fh:
        rows = [ln.split(":", 1) for ln in fh if ln.strip() and not ln.startswith("#")]
    for r, body in rows:
        i = int(r)
        for j, tok in enumerate(body.split()):
            if tok == "0":
                assert A[i, j] == 0.0, (i, j)
            else:
                k, m = map(int, tok.split(","))
                assert abs(A[i, j] - lam[k] * lam[m]) <= 4 * np.spacing(A[i, j]), (i, j)


# ----------------------------------------------------------------- A^{-1} C
def test_cheb2leg_matches_exact_inverse(exact40):
    """Columns of A^{-1}C equal the exact inverse of the rational Legendre->Chebyshev matrix."""
    _, Ei = exact40
    D = dense(oracle.cheb2leg, N_EXACT)
    scale = np.max(np.abs(Ei), axis=0)
    assert np.max(np.abs(D - Ei) / scale) <= 1e-15


def test_cheb2leg_routes_agree():
    """The reverse-kernel route and the back-substitution route agree (n = 400)."""
    rng = np.random.default_rng(7)
    f = rng.standard_normal(400) / np.sqrt(np.arange(1, 401))
    z1, z2 = oracle.cheb2leg(f), oracle.cheb2leg_backsub(f)
    assert oracle.einf(z1, z2) <= 1e-14


# ----------------------------------------------------------------- series evaluation
@pytest.mark.parametrize("n", [64, 513, 1500])
def test_series_agree_at_chebyshev_points(n):
    """sum f_j L_j(x) == sum z_i T_i(x) at Chebyshev points (numpy Clenshaw, legval/chebval).

    Clenshaw's rounding error is bounded by a small multiple of eps * sum |f_j|
    (|L_j|, |T_j| <= 1 on [-1, 1]), so the discrepancy is measured against that.
    """
    rng = np.random.default_rng(n)
    f = rng.standard_normal(n) / np.sqrt(np.arange(1, n + 1))
    x = np.cos((np.arange(257) + 0.5) * np.pi / 257)
    z = oracle.leg2cheb(f)
    pl = np.polynomial.legendre.legval(x, f)
    pc = np.polynomial.chebyshev.chebval(x, z)
    assert np.max(np.abs(pl - pc)) / np.sum(np.abs(f)) <= 4e-14
    g = oracle.cheb2leg(f)
    pc2 = np.polynomial.chebyshev.chebval(x, f)
    pl2 = np.polynomial.legendre.legval(x, g)
    assert np.max(np.abs(pl2 - pc2)) / np.sum(np.abs(f)) <= 4e-14


# ----------------------------------------------------------------- invariants
def test_unit_vectors_and_endpoint_sums():
    for fn in (oracle.leg2cheb, oracle.cheb2leg):
        for j in (0, 1):
            e = np.zeros(50)
            e[j] = 1.0
            assert np.max(np.abs(fn(e) - e)) <= 1e-16
    rng = np.random.default_rng(3)
    f = rng.standard_normal(3000) / np.arange(1, 3001)
    sgn = (-1.0) ** np.arange(3000)
    for fn in (oracle.leg2cheb, oracle.cheb2leg):
        z = fn(f)
        # T_i(1) = L_j(1) = 1 and T_i(-1) = L_i(-1) = (-1)^i
        assert abs(z.sum() - f.sum()) <= 1e-13 * np.abs(f).sum()
        assert abs((sgn * z).sum() - (sgn * f).sum()) <= 1e-13 * np.abs(f).sum()


def test_leg2cheb_entries_nonnegative_columns_sum_to_one():
    D = dense(oracle.leg2cheb, 64)
    assert np.all(D >= 0.0)
    assert np.max(np.abs(D.sum(axis=0) - 1.0)) <= 1e-14


@pytest.mark.parametrize("fn", [oracle.leg2cheb, oracle.cheb2leg])
def test_upper_triangular_and_parity(fn):
    rng = np.random.default_rng(11)
    n = 300
    f = rng.standard_normal(n)
    z0 = fn(f)
    j = 173
    g = f.copy()
    g[j] += 1.0
    dz = fn(g) - z0
    assert np.all(dz[j + 1:] == 0.0)  # upper triangular: rows below j untouched
    assert np.all(dz[(j + 1) % 2::2] == 0.0)  # parity: only rows with i = j mod 2 change
    assert np.all(dz[j % 2:j + 1:2] != 0.0)


def test_linearity_and_zero_padding():
    rng = np.random.default_rng(5)
    f, g = rng.standard_normal(500), rng.standard_normal(500)
    for fn in (oracle.leg2cheb, oracle.cheb2leg):
        lhs = fn(2.5 * f - 0.5 * g)
        rhs = 2.5 * fn(f) - 0.5 * fn(g)
        assert oracle.einf(lhs, rhs) <= 1e-14
        pad = fn(np.concatenate([f, np.zeros(37)]))
        assert np.array_equal(pad[:500], fn(f)) and np.all(pad[500:] == 0.0)


def test_round_trip():
    rng = np.random.default_rng(9)
    f = rng.standard_normal(4000) / np.sqrt(np.arange(1, 4001))
    assert oracle.einf(oracle.cheb2leg(oracle.leg2cheb(f)), f) <= 1e-13
    assert oracle.einf(oracle.leg2cheb(oracle.cheb2leg(f)), f) <= 1e-13


def test_row_sampling_is_bitwise_the_full_result():
    rng = np.random.default_rng(2)
    f = rng.standard_normal(2000)
    rows = np.array([0, 1, 2, 777, 1998, 1999, 5])
    for fn in (oracle.leg2cheb, oracle.cheb2leg):
        assert np.array_equal(fn(f, rows), fn(f)[rows])


def test_invalid_arguments_raise():
    with pytest.raises(ValueError):
        oracle.leg2cheb(np.zeros(0))
    with pytest.raises(ValueError):
        oracle.leg2cheb(np.zeros(4), rows=[4])
