"""The oracle of the grid pipeline (Sec. 1: a Legendre series evaluated on the
Chebyshev-Gauss points through leg2cheb and a DCT, and back), pinned to things other
than itself: scipy's DCTs, numpy's Legendre evaluation, closed forms of single
polynomials, the identity between its two independent routes (the Legendre recurrence
against the closed-form connection matrix plus cosine sums), and round trips."""
import numpy as np
import pytest
import scipy.fft as sfft
from numpy.polynomial import legendre as npleg

import oracle


def cg_points(n):
    return np.cos(np.pi * (2 * np.arange(n) + 1) / (2 * n))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 100])
def test_dct_matches_scipy(n):
    """scipy's unnormalized type 2 is twice the plain cosine sum; its type 3 is
    x_0 + 2 sum_{k>=1} x_k cos(...), i.e. 2 y - x_0."""
    x = np.random.default_rng(n).standard_normal(n)
    assert np.max(np.abs(oracle.dct(x, 2) - sfft.dct(x, 2) / 2)) <= 1e-14 * max(1, n)
    assert np.max(np.abs(oracle.dct(x, 3) - (sfft.dct(x, 3) + x[0]) / 2)) <= 1e-14 * max(1, n)


def test_dct_rows_subset():
    x = np.random.default_rng(1).standard_normal(50)
    rows = [0, 7, 49, 13]
    for kind in (2, 3):
        assert np.array_equal(oracle.dct(x, kind, rows), oracle.dct(x, kind)[rows])


def test_dct_pair_inverts():
    """Chebyshev-Gauss quadrature: DCT-3 of (2 - delta_k0)/n DCT-2 gives back the input."""
    n = 90
    x = np.random.default_rng(2).standard_normal(n)
    c = oracle.dct(x, 2) * (2.0 / n)
    c[0] /= 2
    assert np.max(np.abs(oracle.dct(c, 3) - x)) <= 1e-13


@pytest.mark.parametrize("n", [5, 37, 128])
def test_legval_matches_numpy(n):
    f = np.random.default_rng(n).standard_normal(n)
    ref = npleg.legval(cg_points(n), f)
    assert np.max(np.abs(oracle.legval_cg(f) - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_legval_single_polynomials():
    """f = e_k gives P_k at the points: 1, x, (3x^2 - 1)/2, (5x^3 - 3x)/2."""
    n = 40
    x = cg_points(n)
    closed = [np.ones(n), x, (3 * x ** 2 - 1) / 2, (5 * x ** 3 - 3 * x) / 2]
    for k, ref in enumerate(closed):
        e = np.zeros(n)
        e[k] = 1.0
        assert np.max(np.abs(oracle.legval_cg(e) - ref)) <= 4e-15   # the reference rounds in FP64


def test_two_routes_agree():
    """The Legendre recurrence at the points equals the DCT-3 of the leg2cheb coefficients."""
    n = 300
    f = np.random.default_rng(3).standard_normal(n) / np.sqrt(np.arange(1, n + 1))
    u = oracle.legval_cg(f)
    assert np.max(np.abs(u - oracle.dct(oracle.leg2cheb(f), 3))) <= 1e-14 * np.max(np.abs(u))


def test_grid_round_trip():
    n = 300
    f = np.random.default_rng(4).standard_normal(n)
    assert np.max(np.abs(oracle.grid2leg(oracle.legval_cg(f)) - f)) <= 1e-13 * np.max(np.abs(f))


def test_grid2leg_of_a_polynomial():
    """Values of P_3 on the grid give the coefficient vector e_3."""
    n = 16
    x = cg_points(n)
    e = oracle.grid2leg((5 * x ** 3 - 3 * x) / 2)
    ref = np.zeros(n)
    ref[3] = 1.0
    assert np.max(np.abs(e - ref)) <= 1e-14
