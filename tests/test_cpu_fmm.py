"""The single-threaded CPU FMM (oracle/cpu_fmm.cpp, Alg. 4), the benchmark's CPU baseline,
pinned on the CPU: against the direct oracle in both directions at sizes that span the
direct-only case, one level and many levels with ragged padding; against exact worked
conversions of single Legendre polynomials (through the multipole path, not the direct
one); against the x = +-1 identities and the round trip; and its sizes against
Eq. (numlevels)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import cpu_fmm
from paper_2411_00033_amd import inputs


@pytest.mark.parametrize("n", [1, 2, 5, 64, 127, 128, 129, 255, 257, 1000, 1024, 1025, 3001, 20000, 70001])
@pytest.mark.parametrize("direction", [0, 1])
def test_against_direct_oracle(n, direction):
    f = inputs.decaying(n, 0.5, inputs.SEED_BASE + 500 + n)
    z = cpu_fmm.transform(f, direction)
    err = oracle.einf(z, oracle.transform(f, direction))
    assert err <= 1e-14, (n, direction, err)


def test_single_legendre_polynomials_exact():
    """L_4 = 9/64 T_0 + 5/16 T_2 + 35/64 T_4 and L_5 = 15/64 T_1 + 35/128 T_3 + 63/128 T_5
    (the Legendre recurrence written in the Chebyshev basis): f = e_4 and e_5 in a transform
    of length 1000, which runs the multipole path (L = 3), give those coefficients and
    zeros elsewhere."""
    n = 1000
    with cpu_fmm.CpuFmm(n, 0) as p:
        assert p.L == 3
        for j, coef in ((4, {0: Fraction(9, 64), 2: Fraction(5, 16), 4: Fraction(35, 64)}),
                        (5, {1: Fraction(15, 64), 3: Fraction(35, 128), 5: Fraction(63, 128)})):
            f = np.zeros(n)
            f[j] = 1.0
            z = p.execute(f)
            want = np.zeros(n)
            for k, v in coef.items():
                want[k] = float(v)
            assert np.max(np.abs(z - want)) <= 4e-16, j


@pytest.mark.parametrize("direction", [0, 1])
def test_identities_and_round_trip(direction):
    n = 50000
    f = inputs.decaying(n, 1.0, inputs.SEED_BASE + 510)
    z = cpu_fmm.transform(f, direction)
    sgn = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    for w in (np.ones(n), sgn):
        assert abs(np.dot(w, z) - np.dot(w, f)) <= 1e-13 * np.sum(np.abs(f))
    back = cpu_fmm.transform(z, 1 - direction)
    assert oracle.einf(back, f) <= 1e-13


def test_sizes_follow_numlevels():
    for n, want in ((1024, (3, 32, 1024)), (10 ** 6, (13, 31, 1015808)), (65536, (9, 32, 65536)), (100, (0, 0, 100))):
        with cpu_fmm.CpuFmm(n, 0) as p:
            assert (p.L, p.s, p.N) == want, n


def test_rejects_bad_arguments():
    for args in ((0, 0, 64, 18), (10, 2, 64, 18), (10, 0, 63, 18), (10, 0, 64, 0)):
        with pytest.raises(ValueError):
            cpu_fmm.CpuFmm(*args)
