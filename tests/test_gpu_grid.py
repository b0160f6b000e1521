"""GPU parity of the DCTs (the library's hand-written FFT) and of the grid pipeline
(Legendre series on the Chebyshev-Gauss grid and back, Sec. 1) against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2411_00033_amd import inputs
from tolerances import TOL_DCT, TOL_GRID

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def l2c():
    import torch
    import paper_2411_00033_amd as mod
    assert torch.cuda.is_available()
    mod._lib.load()
    return mod


def rel(z, ref):
    return float(np.max(np.abs(z - ref)) / max(np.max(np.abs(ref)), 1e-300))


# one-pass lengths (<= 4096, mixed radices, a ragged last workgroup of lines) and
# four-step lengths (n1 n2 with n1, n2 <= 4096); a DCT-3 of even length >= 16 takes the
# half-length DFT (16: the shortest, 18: an odd half length; 12 and the odd lengths: the
# full-length DFT)
SMALL = [1, 2, 3, 5, 7, 8, 12, 16, 18, 30, 49, 64, 100, 343, 1000, 1024, 2187, 3125, 4096]
LARGE = [4200, 6000, 65536, 100000, 117649, 177147, 1 << 20]


@pytest.mark.parametrize("kind", [2, 3])
@pytest.mark.parametrize("n", SMALL + LARGE)
def test_dct_against_oracle(l2c, n, kind):
    import torch
    B = 3
    F = inputs.decaying(n, 0.0, inputs.SEED_BASE + 500 + n % 101, batch=B)
    with l2c.Dct(n, kind, max_batch=B) as d:
        Y = d.execute(torch.from_numpy(F).cuda()).cpu().numpy()
    rows = None if n <= 4200 else np.unique(np.r_[0, 1, n // 2, n - 1, np.random.default_rng(n).integers(0, n, 28)])
    worst = 0.0
    for b in range(B):
        ref = oracle.dct(F[b], kind, rows)
        worst = max(worst, rel(Y[b] if rows is None else Y[b][rows], ref))
    print("DCT-%d n=%d E_inf=%.2e" % (kind, n, worst), flush=True)
    assert worst <= TOL_DCT


@pytest.mark.parametrize("kind", [2, 3])
def test_dct_n_1e6_sampled(l2c, kind):
    """The configuration-2 length, 10^6 (three FFT passes; DCT-3 on the half-length DFT): 48 sampled outputs
    against the oracle."""
    import torch
    n = 10 ** 6
    f = inputs.decaying(n, 0.5, inputs.SEED_BASE + 2)
    with l2c.Dct(n, kind) as d:
        y = d.execute(torch.from_numpy(f).cuda()).cpu().numpy()
    rows = np.unique(np.r_[0, 1, 2, n // 2, n - 2, n - 1, np.random.default_rng(7).integers(0, n, 42)])
    err = rel(y[rows], oracle.dct(f, kind, rows)) * np.max(np.abs(y[rows])) / np.max(np.abs(y))
    print("DCT-%d n=1e6 E_inf (sampled rows, relative to max|y|) %.2e" % (kind, err), flush=True)
    assert err <= TOL_DCT


def test_dct_pair_round_trip(l2c):
    import torch
    n = 65536
    x = torch.from_numpy(inputs.decaying(n, 0.0, inputs.SEED_BASE + 510)).cuda()
    with l2c.Dct(n, 2) as d2, l2c.Dct(n, 3) as d3:
        y = d2.execute(x) * (2.0 / n)
        y[0] *= 0.5
        back = d3.execute(y)
    e = rel(back.cpu().numpy(), x.cpu().numpy())
    print("DCT pair round trip n=%d E_inf %.2e" % (n, e), flush=True)
    assert e <= TOL_DCT


def test_dct_unsupported_lengths(l2c):
    for n in (11, 4099, 4097 * 8, (1 << 24) + 4096, 1 << 28):
        with pytest.raises(l2c.L2CError) as ei:
            l2c.Dct(n, 2)
        assert ei.value.code == l2c.L2C_EUNSUPPORTED, n


@pytest.mark.parametrize("n", [1, 30, 1024, 6000, 65536])
def test_leg2grid_against_oracle(l2c, n):
    import torch
    B = 2
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 520 + n % 89, batch=B)
    with l2c.GridPlan(n, l2c.LEG2GRID, max_batch=B) as g:
        U = g.execute(torch.from_numpy(F).cuda()).cpu().numpy()
    rows = None if n <= 6000 else np.unique(np.r_[0, n - 1, np.random.default_rng(n).integers(0, n, 30)])
    worst = 0.0
    for b in range(B):
        ref = oracle.legval_cg(F[b], rows)
        got = U[b] if rows is None else U[b][rows]
        worst = max(worst, np.max(np.abs(got - ref)) / np.max(np.abs(U[b])))
    print("leg2grid n=%d E_inf=%.2e" % (n, worst), flush=True)
    assert worst <= TOL_GRID(n)


@pytest.mark.parametrize("n", [1, 30, 1024, 6000])
def test_grid2leg_against_oracle(l2c, n):
    import torch
    rng = np.random.default_rng(n + 3)
    xs = np.cos(np.pi * (2 * np.arange(n) + 1) / (2 * n))
    u = np.exp(xs) * np.sin(3 * xs) + 0.1 * rng.standard_normal(n)   # values on the grid
    with l2c.GridPlan(n, l2c.GRID2LEG) as g:
        f = g.execute(torch.from_numpy(u).cuda()).cpu().numpy()
    e = rel(f, oracle.grid2leg(u))
    print("grid2leg n=%d E_inf=%.2e" % (n, e), flush=True)
    assert e <= TOL_GRID(n)


@pytest.mark.parametrize("n", [1024, 65536, 10 ** 6])
def test_grid_round_trip(l2c, n):
    """GRID2LEG undoes LEG2GRID (configuration inputs f_j = z_j/sqrt(j+1) at 10^6)."""
    import torch
    f = inputs.decaying(n, 0.5, inputs.SEED_BASE + 2 if n == 10 ** 6 else inputs.SEED_BASE + 530)
    x = torch.from_numpy(f).cuda()
    with l2c.GridPlan(n, l2c.LEG2GRID) as fw, l2c.GridPlan(n, l2c.GRID2LEG) as bw:
        back = bw.execute(fw.execute(x))
    e = rel(back.cpu().numpy(), f)
    print("grid round trip n=%d E_inf=%.2e" % (n, e), flush=True)
    assert e <= TOL_GRID(n)


def test_leg2grid_n_1e6_sampled(l2c):
    import torch
    n = 10 ** 6
    f = inputs.decaying(n, 0.5, inputs.SEED_BASE + 2)
    with l2c.GridPlan(n, l2c.LEG2GRID) as g:
        u = g.execute(torch.from_numpy(f).cuda()).cpu().numpy()
        assert g.fmm_info["path"] == l2c.L2C_PATH_SINGLE
    rows = np.unique(np.r_[0, n - 1, np.random.default_rng(11).integers(0, n, 30)])
    err = np.max(np.abs(u[rows] - oracle.legval_cg(f, rows))) / np.max(np.abs(u))
    print("leg2grid n=1e6 E_inf (sampled rows, relative to max|u|) %.2e" % err, flush=True)
    assert err <= TOL_GRID(n)
