"""GPU parity of the batched FP32 form (16 transforms per matrix-core tile, rank 16).

Tolerance.  The form computes every product in FP32 (unit roundoff u = 2^-24) with FP32
accumulation; inputs are converted once, outputs are scaled and stored in FP64.  An
output row is a sum of at most 2s near-field terms plus a far-field value built through
L upward and L downward transfers of M-term sums, so the rounding error relative to
max|z| is a small multiple of (2s + 2 L M) u ~ 2e-5 at s = 32, L = 9, M = 16 for a
worst-case sign pattern; random signs give about sqrt(2s + 2 L M) u.  The bound used here
is 5e-6 (E_inf, Eq. (Einf)), about 80 u; the rank-16 truncation error (~1e-12) is far below it.
"""
import numpy as np
import pytest

import oracle
from paper_2411_00033_amd import inputs

pytestmark = pytest.mark.gpu

TOL32 = 5e-6


@pytest.fixture(scope="module")
def l2c():
    import torch
    import paper_2411_00033_amd as mod
    assert torch.cuda.is_available()
    mod._lib.load()
    return mod


def run32(l2c, F, direction, rank=16, leaf=64):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(F)).cuda()
    batch = 1 if x.dim() == 1 else x.shape[0]
    with l2c.Plan(F.shape[-1], direction, leaf, rank, precision=l2c.L2C_FP32, max_batch=batch) as p:
        info = p.info
        z = p.execute(x)
        torch.cuda.synchronize()
        return z.cpu().numpy(), info


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("n", [129, 300, 1024, 3000, 20000])
def test_fp32_parity_sizes(l2c, n, direction):
    """A batch of 21 (one full tile and a ragged one): every item against the oracle."""
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 40 + n % 97, batch=21)
    Z, info = run32(l2c, F, direction)
    assert info["precision"] == l2c.L2C_FP32
    if info["levels"] > 0:
        assert info["path"] == l2c.L2C_PATH_BATCHED
    worst = 0.0
    for b in range(F.shape[0]):
        worst = max(worst, oracle.einf(Z[b], oracle.transform(F[b], direction)))
    print("FP32 n=%d dir=%d L=%d E_inf=%.2e" % (n, direction, info["levels"], worst))
    assert worst <= TOL32


def test_fp32_rank12_and_small_leaf(l2c):
    n = 5000
    F = inputs.decaying(n, 0.5, inputs.SEED_BASE + 41, batch=3)
    for rank, leaf in ((12, 64), (16, 32), (16, 40)):
        Z, info = run32(l2c, F, 0, rank=rank, leaf=leaf)
        err = max(oracle.einf(Z[b], oracle.leg2cheb(F[b])) for b in range(3))
        print("FP32 rank=%d leaf=%d s=%d E_inf=%.2e" % (rank, leaf, info["s"], err))
        assert err <= (1e-4 if rank == 12 else TOL32)


def test_fp32_unsupported(l2c):
    with pytest.raises(l2c.L2CError) as ei:
        l2c.Plan(1000, 0, 64, 18, precision=l2c.L2C_FP32)
    assert ei.value.code == l2c.L2C_EUNSUPPORTED
    with pytest.raises(l2c.L2CError) as ei:
        l2c.Plan(1000, 0, 128, 16, precision=l2c.L2C_FP32)
    assert ei.value.code == l2c.L2C_EUNSUPPORTED
    with l2c.Plan(1000, 0, 64, 16, precision=l2c.L2C_FP32) as p:
        with pytest.raises(l2c.L2CError) as ei:
            p.export(l2c.TABLE_AHAT)
        assert ei.value.code == l2c.L2C_EUNSUPPORTED


def test_fp32_ragged_batch(l2c):
    """Ragged FP32 batch: mixed lengths and directions, every output against the oracle."""
    import torch
    sizes = [1, 70, 128, 129, 1000, 1024, 2990, 3000, 3007, 9000, 9001, 20000] * 2
    dirs = [0] * 12 + [1] * 12
    xs = [torch.from_numpy(inputs.decaying(n, 1.0, inputs.SEED_BASE + 200 + i)).cuda() for i, n in enumerate(sizes)]
    with l2c.BatchPlan(sizes, dirs, rank=16, precision=l2c.L2C_FP32) as bp:
        zs = bp.execute(xs)
        zp = [torch.empty_like(x) for x in xs]
        bp.execute_ptrs([x.data_ptr() for x in xs], [z.data_ptr() for z in zp])
        torch.cuda.synchronize()
    for i, (n, d) in enumerate(zip(sizes, dirs)):
        err = oracle.einf(zs[i].cpu().numpy(), oracle.transform(xs[i].cpu().numpy(), d))
        assert err <= TOL32, (n, d, err)
        assert torch.equal(zs[i], zp[i])


def test_config3_fp32_batch_256x65536(l2c):
    """256 x N = 65536, f = z/(j+1): all 256 against the FP64 GPU path, 8 against the oracle
    (rows 0, 255 and 6 random)."""
    import torch
    n, B = 65536, 256
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 3, batch=B)
    x = torch.from_numpy(F).cuda()
    with l2c.Plan(n, 0, 64, 16, precision=l2c.L2C_FP32, max_batch=B) as p32, \
            l2c.Plan(n, 0, 64, 18, max_batch=B) as p64:
        z32 = p32.execute(x)
        z64 = p64.execute(x)
        torch.cuda.synchronize()
    z32, z64 = z32.cpu().numpy(), z64.cpu().numpy()
    e64 = max(oracle.einf(z32[b], z64[b]) for b in range(B))
    rng = np.random.default_rng(inputs.SEED_BASE + 33)
    worst = 0.0
    for b in rng.choice(B, 8, replace=False):
        rows = np.unique(np.concatenate([[0, 255], rng.integers(0, n, 6)]))
        ref = oracle.leg2cheb(F[b], rows)
        worst = max(worst, np.max(np.abs(z32[b][rows] - ref)) / np.max(np.abs(ref)))
    print("cfg3 FP32: E_inf vs FP64 path %.2e, sampled vs oracle %.2e" % (e64, worst))
    assert e64 <= TOL32 and worst <= TOL32


# ----------------------------------------------------------------- BF16 hi+lo form
# Each product is ah bh + ah bl + al bh with hi/lo BF16 splits: the dropped al bl and the
# rounding of the lo parts leave about 2^-17 relative error per product (FP32 accumulation
# adds 2^-24).  With the same (2s + 2 L M)-term error model as above, random signs give
# about sqrt(352) 2^-17 ~ 1.4e-4; the bound is 5e-4.
TOLBF = 5e-4


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("n", [129, 1024, 20000])
def test_bf16x2_parity_sizes(l2c, n, direction):
    import torch
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 50 + n % 97, batch=21)
    x = torch.from_numpy(F).cuda()
    with l2c.Plan(n, direction, 64, 16, precision=l2c.L2C_BF16X2, max_batch=21) as p:
        info = p.info
        Z = p.execute(x).cpu().numpy()
    assert info["precision"] == l2c.L2C_BF16X2
    worst = max(oracle.einf(Z[b], oracle.transform(F[b], direction)) for b in range(21))
    print("BF16X2 n=%d dir=%d E_inf=%.2e" % (n, direction, worst))
    assert worst <= TOLBF


def test_config3_bf16x2_batch_256x65536(l2c):
    """256 x N = 65536: the BF16 hi+lo form against the FP64 GPU path on all 256."""
    import torch
    n, B = 65536, 256
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 3, batch=B)
    x = torch.from_numpy(F).cuda()
    with l2c.Plan(n, 0, 64, 16, precision=l2c.L2C_BF16X2, max_batch=B) as pb, \
            l2c.Plan(n, 0, 64, 18, max_batch=B) as p64:
        zb = pb.execute(x)
        z64 = p64.execute(x)
        torch.cuda.synchronize()
    zb, z64 = zb.cpu().numpy(), z64.cpu().numpy()
    e64 = max(oracle.einf(zb[b], z64[b]) for b in range(B))
    print("cfg3 BF16X2: E_inf vs FP64 path %.2e" % e64)
    assert e64 <= TOLBF


def test_bf16x2_ragged_batch(l2c):
    import torch
    sizes = [70, 300, 1024, 3000, 3001, 20000] * 2
    dirs = [0] * 6 + [1] * 6
    xs = [torch.from_numpy(inputs.decaying(n, 1.0, inputs.SEED_BASE + 300 + i)).cuda() for i, n in enumerate(sizes)]
    with l2c.BatchPlan(sizes, dirs, rank=16, precision=l2c.L2C_BF16X2) as bp:
        zs = bp.execute(xs)
        torch.cuda.synchronize()
    for i, (n, d) in enumerate(zip(sizes, dirs)):
        err = oracle.einf(zs[i].cpu().numpy(), oracle.transform(xs[i].cpu().numpy(), d))
        assert err <= TOLBF, (n, d, err)


# ----------------------------------------------------------------- 3-D line batch
def test_lines_3d_round_trip(l2c):
    """A 256 x 256 x 1024 tensor, f_k = z/(k+1) along the last axis (65536 lines of
    N = 1024): leg2cheb then cheb2leg along that axis, in the FP64 path and the FP32
    form.  Round trip against the input on every line; each direction against the
    oracle on 64 seeded lines."""
    import torch
    n, lines = 1024, 256 * 256
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 5, batch=lines)
    x = torch.from_numpy(F).cuda()
    rng = np.random.default_rng(inputs.SEED_BASE + 55)
    pick = rng.choice(lines, 64, replace=False)
    for prec, rank, tol, tol_rt in ((l2c.L2C_FP64, 18, (1e-13, 1e-12), 1e-12),
                                    (l2c.L2C_FP32, 16, (TOL32, TOL32), 2 * TOL32)):
        with l2c.Plan(n, 0, 64, rank, precision=prec, max_batch=lines) as pf, \
                l2c.Plan(n, 1, 64, rank, precision=prec, max_batch=lines) as pb:
            z = pf.execute(x)
            g = pb.execute(z)
            torch.cuda.synchronize()
        rt = ((g - x).abs().amax(dim=1) / x.abs().amax(dim=1)).max().item()
        zh = z[torch.from_numpy(pick).cuda()].cpu().numpy()
        e_f = max(oracle.einf(zh[i], oracle.leg2cheb(F[b])) for i, b in enumerate(pick))
        e_b = max(oracle.einf(g[int(b)].cpu().numpy(), oracle.cheb2leg(zh[i])) for i, b in enumerate(pick))
        print("lines 3-D precision %d: leg2cheb %.2e cheb2leg %.2e round trip %.2e" % (prec, e_f, e_b, rt))
        assert e_f <= tol[0] and e_b <= tol[1] and rt <= tol_rt


def test_ragged_2048_fp32_sampled(l2c):
    """The 2048-transform ragged batch (n log-uniform in [128, 262144], directions 50/50,
    f_j = z_j/(j+1)) in the FP32 form: sampled rows of every output against the oracle and
    the x = +-1 sums of every full output."""
    import torch
    sizes, dirs = inputs.ragged_sizes(2048, inputs.SEED_BASE + 4)
    rng = np.random.default_rng(inputs.SEED_BASE + 6)
    total = int(sizes.sum())
    flat = rng.standard_normal(total)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    for i, n in enumerate(sizes):
        flat[offs[i]:offs[i + 1]] /= np.arange(1, n + 1, dtype=np.float64)
    x = torch.from_numpy(flat).cuda()
    y = torch.empty_like(x)
    xs = [x[offs[i]:offs[i + 1]] for i in range(len(sizes))]
    ys = [y[offs[i]:offs[i + 1]] for i in range(len(sizes))]
    with l2c.BatchPlan(sizes.tolist(), dirs.tolist(), rank=16, precision=l2c.L2C_FP32) as bp:
        bp.execute(xs, ys)
        torch.cuda.synchronize()
    yh = y.cpu().numpy()
    worst = 0.0
    for i, (n, d) in enumerate(zip(sizes.tolist(), dirs.tolist())):
        f, z = flat[offs[i]:offs[i + 1]], yh[offs[i]:offs[i + 1]]
        rows = np.unique(np.concatenate([[0, 1, n - 1], rng.integers(0, n, 2)]))
        ref = oracle.transform(f, d, rows)
        worst = max(worst, np.max(np.abs(z[rows] - ref)) / np.max(np.abs(ref)))
        sgn = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
        for w in (np.ones(n), sgn):
            assert abs(float(np.dot(w, z)) - float(np.dot(w, f))) <= 1e-4 * np.sum(np.abs(f)), (i, n, d)
    print("ragged 2048 FP32 sampled E_inf %.2e" % worst)
    assert worst <= TOL32
