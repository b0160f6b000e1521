"""GPU parity of the batched forms (16 transforms per matrix-core tile, rank 16): FP32,
BF16 hi+lo and FP16 hi+lo far-field products with FP32 accumulation and an FP64 near field,
and the FP64 tile form.  Error bounds and their models: tests/tolerances.py.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2411_00033_amd import inputs
from tolerances import TOL32, TOL32_U, TOLBF, TOLBF_U, TOLF16, TOLF16_SCALED, TOLF16_U

pytestmark = pytest.mark.gpu


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
        assert err <= (1e-8 if rank == 12 else TOL32)   # rank 12: its truncation error


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
    worst = 0.0
    for i, (n, d) in enumerate(zip(sizes, dirs)):
        err = oracle.einf(zs[i].cpu().numpy(), oracle.transform(xs[i].cpu().numpy(), d))
        worst = max(worst, err)
        assert err <= TOL32, (n, d, err)
        assert torch.equal(zs[i], zp[i])
    print("FP32 ragged E_inf=%.2e" % worst, flush=True)


# ----------------------------------------------------------------- BF16 hi+lo form
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


def test_bf16x2_ragged_batch(l2c):
    import torch
    sizes = [70, 300, 1024, 3000, 3001, 20000] * 2
    dirs = [0] * 6 + [1] * 6
    xs = [torch.from_numpy(inputs.decaying(n, 1.0, inputs.SEED_BASE + 300 + i)).cuda() for i, n in enumerate(sizes)]
    with l2c.BatchPlan(sizes, dirs, rank=16, precision=l2c.L2C_BF16X2) as bp:
        zs = bp.execute(xs)
        torch.cuda.synchronize()
    worst = 0.0
    for i, (n, d) in enumerate(zip(sizes, dirs)):
        err = oracle.einf(zs[i].cpu().numpy(), oracle.transform(xs[i].cpu().numpy(), d))
        worst = max(worst, err)
        assert err <= TOLBF, (n, d, err)
    print("BF16X2 ragged E_inf=%.2e" % worst, flush=True)


# ----------------------------------------------------------------- undecayed inputs
@pytest.fixture(scope="module")
def undecayed():
    """16 transforms of n = 20000 with coefficients uniform on [0, 1) (Table 1's protocol,
    r = 0), and the oracle's output of both directions."""
    n, B = 20000, 16
    F = np.stack([inputs.uniform01(n, inputs.SEED_BASE + 400 + b) for b in range(B)])
    refs = {d: [oracle.transform(F[b], d) for b in range(B)] for d in (0, 1)}
    return F, refs


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("form", ["fp32", "bf16x2", "fp16x2"])
def test_batched_forms_undecayed(l2c, undecayed, form, direction):
    """Inputs without decay give the far part the weight of the whole output: the forms'
    far-field precision shows in E_inf."""
    import torch
    F, refs = undecayed
    prec, tol = {"fp32": (l2c.L2C_FP32, TOL32_U), "bf16x2": (l2c.L2C_BF16X2, TOLBF_U),
                 "fp16x2": (l2c.L2C_FP16X2, TOLF16_U)}[form]
    with l2c.Plan(F.shape[1], direction, 64, 16, precision=prec, max_batch=F.shape[0]) as p:
        Z = p.execute(torch.from_numpy(F).cuda()).cpu().numpy()
    worst = max(oracle.einf(Z[b], refs[direction][b]) for b in range(F.shape[0]))
    print("undecayed %s dir=%d E_inf=%.2e" % (form, direction, worst), flush=True)
    assert worst <= tol


# ----------------------------------------------------------------- FP16 hi+lo form
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("n", [129, 1024, 3000, 20000])
def test_fp16x2_parity_sizes(l2c, n, direction):
    """A batch of 21 (a full tile and a ragged one) against the oracle."""
    import torch
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 150 + n % 97, batch=21)
    x = torch.from_numpy(F).cuda()
    with l2c.Plan(n, direction, 64, 16, precision=l2c.L2C_FP16X2, max_batch=21) as p:
        info = p.info
        Z = p.execute(x).cpu().numpy()
    assert info["precision"] == l2c.L2C_FP16X2 and info["path"] == l2c.L2C_PATH_BATCHED
    worst = max(oracle.einf(Z[b], oracle.transform(F[b], direction)) for b in range(21))
    print("FP16X2 n=%d dir=%d E_inf=%.2e" % (n, direction, worst), flush=True)
    assert worst <= TOLF16


@pytest.mark.parametrize("direction", [0, 1])
def test_fp16x2_transforms_of_any_scale_share_a_tile(l2c, direction):
    """FP16 spans only 2^-24 .. 2^16: transforms scaled by 10^-30 .. 10^30 in one tile of 16
    each keep the form's relative accuracy (every runtime operand is scaled per transform),
    and the scaled results are the unscaled ones times the scale."""
    import torch
    n, B = 5000, 16
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 160, batch=B)
    scale = 10.0 ** np.linspace(-30, 30, B)
    Fs = F * scale[:, None]
    with l2c.Plan(n, direction, 64, 16, precision=l2c.L2C_FP16X2, max_batch=B) as p:
        Z = p.execute(torch.from_numpy(F).cuda()).cpu().numpy()
        Zs = p.execute(torch.from_numpy(Fs).cuda()).cpu().numpy()
    worst = 0.0
    for b in range(B):
        ref = oracle.transform(Fs[b], direction)
        worst = max(worst, oracle.einf(Zs[b], ref))
        assert oracle.einf(Zs[b] / scale[b], Z[b]) <= 1e-6, b
    print("FP16X2 scaled tile dir=%d E_inf=%.2e" % (direction, worst), flush=True)
    assert worst <= TOLF16_SCALED


def test_fp16x2_ragged_batch(l2c):
    import torch
    sizes = [70, 300, 1024, 3000, 3001, 20000] * 2
    dirs = [0] * 6 + [1] * 6
    xs = [torch.from_numpy(inputs.decaying(n, 1.0, inputs.SEED_BASE + 170 + i)).cuda() for i, n in enumerate(sizes)]
    with l2c.BatchPlan(sizes, dirs, rank=16, precision=l2c.L2C_FP16X2) as bp:
        zs = bp.execute(xs)
        torch.cuda.synchronize()
    worst = 0.0
    for i, (n, d) in enumerate(zip(sizes, dirs)):
        err = oracle.einf(zs[i].cpu().numpy(), oracle.transform(xs[i].cpu().numpy(), d))
        worst = max(worst, err)
        assert err <= TOLF16, (n, d, err)
    print("FP16X2 ragged E_inf=%.2e" % worst, flush=True)


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
    for prec, rank, tol, tol_rt in ((l2c.L2C_FP64, 18, (1e-13, 1e-13), 1e-13),
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


# ----------------------------------------------------------------- configuration 3
@pytest.fixture(scope="module")
def cfg3(l2c):
    """256 transforms of N = 65536, f_j = z_j/(j+1): the FP64 path's outputs (all 256) and
    the oracle of whole transforms 0, 255 and 6 seeded others (computed once)."""
    import torch
    n, B = 65536, 256
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 3, batch=B)
    x = torch.from_numpy(F).cuda()
    with l2c.Plan(n, 0, 64, 18, max_batch=B) as p64:
        z64 = p64.execute(x).cpu().numpy()
    rng = np.random.default_rng(inputs.SEED_BASE + 33)
    pick = [0, 255] + sorted(rng.choice(np.arange(1, 255), 6, replace=False).tolist())
    t0 = time.time()
    refs = {b: oracle.leg2cheb(F[b]) for b in pick}
    print("cfg3 oracle: %d whole transforms in %.1f s" % (len(pick), time.time() - t0), flush=True)
    return {"F": F, "x": x, "z64": z64, "refs": refs}


def test_config3_fp64_path(l2c, cfg3):
    """The FP64 path on the picked whole transforms against the oracle."""
    worst = max(oracle.einf(cfg3["z64"][b], ref) for b, ref in cfg3["refs"].items())
    print("cfg3 FP64 path: E_inf vs oracle %.2e" % worst, flush=True)
    assert worst <= 1e-13


@pytest.mark.parametrize("form", ["fp32", "bf16x2", "fp16x2"])
def test_config3_batch_256x65536(l2c, cfg3, form):
    """The batched form on all 256 transforms: whole transforms 0, 255 and 6 seeded others
    against the oracle, and all 256 against the FP64 path."""
    import torch
    prec, tol = {"fp32": (l2c.L2C_FP32, TOL32), "bf16x2": (l2c.L2C_BF16X2, TOLBF),
                 "fp16x2": (l2c.L2C_FP16X2, TOLF16)}[form]
    with l2c.Plan(65536, 0, 64, 16, precision=prec, max_batch=256) as p:
        assert p.info["path"] == l2c.L2C_PATH_BATCHED
        z = p.execute(cfg3["x"]).cpu().numpy()
        torch.cuda.synchronize()
    e_or = max(oracle.einf(z[b], ref) for b, ref in cfg3["refs"].items())
    e64 = max(oracle.einf(z[b], cfg3["z64"][b]) for b in range(256))
    print("cfg3 %s: E_inf vs oracle (8 whole transforms) %.2e, vs FP64 path (all 256) %.2e" % (form, e_or, e64),
          flush=True)
    assert e_or <= tol and e64 <= tol


# ----------------------------------------------------------------- FP64 tile form
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("n", [5000, 20000, 70001])
def test_fp64_tile_form_parity(l2c, n, direction):
    """FP64 plans at rank 16 for batches of 16 or more take the FP64 tile form (16
    transforms per FP64 matrix-core tile): every item of a batch of 21 (a full tile and a
    ragged one) against the oracle at the FP64 bound."""
    import torch
    from tolerances import TOL64
    B = 21
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 180 + n % 97, batch=B)
    x = torch.from_numpy(F).cuda()
    with l2c.Plan(n, direction, 64, 16, max_batch=B) as p:
        info = p.info
        Z = p.execute(x).cpu().numpy()
        z1 = p.execute(x[B - 1]).cpu().numpy()
    assert info["precision"] == l2c.L2C_FP64 and info["path"] == l2c.L2C_PATH_BATCHED
    worst = max(oracle.einf(Z[b], oracle.transform(F[b], direction)) for b in range(B))
    print("FP64 tile form n=%d dir=%d E_inf=%.2e" % (n, direction, worst), flush=True)
    assert worst <= TOL64[(direction, 18)]
    assert np.array_equal(z1, Z[B - 1])


def test_config3_fp64_tile_form(l2c, cfg3):
    """The 256 x 65536 batch in the FP64 tile form (rank 16): whole transforms against the
    oracle at the FP64 bound, all 256 against the FP64 path at rank 18."""
    import torch
    with l2c.Plan(65536, 0, 64, 16, max_batch=256) as p:
        assert p.info["path"] == l2c.L2C_PATH_BATCHED
        z = p.execute(cfg3["x"]).cpu().numpy()
        torch.cuda.synchronize()
    e_or = max(oracle.einf(z[b], ref) for b, ref in cfg3["refs"].items())
    e64 = max(oracle.einf(z[b], cfg3["z64"][b]) for b in range(256))
    print("cfg3 FP64 tile form: E_inf vs oracle %.2e, vs FP64 path rank 18 %.2e" % (e_or, e64), flush=True)
    assert e_or <= 1e-13 and e64 <= 1e-13


# ----------------------------------------------------------------- nodal basis
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("form", ["fp32", "bf16x2", "fp16x2", "fp64"])
def test_nodal_basis_against_oracle(l2c, form, direction):
    """The nodal (Lagrange) basis of Eq. (AijLag) on the batched kernels: the same
    approximation as the modal one, so the same bound; compared with the oracle on every
    transform of a batch of 21 (a full tile and a ragged one)."""
    import torch
    from tolerances import TOL64
    n, B = 20000, 21
    prec, tol = {"fp32": (l2c.L2C_FP32, TOL32), "bf16x2": (l2c.L2C_BF16X2, TOLBF),
                 "fp16x2": (l2c.L2C_FP16X2, TOLF16), "fp64": (l2c.L2C_FP64, TOL64[(direction, 16)])}[form]
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 600 + direction, batch=B)
    x = torch.from_numpy(F).cuda()
    with l2c.Plan(n, direction, 64, 16, precision=prec, max_batch=B, basis=l2c.L2C_NODAL) as p:
        info = p.info
        Z = p.execute(x).cpu().numpy()
    with l2c.Plan(n, direction, 64, 16, precision=prec, max_batch=B) as pm:
        Zm = pm.execute(x).cpu().numpy()
    assert info["basis"] == l2c.L2C_NODAL and info["path"] == l2c.L2C_PATH_BATCHED
    worst = max(oracle.einf(Z[b], oracle.transform(F[b], direction)) for b in range(B))
    dm = max(oracle.einf(Z[b], Zm[b]) for b in range(B))
    print("nodal %s dir=%d E_inf=%.2e (modal differs by %.2e)" % (form, direction, worst, dm), flush=True)
    assert worst <= tol
