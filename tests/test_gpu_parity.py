"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (E_inf of Eq. (Einf) against the direct FP64 oracle) are in tests/tolerances.py
with their error models: 1e-13 for both directions of the FP64 path at rank >= 18 on
decaying inputs; the uniform-input protocol of Table 1 against the printed values.
"""
import os
import time

import numpy as np
import pytest

import oracle
from oracle import fmm_ref
from paper_2411_00033_amd import inputs
from tolerances import TOL32, TOL64 as TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def l2c():
    import torch
    import paper_2411_00033_amd as mod
    assert torch.cuda.is_available()
    mod._lib.load()
    return mod


def run(l2c, f, direction, leaf=64, rank=18, single=None, direct=None):
    """Execute through the C ABI; single=None keeps the plan's default path, True/False forces
    the single-launch / three-launch path (Alg. 4); direct=False keeps Alg. 4 (the plan's
    multipole path) where short transforms would take the direct product."""
    import torch
    x = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    batch = 1 if x.dim() == 1 else x.shape[0]
    with l2c.Plan(f.shape[-1], direction, leaf, rank, max_batch=batch) as p:
        if (single is not None or direct is False) and p.info["levels"] > 0:
            p.set_direct(False)
        if single is not None and p.info["levels"] > 0:
            p.set_single_launch(single)
        z = p.execute(x)
        torch.cuda.synchronize()
        info = p.info
        assert p.status == 0
        if single is not None and info["levels"] > 0:
            assert info["path"] == (l2c.L2C_PATH_SINGLE if single else l2c.L2C_PATH_THREE)
        return z.cpu().numpy(), info


# ----------------------------------------------------------------- plan tables
def test_plan_tables_match_reference(l2c):
    import torch
    for direction in (0, 1):
        with l2c.Plan(1024, direction, 64, 18) as p:
            ref = fmm_ref.plan(1024, direction, 64, 18)
            B = p.export(l2c.TABLE_B).reshape(2, 18, 18)
            assert np.array_equal(B, fmm_ref.b_matrices(18))          # exact dyadic
            T = p.export(l2c.TABLE_T).reshape(2, ref["s"], 18)
            assert np.max(np.abs(T - ref["T"])) <= 1e-14
            A = p.export(l2c.TABLE_AHAT).reshape(-1, 3, 18, 18)
            Aref = np.concatenate([ref["Ahat"][g] for g in range(ref["L"])], axis=0)
            assert A.shape == Aref.shape
            scale = np.max(np.abs(Aref), axis=(2, 3), keepdims=True)
            assert np.max(np.abs(A - Aref) / scale) <= 5e-15, direction
            torch.cuda.synchronize()


@pytest.mark.parametrize("n", [300, 1024, 3000])
@pytest.mark.parametrize("direction", [0, 1])
def test_upward_phase_matches_reference(l2c, n, direction):
    """Steps (0)-(2) on the GPU (k_up, k_top of the three-launch path) against the host
    reference of the same phase: every level's upward vectors of the first item, read
    from the plan's workspace, within rounding of fmm_ref.upward."""
    import torch
    f = inputs.decaying(n, 1.0, inputs.SEED_BASE + 80 + n)
    x = torch.from_numpy(f).cuda()
    with l2c.Plan(n, direction, 64, 18) as p:
        p.set_direct(False)
        p.set_single_launch(False)
        p.execute(x)
        torch.cuda.synchronize()
        info = p.info
        W = p.export(l2c.TABLE_W).reshape(-1, 2, 18)
    sz = fmm_ref.sizes(n, 64, 18)
    assert (info["levels"], info["s"]) == (sz["L"], sz["s"])
    P = dict(sz, direction=direction, T=fmm_ref.vandermonde(sz["s"], 18), B=fmm_ref.b_matrices(18))
    u = fmm_ref.stage_input(P, f)
    L = P["L"]
    assert W.shape[0] == (1 << (L + 2)) - 4
    for sig in (0, 1):
        w = fmm_ref.upward(P, u, sig)
        for g in range(L):
            t = 2 * np.arange(P["b"][g])[:, None] + np.arange(2)[None, :] + 2     # column nodes
            got = W[(1 << (g + 2)) - 4 + t, sig]                                  # (b, q, k)
            err = np.max(np.abs(got - w[g])) / np.max(np.abs(w[g]))
            assert err <= 1e-14, (sig, g, err)


def test_workspace_export_errors(l2c):
    with l2c.Plan(65536, 0, 64, 16, precision=l2c.L2C_FP32) as p:
        with pytest.raises(l2c.L2CError) as ei:
            p.export(l2c.TABLE_W)
        assert ei.value.code == l2c.L2C_EUNSUPPORTED


# ----------------------------------------------------------------- end to end vs oracle
SIZES = [1, 2, 3, 7, 64, 127, 128, 129, 255, 256, 257, 500, 1000, 1024, 1025, 2049, 4096, 5000, 16384, 40000]


def _single_ok(l2c, n, direction=0, leaf=64, rank=18):
    with l2c.Plan(n, direction, leaf, rank) as p:
        if p.info["levels"] > 0:
            p.set_direct(False)
        return p.info["path"] == l2c.L2C_PATH_SINGLE


@pytest.mark.parametrize("single", [True, False])
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("direction", [0, 1])
def test_parity_sizes(l2c, n, direction, single):
    f = inputs.decaying(n, 1.0, inputs.SEED_BASE + 100 + n)
    if single and not _single_ok(l2c, n, direction):
        pytest.skip("no single-launch form for n=%d (L <= 1)" % n)
    z, info = run(l2c, f, direction, single=single if info_levels(l2c, n) > 0 else None)
    err = oracle.einf(z, oracle.transform(f, direction))
    print("n=%d dir=%d L=%d s=%d path=%d E_inf=%.3e" % (n, direction, info["levels"], info["s"], info["path"], err))
    assert err <= TOL[(direction, 18)]


def info_levels(l2c, n, leaf=64, rank=18):
    with l2c.Plan(n, 0, leaf, rank) as p:
        return p.info["levels"]


@pytest.mark.parametrize("n", [257, 1024, 5000, 40000, 300000])
@pytest.mark.parametrize("direction", [0, 1])
def test_paths_agree(l2c, n, direction):
    """Single-launch and three-launch paths: same tables, same arithmetic up to summation order."""
    f = inputs.decaying(n, 0.5, inputs.SEED_BASE + 400 + n)
    z1, i1 = run(l2c, f, direction, single=True)
    z3, i3 = run(l2c, f, direction, single=False)
    assert i1["path"] == l2c.L2C_PATH_SINGLE and i3["path"] == l2c.L2C_PATH_THREE
    d = np.max(np.abs(z1 - z3)) / np.max(np.abs(z3))
    print("n=%d dir=%d paths differ by %.3e" % (n, direction, d))
    assert d <= 1e-14


@pytest.mark.parametrize("leaf", [4, 8, 16, 32, 40, 128])
@pytest.mark.parametrize("direction", [0, 1])
def test_parity_leaf_sizes(l2c, leaf, direction):
    n = 3001
    f = inputs.decaying(n, 0.5, inputs.SEED_BASE + 200 + leaf)
    z, info = run(l2c, f, direction, leaf=leaf, direct=False)
    assert info["levels"] == 0 or info["path"] in (l2c.L2C_PATH_SINGLE, l2c.L2C_PATH_THREE)
    err = oracle.einf(z, oracle.transform(f, direction))
    print("leaf=%d dir=%d L=%d s=%d E_inf=%.3e" % (leaf, direction, info["levels"], info["s"], err))
    assert err <= TOL[(direction, 18)] * (10 if leaf <= 8 else 1)


@pytest.mark.parametrize("rank", [12, 16, 18, 20, 24])
@pytest.mark.parametrize("direction", [0, 1])
def test_parity_ranks(l2c, rank, direction):
    n = 9000
    f = inputs.decaying(n, 0.5, inputs.SEED_BASE + 300 + rank)
    z, _ = run(l2c, f, direction, rank=rank)
    err = oracle.einf(z, oracle.transform(f, direction))
    print("rank=%d dir=%d E_inf=%.3e" % (rank, direction, err))
    assert err <= TOL[(direction, rank)]


@pytest.mark.parametrize("direct", [None, False])
def test_config1_leg2cheb_1024(l2c, direct):
    """N = 1024, f_j = z_j/(j+1), leaf 64, rank 18; all rows against the oracle, on the
    plan's default path (the direct product) and on Alg. 4."""
    f = inputs.decaying(1024, 1.0, inputs.SEED_BASE + 1)
    z, info = run(l2c, f, 0, direct=direct)
    assert (info["levels"], info["s"], info["n_pad"]) == (3, 32, 1024)
    assert info["path"] == (l2c.L2C_PATH_DIRECT if direct is None else l2c.L2C_PATH_SINGLE)
    assert oracle.einf(z, oracle.leg2cheb(f)) <= 1e-13


def test_table1_sizes_uniform_input(l2c):
    """Table 1 protocol (uniform [0,1] input, r = 0): our E_inf is of the printed order."""
    rows = [ln.split() for ln in open(os.path.join(os.path.dirname(__file__), "golden", "table1_einf.txt"))
            if ln.strip() and not ln.startswith("#")]
    for row in rows[:6]:
        n = int(row[0])
        f = inputs.uniform01(n, 1)
        z1, _ = run(l2c, f, 0, direct=False)    # Alg. 4, the method Table 1 measures
        z2, _ = run(l2c, f, 1, direct=False)
        e1 = oracle.einf(z1, oracle.leg2cheb(f))
        e2 = oracle.einf(z2, oracle.cheb2leg(f))
        print("N=%d L2C %.2e (paper %s)  C2L %.2e (paper %s)" % (n, e1, row[1], e2, row[3]))
        assert e1 <= 4 * float(row[1]) and e2 <= 4 * float(row[3])


@pytest.mark.parametrize("single", [None, True, False])
def test_batch_matches_single_and_is_deterministic(l2c, single):
    """Every path (None: the plan's default, the direct product at this size; True / False:
    the single-launch / three-launch multipole paths) gives bit-identical results on a
    repeat and for each item of a batch executed alone: the reduction order is fixed."""
    import torch
    n, batch = 3000, 5
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 7, batch=batch)
    for direction in (0, 1):
        Z, info = run(l2c, F, direction, single=single)
        Z2, _ = run(l2c, F, direction, single=single)
        assert np.array_equal(Z, Z2)
        for b in range(batch):
            zb, ib = run(l2c, F[b], direction, single=single)
            assert ib["path"] == info["path"]
            assert np.array_equal(Z[b], zb)
            assert oracle.einf(zb, oracle.transform(F[b], direction)) <= TOL[(direction, 18)]
    torch.cuda.synchronize()


def test_single_launch_is_deterministic_at_1e6(l2c):
    """The single-launch kernel at N = 10^6 (256 workgroups exchanging tree nodes through
    the grid-wide buffer): repeated executes of one plan, and a second plan, agree bit for
    bit."""
    import torch
    n = 1_000_000
    x = torch.from_numpy(inputs.decaying(n, 0.5, inputs.SEED_BASE + 2)).cuda()
    with l2c.Plan(n, 0) as p, l2c.Plan(n, 0) as q:
        assert p.info["path"] == l2c.L2C_PATH_SINGLE
        z0 = p.execute(x)
        zs = [p.execute(x) for _ in range(3)] + [q.execute(x)]
        torch.cuda.synchronize()
        assert p.status == 0 and q.status == 0
    for z in zs:
        assert torch.equal(z, z0)


def test_round_trip(l2c):
    n = 20000
    f = inputs.decaying(n, 0.5, inputs.SEED_BASE + 11)
    z, _ = run(l2c, f, 0)
    g, _ = run(l2c, z, 1)
    err = oracle.einf(g, f)
    print("round trip E_inf=%.3e" % err)
    assert err <= 1e-12


def test_edge_cases(l2c):
    import torch
    # n = 1: out = in up to rounding (lambda_0^2 / pi is 1 within an ulp); batch 0 is a no-op
    x = torch.tensor([3.25], dtype=torch.float64, device="cuda")
    for direction in (0, 1):
        with l2c.Plan(1, direction) as p:
            assert abs(p.execute(x).item() - 3.25) <= 2 * np.spacing(3.25)
            p.execute(x[:0].reshape(0, 1))
    # overlapping in/out is rejected
    n = 300
    buf = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    with l2c.Plan(n, 0) as p:
        with pytest.raises(l2c.L2CError) as ei:
            l2c.leg2cheb_execute(p.handle, buf.data_ptr(), buf.data_ptr() + 8 * 10, 1, 0)
        assert ei.value.code == l2c.L2C_EINVAL
        # in-place is overlap too
        with pytest.raises(l2c.L2CError):
            l2c.leg2cheb_execute(p.handle, buf.data_ptr(), buf.data_ptr(), 1, 0)
    # zero input gives zero output
    z, _ = run(l2c, np.zeros(5000), 1, direct=False)
    assert np.all(z == 0.0)
    torch.cuda.synchronize()


def test_single_launch_repeats_batches_and_streams(l2c):
    """Epoch-tagged flags across repeated executes, batches split over several launches
    (n = 40000: 16 units per item, 16 items per launch), and two plans on two streams."""
    import torch
    n, batch = 40000, 40
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 17, batch=batch)
    x = torch.from_numpy(F).cuda()
    with l2c.Plan(n, 0, max_batch=1) as p:
        assert p.info["path"] == l2c.L2C_PATH_SINGLE
        z0 = p.execute(x).cpu().numpy()
        for _ in range(3):
            assert np.array_equal(p.execute(x).cpu().numpy(), z0)
        assert p.status == 0
    for b in (0, 15, 16, 39):
        assert oracle.einf(z0[b], oracle.leg2cheb(F[b])) <= 1e-13
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    f1, f2 = x[0].clone(), x[1].clone()
    with l2c.Plan(n, 0) as pa, l2c.Plan(n, 1) as pb:
        outs = []
        for _ in range(4):
            with torch.cuda.stream(s1):
                outs.append(("a", pa.execute(f1, stream=s1)))
            with torch.cuda.stream(s2):
                outs.append(("b", pb.execute(f2, stream=s2)))
        torch.cuda.synchronize()
        assert pa.status == 0 and pb.status == 0
        ra, rb = oracle.leg2cheb(F[0]), oracle.cheb2leg(F[1])
        for tag, z in outs:
            ref = ra if tag == "a" else rb
            assert oracle.einf(z.cpu().numpy(), ref) <= TOL[(0 if tag == "a" else 1, 18)]


def test_workspace_grows_with_batch(l2c):
    import torch
    n = 2000
    with l2c.Plan(n, 0, max_batch=1) as p:
        F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 13, batch=9)
        z = p.execute(torch.from_numpy(F).cuda())
        torch.cuda.synchronize()
        assert p.info["workspace_bytes"] > 0
        for b in (0, 8):
            assert oracle.einf(z[b].cpu().numpy(), oracle.leg2cheb(F[b])) <= 1e-13


# ----------------------------------------------------------------- configuration 2: N = 10^6
N_MILLION = 10 ** 6
CHUNKS = 4


def _chunk_rows(n, k, chunks=CHUNKS):
    """Rows of chunk k: equal shares of the oracle's work (row i costs (n - i)/2 terms)."""
    edge = [int(round(n * (1.0 - np.sqrt(1.0 - c / chunks)))) for c in range(chunks + 1)]
    edge[-1] = n
    return np.arange(edge[k], edge[k + 1], dtype=np.int64)


@pytest.fixture(scope="module")
def million(l2c):
    """Configuration 2: f_j = z_j/sqrt(j+1), N = 10^6, leaf 64, rank 18; the GPU outputs of
    both directions on both Alg. 4 paths, computed once."""
    f = inputs.decaying(N_MILLION, 0.5, inputs.SEED_BASE + 2)
    out = {"f": f}
    for direction in (0, 1):
        for single in (True, False):
            z, info = run(l2c, f, direction, single=single)
            assert (info["levels"], info["s"], info["n_pad"]) == (13, 31, 1015808)
            out[(direction, single)] = z
    return out


@pytest.mark.parametrize("direction,chunk", [(d, c) for d in (0, 1) for c in range(CHUNKS)])
def test_config2_million_every_row(l2c, million, direction, chunk):
    """N = 10^6, every output row against the direct oracle, on both Alg. 4 paths (each
    test one chunk of rows, equal shares of the oracle's O(N^2) work; the last chunk of a
    direction checks E_inf over the whole output).  Each chunk's largest deviation is held
    to the bound relative to the largest |z*| seen so far."""
    f = million["f"]
    rows = _chunk_rows(N_MILLION, chunk)
    t0 = time.time()
    ref = oracle.transform(f, direction, rows)
    scale = max(million.get(("scale", direction), 0.0), float(np.max(np.abs(ref))))
    million[("scale", direction)] = scale
    for single in (True, False):
        dz = float(np.max(np.abs(million[(direction, single)][rows] - ref)))
        key = ("dz", direction, single)
        million[key] = max(million.get(key, 0.0), dz)
        print("N=1e6 dir=%d single=%s rows [%d, %d): max|dz| / max|z*| %.3e (oracle %.1f s)"
              % (direction, single, rows[0], rows[-1] + 1, dz / scale, time.time() - t0), flush=True)
        assert dz <= TOL[(direction, 18)] * scale
    if chunk == CHUNKS - 1:
        for single in (True, False):
            print("N=1e6 dir=%d single=%s E_inf over all rows %.3e"
                  % (direction, single, million[("dz", direction, single)] / scale), flush=True)


def test_config2_invariants_and_round_trip(l2c, million):
    """The full outputs against the x = +-1 identities (sum_i z_i = sum_j f_j and the
    alternating sums: T_i(+-1) = L_j(+-1) = (+-1)^i), and the round trip leg2cheb ->
    cheb2leg against the input."""
    import torch
    f = million["f"]
    n = f.size
    sgn = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    for direction in (0, 1):
        z = million[(direction, True)]
        for w in (np.ones(n), sgn):
            lhs, rhs = float(np.dot(w, z)), float(np.dot(w, f))
            assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(f)), (direction, lhs, rhs)
    back, _ = run(l2c, million[(0, True)], 1)
    err = oracle.einf(back, f)
    print("N=1e6 round trip E_inf %.3e" % err, flush=True)
    assert err <= 1e-13
    torch.cuda.synchronize()


# ----------------------------------------------------------------- ragged batches
def test_ragged_batch_small(l2c):
    """Mixed lengths (direct-only, one and several levels, equal L with different n) and
    mixed directions in one batch plan: every output against the oracle, repeatable bit for
    bit, and within the tolerance of the same transform planned alone (a ragged group uses
    the full half-leaf s = 32, a single plan the smallest s that covers n)."""
    import torch
    sizes = [1, 2, 5, 63, 64, 65, 127, 128, 129, 300, 1000, 1024, 2990, 3000, 3007, 4096, 9000, 9001,
             16384, 20000, 511, 3001]
    dirs = [i % 2 for i in range(len(sizes))]
    dirs[12] = dirs[13] = dirs[14] = 0
    xs = [torch.from_numpy(inputs.decaying(n, 1.0, inputs.SEED_BASE + 100 + i)).cuda() for i, n in enumerate(sizes)]
    with l2c.BatchPlan(sizes, dirs, leaf_size=64, rank=18) as bp:
        info = bp.info
        assert 1 <= info["groups"] < len(sizes) and info["table_bytes"] > 0
        # groups are (levels, direction): n = 1..64 direct, then L = 1..7
        assert info["groups"] == len({(l2c.Plan(n, 0).info["levels"], d) for n, d in zip(sizes, dirs)})
        zs = bp.execute(xs)
        zs2 = bp.execute(xs)
        torch.cuda.synchronize()
    for i, (n, d) in enumerate(zip(sizes, dirs)):
        z = zs[i].cpu().numpy()
        assert np.array_equal(z, zs2[i].cpu().numpy())
        f = xs[i].cpu().numpy()
        err = oracle.einf(z, oracle.transform(f, d))
        assert err <= TOL[(d, 18)], (n, d, err)
        alone, _ = run(l2c, f, d)
        assert oracle.einf(z, alone) <= 2 * TOL[(d, 18)], (n, d)


def test_ragged_batch_errors(l2c):
    import torch
    with pytest.raises(l2c.L2CError) as ei:
        l2c.leg2cheb_batch_plan([100, 0], [0, 0])
    assert ei.value.code == l2c.L2C_EINVAL
    with pytest.raises(l2c.L2CError) as ei:
        l2c.leg2cheb_batch_plan([100], [2])
    assert ei.value.code == l2c.L2C_EINVAL
    with pytest.raises(l2c.L2CError) as ei:
        l2c.leg2cheb_batch_plan([100], [0], precision=l2c.L2C_BF16X2, tuning=[(1 << 62, 64, 18)])
    assert ei.value.code == l2c.L2C_EUNSUPPORTED
    buf = torch.zeros(1000, dtype=torch.float64, device="cuda")
    p0 = buf.data_ptr()
    with l2c.BatchPlan([300, 300], [0, 1]) as bp:
        # an output overlapping another output, and an output overlapping an input
        for ins, outs in (([p0, p0], [p0 + 8 * 400, p0 + 8 * 500]),
                          ([p0, p0 + 8 * 300], [p0 + 8 * 600, p0 + 8 * 100])):
            with pytest.raises(l2c.L2CError) as ei:
                l2c.leg2cheb_batch_execute(bp.handle, ins, outs)
            assert ei.value.code == l2c.L2C_EINVAL
        # shared input, disjoint outputs: allowed
        l2c.leg2cheb_batch_execute(bp.handle, [p0, p0], [p0 + 8 * 300, p0 + 8 * 600])
        torch.cuda.synchronize()


@pytest.fixture(scope="module")
def ragged():
    """Configuration 4: 2048 transforms, n log-uniform in [128, 262144], directions 50/50,
    f_j = z_j/(j+1); the oracle of every transform with n <= 16384 and of 32 seeded longer
    ones (computed once)."""
    sizes, dirs = inputs.ragged_sizes(2048, inputs.SEED_BASE + 4)
    rng = np.random.default_rng(inputs.SEED_BASE + 5)
    total = int(sizes.sum())
    flat = rng.standard_normal(total)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    for i, n in enumerate(sizes):
        flat[offs[i]:offs[i + 1]] /= np.arange(1, n + 1, dtype=np.float64)
    long_ = np.flatnonzero(sizes > 16384)
    pick = set(np.flatnonzero(sizes <= 16384).tolist()) | set(rng.choice(long_, 32, replace=False).tolist())
    t0 = time.time()
    refs = {i: oracle.transform(flat[offs[i]:offs[i + 1]], int(dirs[i])) for i in sorted(pick)}
    print("ragged oracle: %d transforms in %.1f s" % (len(refs), time.time() - t0), flush=True)
    return {"sizes": sizes, "dirs": dirs, "flat": flat, "offs": offs, "refs": refs}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config4_ragged_2048(l2c, ragged, precision):
    """The ragged batch in one BatchPlan with the library's autotuned leaf size and rank per
    size bucket: every transform with n <= 16384 and 32 longer ones against the oracle on all
    rows, per direction; every full output against the x = +-1 identities."""
    import torch
    sizes, dirs, flat, offs = ragged["sizes"], ragged["dirs"], ragged["flat"], ragged["offs"]
    prec = l2c.L2C_FP64 if precision == "fp64" else l2c.L2C_FP32
    x = torch.from_numpy(flat).cuda()
    y = torch.empty_like(x)
    xs = [x[offs[i]:offs[i + 1]] for i in range(len(sizes))]
    ys = [y[offs[i]:offs[i + 1]] for i in range(len(sizes))]
    # leaf size and rank per size bucket from the library's autotuned table (tuning NULL)
    with l2c.BatchPlan(sizes.tolist(), dirs.tolist(), precision=prec) as bp:
        groups = bp.info["groups"]
        bp.execute(xs, ys)
        torch.cuda.synchronize()
    yh = y.cpu().numpy()
    worst = {0: 0.0, 1: 0.0}
    for i, ref in ragged["refs"].items():
        err = oracle.einf(yh[offs[i]:offs[i + 1]], ref)
        worst[int(dirs[i])] = max(worst[int(dirs[i])], err)
    sum_tol = 1e-11 if precision == "fp64" else 1e-4
    for i, (n, d) in enumerate(zip(sizes.tolist(), dirs.tolist())):
        f, z = flat[offs[i]:offs[i + 1]], yh[offs[i]:offs[i + 1]]
        sgn = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
        for w in (np.ones(n), sgn):
            assert abs(float(np.dot(w, z)) - float(np.dot(w, f))) <= sum_tol * np.sum(np.abs(f)), (i, n, d)
    print("ragged 2048 %s (%d groups, %d transforms against the oracle): E_inf leg2cheb %.2e  cheb2leg %.2e"
          % (precision, groups, len(ragged["refs"]), worst[0], worst[1]), flush=True)
    if precision == "fp64":
        assert worst[0] <= TOL[(0, 18)] and worst[1] <= TOL[(1, 18)]
    else:
        assert max(worst.values()) <= TOL32


# ----------------------------------------------------------------- dense path (short transforms)
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("n", [129, 300, 999, 1000, 1024, 4096])
def test_dense_batches_of_short_transforms(l2c, n, direction):
    """FP64 plans for n <= 4096 made for batches of 64 or more apply Alg. 1 as dense
    per-parity products on the matrix cores: every output against the oracle (the direct
    product is exact up to rounding), a ragged tail of transforms past a 64-transform tile,
    and the plain (batch 1) execute of the same plan."""
    import torch
    B = 70
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 60 + n % 89, batch=B)
    x = torch.from_numpy(F).cuda()
    with l2c.Plan(n, direction, 64, 18, max_batch=B) as p:
        assert p.info["path"] == l2c.L2C_PATH_DENSE
        Z = p.execute(x).cpu().numpy()
        z1 = p.execute(x[B - 1]).cpu().numpy()
        torch.cuda.synchronize()
    worst = max(oracle.einf(Z[b], oracle.transform(F[b], direction)) for b in range(B))
    print("dense n=%d dir=%d E_inf=%.2e" % (n, direction, worst))
    assert worst <= 1e-14
    assert np.array_equal(z1, Z[B - 1])


@pytest.mark.parametrize("n", [129, 255, 256, 257, 1000, 1024, 1025, 2049, 4096, 5000, 8191, 8192])
@pytest.mark.parametrize("direction", [0, 1])
def test_direct_short_transforms(l2c, n, direction):
    """FP64 plans for n <= 8192 (L >= 1) and batch n^2 <= W (2^27 up to n = 4096, 2^26
    above) apply Alg. 1 row by row:
    every output of a batch of up to three against the oracle (the direct product is exact
    up to rounding), the batch-1 execute of the same plan bit for bit, agreement with the
    multipole path of the same plan to the multipole tolerance, and a batch past the work
    bound that runs the multipole path."""
    import torch
    W = (1 << 27) if n <= 4096 else (1 << 26)
    B = max(1, min(3, W // (n * n)))
    F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 70 + n % 97, batch=B)
    x = torch.from_numpy(F).cuda()
    with l2c.Plan(n, direction, 64, 18, max_batch=B) as p:
        assert p.info["levels"] > 0 and p.info["path"] == l2c.L2C_PATH_DIRECT
        Z = p.execute(x).cpu().numpy()
        z1 = p.execute(x[B - 1]).cpu().numpy()
        # a batch past the work bound runs Alg. 4: same result to the multipole tolerance
        nb = W // (n * n) + 1
        xb = x[torch.arange(nb) % B].contiguous()
        Zb = p.execute(xb).cpu().numpy()
        p.set_direct(False)
        assert p.info["path"] in (l2c.L2C_PATH_SINGLE, l2c.L2C_PATH_THREE)
        Zm = p.execute(x).cpu().numpy()
        p.set_direct(True)
        assert p.info["path"] == l2c.L2C_PATH_DIRECT
        torch.cuda.synchronize()
    worst = max(oracle.einf(Z[b], oracle.transform(F[b], direction)) for b in range(B))
    dm = max(oracle.einf(Zm[b], Z[b]) for b in range(B))
    assert max(oracle.einf(Zb[b], Zm[b]) for b in range(B)) <= 1e-15
    print("direct n=%d dir=%d E_inf=%.2e, multipole differs by %.2e" % (n, direction, worst, dm))
    # both sides sum the same FP64 terms in different orders; cheb2leg rows cancel more
    # (their terms grow like (2i+1) j), hence the looser bound
    assert worst <= (1e-14 if direction == 0 else 5e-14)
    assert np.array_equal(z1, Z[B - 1])
    assert dm <= TOL[(direction, 18)]


def test_direct_option_errors(l2c):
    """L2C_OPT_DIRECT = 1 only on short FP64 plans with L >= 1."""
    with l2c.Plan(20000, 0) as p:
        assert p.info["path"] != l2c.L2C_PATH_DIRECT
        p.set_direct(False)
        with pytest.raises(l2c.L2CError) as ei:
            p.set_direct(True)
        assert ei.value.code == l2c.L2C_EUNSUPPORTED
        with pytest.raises(l2c.L2CError) as ei:
            l2c.leg2cheb_plan_set_option(p.handle, l2c.L2C_OPT_DIRECT, 2)
        assert ei.value.code == l2c.L2C_EINVAL
    with l2c.Plan(1024, 0, 64, 16, precision=l2c.L2C_FP32) as p:
        with pytest.raises(l2c.L2CError):
            p.set_direct(True)


# ----------------------------------------------------------------- ragged batches in graphs
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ragged_batch_graph_capture_and_replay(l2c, precision):
    """A ragged batch captured by the caller into a graph (torch.cuda.graph) and replayed
    three times, with eager executes of the same batch (other outputs) and synchronizations
    between the replays: every replay equals the eager execute bit for bit (the same
    kernels), and the eager executes (replays of the batch's own internal graph) stay
    right as well."""
    import torch
    sizes, dirs = inputs.ragged_sizes(96, inputs.SEED_BASE + 44)
    sizes = np.concatenate([sizes, [1, 5, 100, 129, 1000, 4096]])
    dirs = np.concatenate([dirs, [0, 1, 0, 1, 0, 1]])
    offs = np.concatenate([[0], np.cumsum(sizes)])
    rng = np.random.default_rng(inputs.SEED_BASE + 45)
    flat = rng.standard_normal(int(offs[-1]))
    for i, n in enumerate(sizes):
        flat[offs[i]:offs[i + 1]] /= np.arange(1, n + 1, dtype=np.float64)
    prec, rank = (l2c.L2C_FP64, 18) if precision == "fp64" else (l2c.L2C_FP32, 16)
    x = torch.from_numpy(flat).cuda()
    y_eager, y_graph, y_other = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
    ptrs = lambda t: [t.data_ptr() + 8 * int(o) for o in offs[:-1]]
    with l2c.BatchPlan(sizes.tolist(), dirs.tolist(), rank=rank, precision=prec) as bp:
        bp.execute_ptrs(ptrs(x), ptrs(y_eager))
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            bp.execute_ptrs(ptrs(x), ptrs(y_graph))
        for rep in range(3):
            y_graph.fill_(float("nan"))
            y_other.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            bp.execute_ptrs(ptrs(x), ptrs(y_other))        # eager work between replays
            torch.cuda.synchronize()
            assert torch.equal(y_graph, y_eager), rep
            assert torch.equal(y_other, y_eager), rep
        del g
    yh = y_eager.cpu().numpy()
    tol = TOL[(0, 18)] if precision == "fp64" else TOL32
    for i in range(0, len(sizes), 7):
        d = int(dirs[i])
        err = oracle.einf(yh[offs[i]:offs[i + 1]], oracle.transform(flat[offs[i]:offs[i + 1]], d))
        assert err <= (TOL[(d, 18)] if precision == "fp64" else tol), (i, err)


def test_plan_cache_shares_and_releases(l2c):
    """Two cached requests with the same arguments share one plan; other arguments make
    another; each close releases one reference and the last frees the plan; results equal
    an uncached plan's."""
    import torch
    n = 5000
    x = torch.from_numpy(inputs.decaying(n, 1.0, inputs.SEED_BASE + 700)).cuda()
    p0 = l2c.leg2cheb_plan_cache_size()
    a = l2c.Plan(n, 0, cached=True)
    b = l2c.Plan(n, 0, cached=True)
    c = l2c.Plan(n, 1, cached=True)
    assert a.handle == b.handle and c.handle != a.handle
    assert l2c.leg2cheb_plan_cache_size() == (p0[0] + 2, p0[1] + 3)
    with l2c.Plan(n, 0) as u:
        assert torch.equal(a.execute(x), u.execute(x))
    a.close()
    assert torch.equal(b.execute(x), b.execute(x))     # b still holds the shared plan
    b.close()
    c.close()
    assert l2c.leg2cheb_plan_cache_size() == p0
