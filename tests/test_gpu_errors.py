"""Error paths forced from the host on the GPU: allocation failures.

Every device and pinned host allocation of the library passes one process-wide countdown
(leg2cheb_debug_alloc_hook).  For each plan kind below, the k-th allocation is failed for
k = 1, 2, ... until a plan is made with the hook not reached.  Each failed call must return
L2C_ENOMEM, leave the handle NULL and hold no allocation afterwards.  The last, successful
plan must still give the result of a plan made without the hook.  No kernel is made to fail
and nothing runs out of memory on the device: the failures are decided on the host before
the allocation call.
"""
import ctypes

import numpy as np
import pytest

from paper_2411_00033_amd import inputs

pytestmark = pytest.mark.gpu

ENOMEM = -2


@pytest.fixture(scope="module")
def l2c():
    import torch
    import paper_2411_00033_amd as mod
    assert torch.cuda.is_available()
    mod._lib.load()
    yield mod
    mod.leg2cheb_debug_alloc_hook(0)


def fail_each(l2c, make):
    """Fail allocation k = 1, 2, ... of make() until it succeeds.  Returns the handle of
    the successful call and the number of allocations the call makes."""
    _, live0 = l2c.leg2cheb_debug_alloc_hook(-1)
    for k in range(1, 200):
        l2c.leg2cheb_debug_alloc_hook(k)
        rc, h = make()
        pending, live = l2c.leg2cheb_debug_alloc_hook(0)
        if rc == 0:
            assert pending > 0, "the call succeeded although its allocation %d failed" % k
            assert h.value is not None
            return h, k - 1
        print("fail allocation %d: rc %d, live %d" % (k, rc, live), flush=True)
        assert rc == ENOMEM, (k, rc)
        assert pending == 0 and h.value is None
        assert live == live0, "allocation %d failed and %d allocations leaked" % (k, live - live0)
    raise AssertionError("the call kept allocating")


def plan_maker(l2c, n, direction, precision, max_batch, rank=18):
    L = l2c._lib.load()

    def make():
        h = ctypes.c_void_p(1)
        rc = L.leg2cheb_plan_ex(ctypes.byref(h), n, direction, 64, rank, precision, max_batch, None)
        return rc, h
    return make


def batch_maker(l2c, ns, dirs, precision, rank=18):
    L = l2c._lib.load()
    na = (ctypes.c_int64 * len(ns))(*ns)
    da = (ctypes.c_int * len(dirs))(*dirs)

    t, keep = l2c._lib._tuning([(1 << 62, 64, rank)])

    def make():
        h = ctypes.c_void_p(1)
        rc = L.leg2cheb_batch_plan(ctypes.byref(h), len(ns), na, da, precision, ctypes.byref(t), None)
        return rc, h
    make.keep = (t, keep)
    return make


@pytest.mark.parametrize("n,direction,precision,max_batch,rank,path", [
    (1_000_000, 0, 0, 1, 18, "single"),     # single-launch tables, exchange buffer, workspace
    (100_000, 1, 0, 4, 18, "single"),
    (1000, 1, 0, 70, 18, "dense"),          # dense coefficient matrices
    (65536, 0, 1, 32, 16, "batched"),       # batched FP32 tables and workspace
    (65536, 1, 2, 32, 16, "batched"),       # BF16X2
    (100, 0, 0, 1, 18, "direct"),           # L = 0: no allocation
])
def test_plan_allocation_failures(l2c, n, direction, precision, max_batch, rank, path):
    import torch
    print("case n=%d dir=%d precision=%d batch=%d" % (n, direction, precision, max_batch), flush=True)
    h, count = fail_each(l2c, plan_maker(l2c, n, direction, precision, max_batch, rank))
    assert count >= (0 if path == "direct" else 3)
    # the plan made after the failures gives the same result as one made without the hook
    x = torch.from_numpy(inputs.decaying(n, 0.5, seed=11)).cuda()
    y = torch.empty_like(x)
    l2c.leg2cheb_execute(h.value, x.data_ptr(), y.data_ptr(), 1, 0)
    with l2c.Plan(n, direction, 64, rank, precision=precision, max_batch=max_batch) as p:
        z = p.execute(x)
    torch.cuda.synchronize()
    l2c.leg2cheb_destroy(h.value)
    assert torch.equal(y, z)
    _, live = l2c.leg2cheb_debug_alloc_hook(-1)
    print("allocations per plan: %d, held after destroy: %d" % (count, live), flush=True)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_allocation_failures(l2c, precision):
    import torch
    rank = 18 if precision == 0 else 16
    ns = [300, 5000, 70000, 100, 5000, 1000]
    dirs = [0, 1, 0, 1, 0, 1]
    print("case batch precision=%d" % precision, flush=True)
    _, live0 = l2c.leg2cheb_debug_alloc_hook(-1)
    h, count = fail_each(l2c, batch_maker(l2c, ns, dirs, precision, rank))
    assert count >= 4
    xs = [torch.from_numpy(inputs.decaying(n, 0.5, seed=20 + i)).cuda() for i, n in enumerate(ns)]
    ys = [torch.empty_like(x) for x in xs]
    zs = [torch.empty_like(x) for x in xs]
    l2c.leg2cheb_batch_execute(h.value, [x.data_ptr() for x in xs], [y.data_ptr() for y in ys], 0)
    with l2c.BatchPlan(ns, dirs, 64, rank, precision) as b:
        b.execute(xs, zs)
    torch.cuda.synchronize()
    l2c.leg2cheb_batch_destroy(h.value)
    for y, z in zip(ys, zs):
        assert torch.equal(y, z)
    _, live = l2c.leg2cheb_debug_alloc_hook(-1)
    assert live == live0


def test_execute_and_export_allocation_failures(l2c):
    """Allocations made after planning: the FP64 workspace grows on an execute with a
    larger batch than planned, and plan_export stages Ahat in device memory.  A failed
    allocation returns L2C_ENOMEM; the plan stays usable and later calls succeed."""
    import torch
    n, B = 100_000, 3
    x = torch.from_numpy(np.stack([inputs.decaying(n, 0.5, seed=30 + b) for b in range(B)])).cuda()
    with l2c.Plan(n, 0) as p:
        p.set_single_launch(False)   # three-launch path: workspace per item
        ref = torch.stack([p.execute(x[b]) for b in range(B)])
        y = torch.empty_like(x)
        _, live0 = l2c.leg2cheb_debug_alloc_hook(1)
        with pytest.raises(l2c.L2CError) as ei:
            l2c.leg2cheb_execute(p.handle, x.data_ptr(), y.data_ptr(), B, 0)
        assert ei.value.code == l2c.L2C_ENOMEM
        pending, live = l2c.leg2cheb_debug_alloc_hook(0)
        assert pending == 0 and live == live0 - 1      # the old workspace was released
        l2c.leg2cheb_execute(p.handle, x.data_ptr(), y.data_ptr(), B, 0)
        torch.cuda.synchronize()
        assert (y - ref).abs().max().item() <= 1e-14 * ref.abs().max().item()
        need = l2c.leg2cheb_plan_export(p.handle, l2c.TABLE_AHAT)
        buf = np.empty(need // 8)
        l2c.leg2cheb_debug_alloc_hook(1)
        with pytest.raises(l2c.L2CError) as ei:
            l2c.leg2cheb_plan_export(p.handle, l2c.TABLE_AHAT, buf.ctypes.data, need)
        assert ei.value.code == l2c.L2C_ENOMEM
        pending, live = l2c.leg2cheb_debug_alloc_hook(0)
        assert pending == 0 and live == live0
        l2c.leg2cheb_plan_export(p.handle, l2c.TABLE_AHAT, buf.ctypes.data, need)
        assert np.array_equal(buf, p.export(l2c.TABLE_AHAT).ravel())


def test_single_launch_wait_timeout_is_reported(l2c):
    """A single-launch wait that gives up is reported, forced from the host: with the
    exchange timeout at 0 every wait for another workgroup gives up after its first poll
    (every kernel still ends), the plan's status shows L2C_STATUS_EXCHANGE, the next
    execute returns L2C_EHIP without running, and once the status has been read (which
    clears it) the plan with the default timeout gives the oracle's result again."""
    import torch
    import oracle
    n = 40000
    f = inputs.decaying(n, 1.0, inputs.SEED_BASE + 90)
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    with l2c.Plan(n, 0) as p:
        assert p.info["path"] == l2c.L2C_PATH_SINGLE
        with pytest.raises(l2c.L2CError) as ei:
            p.set_exchange_timeout_us(-1)
        assert ei.value.code == l2c.L2C_EINVAL
        p.set_exchange_timeout_us(0)
        p.execute(x, y)
        torch.cuda.synchronize()
        with pytest.raises(l2c.L2CError) as ei:
            p.execute(x, y)
        assert ei.value.code == l2c.L2C_EHIP
        st = p.status
        print("forced give-up: status %#x" % st, flush=True)
        assert st & l2c.L2C_STATUS_EXCHANGE
        assert p.status == 0                    # read and cleared
        p.set_exchange_timeout_us(1000000)
        z = p.execute(x, y)
        torch.cuda.synchronize()
        assert p.status == 0
    assert oracle.einf(z.cpu().numpy(), oracle.leg2cheb(f)) <= 1e-13


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_reused_on_another_stream(l2c, precision):
    """A ragged batch executed on one stream and immediately again, with other pointers, on
    a second stream: the second call waits for the first, so both outputs are right."""
    import torch
    import oracle
    rank = 18 if precision == 0 else 16
    ns = [300, 5000, 70000, 1000, 20000]
    dirs = [0, 1, 0, 1, 1]
    xs = [torch.from_numpy(inputs.decaying(n, 1.0, inputs.SEED_BASE + 95 + i)).cuda() for i, n in enumerate(ns)]
    xs2 = [(2.0 * x).flip(0).contiguous() for x in xs]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with l2c.BatchPlan(ns, dirs, 64, rank, precision) as b:
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            y1 = b.execute(xs, stream=s1)
        with torch.cuda.stream(s2):
            y2 = b.execute(xs2, stream=s2)
        torch.cuda.synchronize()
    tol = 1e-13 if precision == 0 else 2.5e-6
    for i, d in enumerate(dirs):
        for xx, yy in ((xs, y1), (xs2, y2)):
            err = oracle.einf(yy[i].cpu().numpy(), oracle.transform(xx[i].cpu().numpy(), d))
            assert err <= tol, (i, err)
