"""leg2cheb_execute_noalloc (the entry point for callers that cannot allocate) against
leg2cheb_execute through the C ABI.

The no-allocation entry point runs the three-launch path of Alg. 4 with its workspace in
the library's fixed device array; its output must equal leg2cheb_execute's on the same
path bit for bit, on two calls in a row (the second with a smaller input), and the call
must allocate nothing: with the allocation-failure hook armed to fail the next allocation,
it still succeeds and the hook's countdown is untouched.
"""
import numpy as np
import pytest

import oracle
from paper_2411_00033_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def l2c():
    import torch
    import paper_2411_00033_amd as mod
    assert torch.cuda.is_available()
    mod._lib.load()
    yield mod
    mod.leg2cheb_debug_alloc_hook(0)


def _noalloc(l2c, plan, x, y, batch):
    """One leg2cheb_execute_noalloc call with the allocation hook armed to fail the next
    allocation: the call must succeed without reaching it."""
    import torch
    l2c.leg2cheb_debug_alloc_hook(1)
    try:
        l2c.leg2cheb_execute_noalloc(plan.handle, x.data_ptr(), y.data_ptr(), batch,
                                     torch.cuda.current_stream().cuda_stream)
    finally:
        pending, _ = l2c.leg2cheb_debug_alloc_hook(0)
    assert pending == 1, "leg2cheb_execute_noalloc reached an allocation"


@pytest.mark.parametrize("direction", [0, 1])
def test_noalloc_matches_execute_two_calls(l2c, direction):
    import torch
    cases = [(300000, 3), (40000, 2)]            # the second call has the smaller input
    for call, (n, batch) in enumerate(cases):
        print("noalloc call %d: n=%d batch=%d direction=%d" % (call, n, batch, direction), flush=True)
        F = inputs.decaying(n, 0.5, inputs.SEED_BASE + 120 + call, batch=batch)
        x = torch.from_numpy(F).cuda()
        with l2c.Plan(n, direction, 64, 18, max_batch=batch) as p:
            p.set_single_launch(False)
            y_ref = p.execute(x)
            y = torch.full_like(x, float("nan"))
            _noalloc(l2c, p, x, y, batch)
            torch.cuda.synchronize()
            assert torch.equal(y, y_ref)
        # the first and last items against the oracle on sampled rows (|z| peaks at the
        # first rows for these decaying inputs)
        zh = y.cpu().numpy()
        rows = np.unique(np.concatenate([np.arange(0, 256), np.arange(n - 64, n), np.arange(0, n, 997)]))
        for b in (0, batch - 1):
            ref = oracle.transform(F[b], direction, rows)
            assert np.max(np.abs(zh[b][rows] - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_noalloc_short_and_dense_plans(l2c):
    """Plans on the direct and dense paths run their own kernels (no workspace)."""
    import torch
    for n, batch in ((1000, 2), (1000, 70), (100, 3)):
        F = inputs.decaying(n, 1.0, inputs.SEED_BASE + 130 + batch, batch=batch)
        x = torch.from_numpy(F).cuda()
        with l2c.Plan(n, 0, 64, 18, max_batch=batch) as p:
            y_ref = p.execute(x)
            y = torch.full_like(x, float("nan"))
            _noalloc(l2c, p, x, y, batch)
            torch.cuda.synchronize()
            assert torch.equal(y, y_ref)


def test_noalloc_limits(l2c):
    """A batch whose workspace exceeds the fixed array is rejected; batched forms are not
    served."""
    import torch
    n = 1_000_000
    x = torch.zeros((8, n), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with l2c.Plan(n, 0, 64, 18) as p:
        with pytest.raises(l2c.L2CError) as ei:
            l2c.leg2cheb_execute_noalloc(p.handle, x.data_ptr(), y.data_ptr(), 8, 0)
        assert ei.value.code == l2c.L2C_EINVAL
        l2c.leg2cheb_execute_noalloc(p.handle, x.data_ptr(), y.data_ptr(), 7, 0)
        torch.cuda.synchronize()
        assert torch.count_nonzero(y[:7]).item() == 0
    with l2c.Plan(65536, 0, 64, 16, precision=l2c.L2C_FP32) as p:
        with pytest.raises(l2c.L2CError) as ei:
            l2c.leg2cheb_execute_noalloc(p.handle, x.data_ptr(), y.data_ptr(), 1, 0)
        assert ei.value.code == l2c.L2C_EUNSUPPORTED
