"""pf_solve_batch_noalloc (the entry point for callers that cannot allocate) against
pf_solve_batch through the C ABI: identical results (same kernels, same configuration)
on two calls in a row on one device, the second with fewer instances, so the fixed
scratch keeps the first call's contents when the second runs; a batch whose workspace
exceeds the fixed scratch is rejected with an error."""
import numpy as np
import pytest

import gridgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2101_02270_amd as pf  # noqa: E402

DEV = "cuda"


def _result(B, n):
    return pf.Result(v=torch.empty((B, n, 2), dtype=torch.float64, device=DEV),
                     iters=torch.empty(B, dtype=torch.int32, device=DEV),
                     converged=torch.empty(B, dtype=torch.uint8, device=DEV),
                     status=torch.empty(B, dtype=torch.int8, device=DEV))


def _same(a, b):
    torch.cuda.synchronize()
    assert torch.equal(a.iters, b.iters)
    assert torch.equal(a.converged, b.converged)
    assert torch.equal(a.status, b.status)
    assert torch.equal(a.v, b.v)      # bitwise: same kernels, same configuration


@pytest.mark.parametrize("key,counts,prec", [("c1", (200, 77), pf.PF_FP64), ("c1", (200, 77), pf.PF_FP32_LU),
                                             ("c0", (64, 5), pf.PF_FP64)])
def test_noalloc_matches_workspace_entry_point(key, counts, prec):
    (g, yb, sc), = gg.workload(key, count=counts[0])
    plan = pf.Plan.from_ybus(yb, g.bus_type)
    y = torch.from_numpy(yb.val).to(DEV)
    for B in counts:                      # second call smaller than the first
        s = torch.from_numpy(np.ascontiguousarray(sc.sbus[:B])).to(DEV)
        v = torch.from_numpy(np.ascontiguousarray(sc.v0[:B])).to(DEV)
        ref = pf.solve_batch(plan, y, s, v, precision=prec)
        got = pf.solve_batch_noalloc(plan, y, s, v, _result(B, g.n), precision=prec)
        _same(got, ref)
        assert bool(got.converged.bool().any())


def test_noalloc_rejects_batches_beyond_the_scratch():
    (g, yb, sc), = gg.workload("c1", count=8)
    plan = pf.Plan.from_ybus(yb, g.bus_type)
    B = 4096                              # about 1.2 GB of workspace for this grid
    assert plan.workspace_bytes(B) > 128 << 20
    y = torch.from_numpy(yb.val).to(DEV)
    s = torch.zeros((B, g.n, 2), dtype=torch.float64, device=DEV)
    v = torch.ones((B, g.n, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(pf.PfError, match="scratch"):
        pf.solve_batch_noalloc(plan, y, s, v, _result(B, g.n))
