"""The batched CPU engine (pf_cpu_solve_batch: Alg. 2 over mini-batches of 8 instances in
SIMD lanes, worker threads over mini-batches) against the FP64 oracle, on the CPU.

Bars: the FP64 full-solve bar of the GPU path (identical convergence flags and iteration
counts, |V| and angle within 1e-6, borderline instances only need a valid result); results
independent of the thread count (bit-identical); a non-finite instance does not affect the
other lanes of its mini-batch; max_iter 0 / 1 semantics as the oracle's.
"""
import numpy as np
import pytest

import gridgen as gg
import oracle
import paper_2101_02270_amd as pf


def compare(osys, ro, rc, sbus, tol=1e-8):
    k = ro.iters.astype(np.int64)
    B = k.shape[0]
    last = ro.hist[np.arange(B), k]
    prev = ro.hist[np.arange(B), np.maximum(k - 1, 0)]
    band = lambda x: np.isfinite(x) & (x >= 0.5 * tol) & (x <= 2 * tol)
    full = ~(band(last) | band(prev))
    assert np.array_equal(rc.converged[full], ro.converged[full])
    both = full & ro.converged
    assert np.array_equal(rc.iters[both], ro.iters[both])
    if both.any():
        assert np.abs(rc.v[both] - ro.v[both]).max() <= 1e-6
    for b in np.flatnonzero(~full & rc.converged):
        assert osys.mismatch(sbus[b], rc.v[b])[1] < tol
    return int((~full).sum())


@pytest.mark.parametrize("key,count", [("c0", None), ("c4", 300), ("c1", 203)])
def test_cpu_engine_matches_oracle(key, count):
    g, yb, sc = gg.workload(key, count=count)[0]
    plan = pf.Plan.from_ybus(yb, g.bus_type)
    osys = oracle.System.from_ybus(yb, g.bus_type)
    ro = osys.solve(sc.sbus, sc.v0)
    rc = pf.cpu_solve_batch(plan, yb.val, sc.sbus, sc.v0, threads=3)
    assert compare(osys, ro, rc, sc.sbus) <= sc.batch // 20
    assert rc.converged.mean() > 0.99
    assert (rc.status[rc.converged] == pf.PF_ST_CONVERGED).all()


def test_cpu_engine_thread_count_does_not_change_results():
    g, yb, sc = gg.workload("c4", count=77)[0]
    plan = pf.Plan.from_ybus(yb, g.bus_type)
    a = pf.cpu_solve_batch(plan, yb.val, sc.sbus, sc.v0, threads=1)
    b = pf.cpu_solve_batch(plan, yb.val, sc.sbus, sc.v0, threads=5)
    assert np.array_equal(a.v, b.v) and np.array_equal(a.iters, b.iters) and np.array_equal(a.status, b.status)


def test_cpu_engine_edge_cases():
    g, yb, sc = gg.workload("c4", count=20)[0]
    plan = pf.Plan.from_ybus(yb, g.bus_type)
    osys = oracle.System.from_ybus(yb, g.bus_type)
    for mi in (0, 1, 2):
        r = pf.cpu_solve_batch(plan, yb.val, sc.sbus, sc.v0, max_iter=mi)
        o = osys.solve(sc.sbus, sc.v0, max_iter=mi)
        assert np.array_equal(r.iters, o.iters) and np.array_equal(r.converged, o.converged)
        assert np.abs(r.v - o.v).max() < 1e-9
    sb = sc.sbus.copy()
    sb[3, 5] = np.nan                                   # same mini-batch as instances 0..7
    r = pf.cpu_solve_batch(plan, yb.val, sb, sc.v0)
    assert r.status[3] == pf.PF_ST_NONFINITE and not r.converged[3]
    mask = np.ones(20, bool); mask[3] = False
    ref = pf.cpu_solve_batch(plan, yb.val, sc.sbus, sc.v0)
    assert np.array_equal(r.v[mask], ref.v[mask]) and np.array_equal(r.iters[mask], ref.iters[mask])
    empty = pf.cpu_solve_batch(plan, yb.val, sc.sbus[:0], sc.v0[:0])
    assert empty.v.shape == (0, g.n, 2)
    with pytest.raises(pf.PfError):
        pf.cpu_solve_batch(plan, yb.val, sc.sbus, sc.v0, max_iter=-1)
