"""Comparison of GPU solve results with the oracle's, shared by the GPU test modules.

The bars, written out:
  * FP64 (compare_solve): identical convergence flags and iteration counts, |V| within
    1e-6 pu and angle within 1e-6 rad, except for borderline instances (the oracle's final
    or penultimate max|F| within a factor 2 of the tolerance), where the two may stop one
    iteration apart and a GPU result reported converged must instead meet the tolerance in
    the oracle's own FP64 mismatch;
  * FP32-LU (compare_fp32lu): every instance the oracle converges converges, every GPU
    result reported converged meets the oracle's FP64 mismatch test, and both-converged
    results lie within 1e-6 of the oracle's;
  * no instance reports PF_ST_INTERNAL.
"""
import numpy as np

import paper_2101_02270_amd as pf


def _host(res_g):
    return (res_g.v.cpu().numpy(), res_g.iters.cpu().numpy(), res_g.converged.cpu().numpy().astype(bool),
            res_g.status.cpu().numpy())


def compare_solve(osys, res_o, res_g, sbus=None, tol=1e-8, vtol=1e-6):
    """The FP64 full-solve bar, vectorised over the batch.  Every instance whose oracle
    mismatch history ends (final or penultimate value) within a factor 2 of the tolerance
    is borderline: there the two implementations may stop one iteration apart, so only
    validity is required -- a GPU result reported converged must meet the tolerance in
    the oracle's own FP64 mismatch (checked when sbus is given).  Every other instance must
    match in convergence flag, iteration count, |V| and angle.  No instance may report
    PF_ST_INTERNAL.  Returns the borderline indices."""
    v_g, it_g, cv_g, st_g = _host(res_g)
    B = v_g.shape[0]
    assert not (st_g == pf.PF_ST_INTERNAL).any(), np.flatnonzero(st_g == pf.PF_ST_INTERNAL)
    k = res_o.iters.astype(np.int64)
    h = res_o.hist
    last = h[np.arange(B), k]
    prev = h[np.arange(B), np.maximum(k - 1, 0)]
    band = lambda x: np.isfinite(x) & (x >= 0.5 * tol) & (x <= 2 * tol)
    border = band(last) | band(prev)
    full = ~border
    bad = np.flatnonzero(full & (cv_g != res_o.converged))
    assert bad.size == 0, [(b, st_g[b], res_o.status[b]) for b in bad[:10]]
    both = full & res_o.converged
    bad = np.flatnonzero(both & (it_g != res_o.iters))
    assert bad.size == 0, [(b, it_g[b], res_o.iters[b]) for b in bad[:10]]
    if both.any():
        dvm = np.abs(v_g[both, :, 0] - res_o.v[both, :, 0]).max()
        dva = np.abs(v_g[both, :, 1] - res_o.v[both, :, 1]).max()
        assert dvm <= vtol and dva <= vtol, (dvm, dva)
        assert (st_g[both] == pf.PF_ST_CONVERGED).all()
    if sbus is not None:
        for b in np.flatnonzero(border & cv_g):
            assert osys.mismatch(sbus[b], v_g[b])[1] < tol, b
    return np.flatnonzero(border)


def compare_fp32lu(osys, res_o, res_g, sbus, tol=1e-8, vtol=1e-6, name=""):
    """The FP32-LU bar: the stopping test is FP64, so every instance the GPU reports
    converged must meet the tolerance in the oracle's FP64 mismatch at the returned V and
    lie within 1e-6 pu / rad of the oracle's solution where both converged; every instance
    the oracle converges must converge (the inexact Newton step may cost iterations but not
    convergence on these workloads); no PF_ST_INTERNAL.  Returns (max error, extra
    iterations of the instances both converged)."""
    v_g, it_g, cv_g, st_g = _host(res_g)
    assert not (st_g == pf.PF_ST_INTERNAL).any()
    missing = np.flatnonzero(res_o.converged & ~cv_g)
    assert missing.size == 0, missing[:10]
    both = cv_g & res_o.converged
    err = float(np.abs(v_g[both] - res_o.v[both]).max()) if both.any() else 0.0
    assert err <= vtol, err
    for b in np.flatnonzero(cv_g):
        assert osys.mismatch(sbus[b], v_g[b])[1] < tol, b
    extra = it_g[both] - res_o.iters[both]
    print(f"\n{name}: FP32-LU max |V|/angle error vs oracle {err:.2e}; extra iterations mean "
          f"{extra.mean():.3f}, max {extra.max() if extra.size else 0}, histogram "
          f"{np.bincount(extra - extra.min()).tolist() if extra.size else []} from {extra.min() if extra.size else 0}")
    return err, extra
