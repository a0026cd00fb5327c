"""The second chance for instances whose fixed-order refactorization fails (Sec. 3.2: such
a task is solved again with a pivoting factorization; Sec. 4.1: partial pivoting updates
the row permutation of Eq. 3).  CPU tests: the library's threshold-pivoting Newton solve
(pf_cpu_solve_pivoting, the factorization pf_solve_fallback uses) against the oracle, and
a seeded instance whose first diagonal pivot vanishes under the fixed pre-order.

The failing instance: every branch at the first bus of the pre-order is made purely
resistive (x = 0, no charging).  The diagonal derivative is
dP_i/dangle_i = sum_k |V_i||V_k| (B_ik cos angle_ik - G_ik sin angle_ik); at flat start
every angle difference is zero, so it is sum_k |V_i||V_k| B_ik, and B_ik = 0 on a
resistive branch: the first column's pivot is exactly zero, while J as a whole is
nonsingular (the column has a nonzero entry in a neighbour's Q row), so a pivoting
factorization solves the instance."""
import dataclasses

import numpy as np
import pytest

import gridgen as gg
import oracle
import paper_2101_02270_amd as pf


def resistive_first_bus(name):
    """(grid, ybus, plan) of `name` with every branch at the pre-order's first bus made
    purely resistive; the Ybus pattern, and so the plan, is unchanged."""
    g = gg.grid(name)
    yb = gg.ybus(g)
    plan = pf.Plan.from_ybus(yb, g.bus_type)
    u = int(plan.order()[0])
    pv = np.flatnonzero(g.bus_type == 2)
    pq = np.flatnonzero(g.bus_type == 1)
    bus = int(np.concatenate([pv, pq, pq])[u])
    lines = np.flatnonzero((g.f == bus) | (g.t == bus))
    x = g.x.copy()
    b = g.b.copy()
    x[lines] = 0.0
    b[lines] = 0.0
    g2 = dataclasses.replace(g, x=x, b=b)
    yb2 = gg.ybus(g2)
    assert np.array_equal(yb2.col_idx, yb.col_idx) and np.array_equal(yb2.row_ptr, yb.row_ptr)
    return g2, yb2, plan, bus


@pytest.mark.parametrize("key", ["c0", "c1"])
def test_pivoting_solve_matches_oracle(key):
    (g, yb, sc), = gg.workload(key, count=300)
    plan = pf.Plan.from_ybus(yb, g.bus_type)
    ro = oracle.System.from_ybus(yb, g.bus_type).solve(sc.sbus, sc.v0)
    r = pf.cpu_solve_pivoting(plan, yb.val, sc.sbus, sc.v0)
    assert np.array_equal(r.converged, ro.converged)
    both = r.converged & ro.converged
    assert np.array_equal(r.iters[both], ro.iters[both])
    assert np.abs(r.v[both] - ro.v[both]).max() <= 1e-10
    assert (r.status[both] == pf.PF_ST_CONVERGED).all()


def test_pivoting_solve_batched_ybus_matches_oracle():
    """N-1 values (one branch out per instance) through the batched-Ybus path."""
    g = gg.grid("c4_100bus")
    yb = gg.ybus(g)
    sc = gg.make_scenarios(g, 40, 91, "mc")
    plan = pf.Plan.from_ybus(yb, g.bus_type)
    out = np.random.default_rng(5).choice(gg.non_bridge_branches(g), sc.batch)
    yv = gg.ybus_outage_values(g, yb, out)
    r = pf.cpu_solve_pivoting(plan, yv, sc.sbus, sc.v0)
    for b in range(sc.batch):
        ob = oracle.System(yb.row_ptr, yb.col_idx, yv[b], g.bus_type).solve(sc.sbus[b:b + 1], sc.v0[b:b + 1])
        assert bool(r.converged[b]) == bool(ob.converged[0])
        if ob.converged[0]:
            assert r.iters[b] == ob.iters[0]
            assert np.abs(r.v[b] - ob.v[0]).max() <= 1e-10


@pytest.mark.parametrize("name", ["c0_14bus", "c4_100bus"])
def test_zero_pivot_instance_fails_fixed_order_and_is_rescued(name):
    g, yb, plan, bus = resistive_first_bus(name)
    sc = gg.make_scenarios(g, 16, 77, "uniform20" if name == "c0_14bus" else "mc")
    osys = oracle.System.from_ybus(yb, g.bus_type)
    # the zero is exact at flat start: the first column's diagonal Jacobian entry
    rp, ci = osys.jacobian_pattern()
    u = int(plan.order()[0])
    J = osys.jacobian(sc.v0[0])
    diag = J[rp[u] + np.flatnonzero(ci[rp[u]:rp[u + 1]] == u)[0]]
    assert diag == 0.0
    # the fixed-order refactorization (CPU engine, same plan and pivot rule as the GPU)
    # fails every instance at the first iteration
    rc = pf.cpu_solve_batch(plan, yb.val, sc.sbus, sc.v0)
    assert (rc.status == pf.PF_ST_PIVOT).all() and not rc.converged.any()
    assert (rc.iters == 0).all()
    # the threshold-pivoting solve converges to the oracle's result
    ro = osys.solve(sc.sbus, sc.v0)
    assert ro.converged.all()
    r = pf.cpu_solve_pivoting(plan, yb.val, sc.sbus, sc.v0)
    assert r.converged.all()
    assert np.array_equal(r.iters, ro.iters)
    assert np.abs(r.v - ro.v).max() <= 1e-10


def test_pivoting_solve_edge_cases():
    (g, yb, sc), = gg.workload("c0", count=3)
    plan = pf.Plan.from_ybus(yb, g.bus_type)
    r = pf.cpu_solve_pivoting(plan, yb.val, sc.sbus, sc.v0, max_iter=0)
    assert (r.iters == 0).all()
    ro = oracle.System.from_ybus(yb, g.bus_type).solve(sc.sbus, sc.v0, max_iter=0)
    assert np.array_equal(r.converged, ro.converged)
    e = pf.cpu_solve_pivoting(plan, yb.val, sc.sbus[:0], sc.v0[:0])
    assert e.v.shape == (0, g.n, 2)
    with pytest.raises(pf.PfError):
        pf.cpu_solve_pivoting(plan, yb.val[:-1], sc.sbus, sc.v0)
