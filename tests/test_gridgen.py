"""The synthetic inputs: structure of the grids, admittance assembly and the workload
property that the stress factors were chosen for (checked with the CPU oracle)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as cg

import gridgen as gg
import oracle


@pytest.mark.parametrize("name", ["c0_14bus", "c1_1350bus", "c4_100bus", "c4_1000bus"])
def test_grid_structure(name):
    g = gg.grid(name)
    spec = gg.GRID_SPECS[name]
    assert (g.bus_type == gg.REF).sum() == 1 and g.bus_type[0] == gg.REF
    if spec["kind"] == "tree":
        assert g.n == 14 and g.m == 20
        assert (g.bus_type == gg.PV).sum() == 4 and (g.bus_type == gg.PQ).sum() == 9
    else:
        assert g.m == round(spec["avg_degree"] * g.n / 2)
        assert (g.bus_type == gg.PV).sum() == round(spec["pv_frac"] * g.n)
    # distinct branches, no self loops, connected
    assert np.all(g.f != g.t)
    assert len(set(zip(np.minimum(g.f, g.t), np.maximum(g.f, g.t)))) == g.m
    A = sp.coo_matrix((np.ones(g.m), (g.f, g.t)), shape=(g.n, g.n))
    assert cg.connected_components(A, directed=False)[0] == 1
    # parameter ranges (before the stress factor for b)
    assert np.all((g.r >= 0.01) & (g.r <= 0.1))
    assert np.all((g.x / g.r >= 2) & (g.x / g.r <= 5))
    k = g.meta["stress"]
    assert np.all((g.b >= 0) & (g.b <= 0.05 * k + 1e-15))


def test_ybus_assembly():
    g = gg.grid("c4_100bus")
    yb = gg.ybus(g)
    Y = sp.csr_matrix((yb.val, yb.col_idx, yb.row_ptr), shape=(g.n, g.n)).toarray()
    assert np.allclose(Y, Y.T)                            # no phase shifters
    assert np.all(np.diff(yb.row_ptr) >= 2)
    for i in range(g.n):                                  # sorted unique columns, diagonal present
        cols = yb.col_idx[yb.row_ptr[i]:yb.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
    # row sums equal the shunt admittance j * sum(b/2) of incident branches
    sh = np.zeros(g.n)
    np.add.at(sh, g.f, g.b / 2)
    np.add.at(sh, g.t, g.b / 2)
    assert np.allclose(Y.sum(axis=1), 1j * sh, atol=1e-12)


def test_scenarios_shapes_and_flat_start():
    g = gg.grid("c0_14bus")
    sc = gg.make_scenarios(g, 64, 2000, "uniform20")
    assert sc.sbus.shape == (64, 14) and sc.v0.shape == (64, 14, 2)
    assert np.all(sc.v0[:, :, 1] == 0)
    pq = g.bus_type == gg.PQ
    assert np.all(sc.v0[:, pq, 0] == 1.0)
    assert np.all(sc.v0[:, ~pq, 0] == g.v_set[~pq])
    assert np.all(sc.sbus[:, pq].real <= 0) and np.all(sc.sbus[:, g.bus_type == gg.PV].real >= 0)
    assert np.all(sc.sbus[:, g.bus_type == gg.PV].imag == 0)
    # same seed, same draw
    assert np.array_equal(sc.sbus, gg.make_scenarios(g, 64, 2000, "uniform20").sbus)


@pytest.mark.slow
@pytest.mark.parametrize("name,count", [("c0_14bus", 64), ("c4_100bus", 200), ("c4_1000bus", 200),
                                        ("c1_1350bus", 200), ("c4_3000bus", 100),
                                        ("c2_9000bus", 100), ("c4_9000bus", 100)])
def test_stress_factor_choice(name, count):
    """Base case from flat start converges in <= 5 iterations; >= 99 % of a scenario
    sample converges within 10 (the rule the stress factors were picked by)."""
    g = gg.grid(name)
    kind = "uniform20" if name.startswith("c0") else "mc"
    s = oracle.System.from_ybus(gg.ybus(g), g.bus_type)
    bc = gg.base_case(g, kind)
    r = s.solve(bc.sbus, bc.v0, threads=8)
    assert r.converged[0] and r.iters[0] <= 5
    sc = gg.make_scenarios(g, count, 424242, kind)
    r = s.solve(sc.sbus, sc.v0, threads=8)
    assert r.converged.mean() >= 0.99 - 1.0 / count


def test_outage_ybus_keeps_pattern_and_matches_reduced_grid():
    g = gg.grid("c4_100bus")
    full = gg.ybus(g)
    nb = gg.non_bridge_branches(g)
    assert 0 < nb.size < g.f.size              # the spanning tree's branches are bridges
    for k in nb[:5]:
        yk = gg.ybus_outage(g, int(k))
        assert np.array_equal(yk.row_ptr, full.row_ptr) and np.array_equal(yk.col_idx, full.col_idx)
        # the outaged branch's two off-diagonal entries are explicit zeros
        f, t = int(g.f[k]), int(g.t[k])
        for i, j in ((f, t), (t, f)):
            q = full.row_ptr[i] + np.flatnonzero(full.col_idx[full.row_ptr[i]:full.row_ptr[i + 1]] == j)[0]
            assert yk.val[q] == 0
        # every other entry equals the full Ybus minus the branch's pi model
        ys = 1.0 / (g.r[k] + 1j * g.x[k])
        d = full.val - yk.val
        dense = np.zeros((g.n, g.n), complex)
        for i in range(g.n):
            for q in range(full.row_ptr[i], full.row_ptr[i + 1]):
                dense[i, full.col_idx[q]] = d[q]
        expect = np.zeros((g.n, g.n), complex)
        expect[f, f] = expect[t, t] = ys + 0.5j * g.b[k]
        expect[f, t] = expect[t, f] = -ys
        assert np.allclose(dense, expect, atol=1e-12)


def test_outage_solution_equals_reduced_grid_solution():
    # the explicit zeros do not change the oracle's power flow: solving on the full pattern
    # with the outage values equals solving the grid rebuilt without the branch
    g = gg.grid("c4_100bus")
    k = int(gg.non_bridge_branches(g)[3])
    keep = np.ones(g.f.size, bool)
    keep[k] = False
    sub = gg.Grid(**{**g.__dict__, "f": g.f[keep], "t": g.t[keep], "r": g.r[keep], "x": g.x[keep], "b": g.b[keep]})
    sc = gg.make_scenarios(g, 4, 17, "mc")
    a = oracle.System.from_ybus(gg.ybus_outage(g, k), g.bus_type).solve(sc.sbus, sc.v0)
    b = oracle.System.from_ybus(gg.ybus(sub), g.bus_type).solve(sc.sbus, sc.v0)
    assert np.array_equal(a.converged, b.converged) and np.array_equal(a.iters, b.iters)
    assert np.abs(a.v - b.v).max() <= 1e-10
