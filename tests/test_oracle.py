"""Pins of the FP64 CPU oracle against facts fixed by the mathematics, independent of it.

* two-bus closed form (and an infeasible two-bus case with no real solution);
* a dense brute-force Newton iteration that builds the Jacobian from the complex matrix
  identities dS/dVa = j diag(V) conj(diag(I) - Y diag(V)) and
  dS/dVm = diag(V) conj(Y diag(V/|V|)) + conj(diag(I)) diag(V/|V|), solved with
  numpy.linalg.solve;
* central finite differences of the mismatch for the Jacobian;
* the power-balance invariant at convergence, with branch flows taken from the branch
  list rather than from Ybus;
* quadratic convergence in the final Newton steps;
* the sparse pivoting LU against dense LAPACK solves, including matrices that need
  off-diagonal pivots;
* the minimum-degree order on graphs whose optimal elimination is known.
"""
import numpy as np
import pytest

import gridgen as gg
import oracle


# ------------------------------------------------------------------ helpers
def two_bus(v1, r, x, p, q):
    y = 1.0 / (r + 1j * x)
    yb = gg.Ybus(n=2, row_ptr=np.array([0, 2, 4], np.int32), col_idx=np.array([0, 1, 0, 1], np.int32),
                 val=np.array([y, -y, -y, y]))
    bt = np.array([gg.REF, gg.PQ], np.int8)
    sbus = np.array([[0.0, -(p + 1j * q)]])
    v0 = np.array([[[v1, 0.0], [1.0, 0.0]]])
    return yb, bt, sbus, v0


def two_bus_closed_form(v1, r, x, p, q):
    """High-voltage root of V2 conj(y (V2 - V1)) = -(P + jQ) with V1 real:
    |V2|^2 = (a + sqrt(a^2 - 4 (r^2 + x^2)(P^2 + Q^2))) / 2, a = V1^2 - 2 (rP + xQ),
    angle V2 = atan2(Qr - Px, |V2|^2 + Pr + Qx)."""
    a = v1 ** 2 - 2.0 * (r * p + x * q)
    disc = a * a - 4.0 * (r * r + x * x) * (p * p + q * q)
    if disc < 0:
        return None
    u = 0.5 * (a + np.sqrt(disc))
    return np.sqrt(u), np.arctan2(q * r - p * x, u + p * r + q * x)


def dense_nr(yb, bt, sbus, v0, tol=1e-8, max_iter=10):
    """Brute-force NR with dense matrices and numpy.linalg.solve (same step rules)."""
    n = yb.n
    Y = np.zeros((n, n), complex)
    for i in range(n):
        for p in range(yb.row_ptr[i], yb.row_ptr[i + 1]):
            Y[i, yb.col_idx[p]] += yb.val[p]
    pv = np.flatnonzero(bt == gg.PV)
    pq = np.flatnonzero(bt == gg.PQ)
    pvpq = np.r_[pv, pq]
    vm = v0[:, 0].copy()
    va = v0[:, 1].copy()
    hist = []
    for k in range(max_iter + 1):
        V = vm * np.exp(1j * va)
        I = Y @ V
        mis = V * np.conj(I) - sbus
        F = np.r_[mis[pvpq].real, mis[pq].imag]
        nf = np.max(np.abs(F))
        hist.append(nf)
        if not np.isfinite(nf):
            return vm, va, k, False, hist
        if nf < tol:
            return vm, va, k, True, hist
        if k == max_iter:
            return vm, va, k, False, hist
        dVa = 1j * np.diag(V) @ np.conj(np.diag(I) - Y @ np.diag(V))
        dVm = np.diag(V) @ np.conj(Y @ np.diag(V / np.abs(V))) + np.conj(np.diag(I)) @ np.diag(V / np.abs(V))
        J = np.block([[dVa[np.ix_(pvpq, pvpq)].real, dVm[np.ix_(pvpq, pq)].real],
                      [dVa[np.ix_(pq, pvpq)].imag, dVm[np.ix_(pq, pq)].imag]])
        dx = np.linalg.solve(J, F)
        va[pvpq] -= dx[:pvpq.size]
        vm[pq] -= dx[pvpq.size:]


def small_grids():
    out = [gg.grid("c0_14bus")]
    for seed in (11, 12, 13):
        out.append(gg.make_tree_grid(n_pv=5, n_pq=22, n_chords=6, seed=seed, stress=0.5,
                                     name=f"tree28_{seed}"))
    out.append(gg.make_geometric_grid(n=30, avg_degree=2.8, pv_frac=0.15, seed=21, stress=0.3,
                                      name="geo30"))
    return out


# ------------------------------------------------------------------ two-bus closed form
@pytest.mark.parametrize("case", [(1.0, 0.02, 0.06, 0.5, 0.2), (1.05, 0.05, 0.2, 0.8, 0.3),
                                  (1.02, 0.01, 0.05, 0.3, -0.1)])
def test_two_bus_closed_form(case):
    yb, bt, sbus, v0 = two_bus(*case)
    exp = two_bus_closed_form(*case)
    sysm = oracle.System.from_ybus(yb, bt)
    res = sysm.solve(sbus, v0, tol=1e-12, max_iter=20, threads=1)
    assert res.converged[0]
    assert abs(res.v[0, 1, 0] - exp[0]) < 1e-10
    assert abs(res.v[0, 1, 1] - exp[1]) < 1e-10
    assert res.v[0, 0, 0] == case[0] and res.v[0, 0, 1] == 0.0


def test_two_bus_known_values():
    # (V1, r, x, P, Q) -> (|V2|, angle V2), evaluated from the closed form to 12 digits
    assert np.allclose(two_bus_closed_form(1.0, 0.02, 0.06, 0.5, 0.2),
                       (0.977131038746, -0.026611649822), atol=1e-11)
    assert np.allclose(two_bus_closed_form(1.05, 0.05, 0.2, 0.8, 0.3),
                       (0.930969087584, -0.148884366866), atol=1e-11)


def test_two_bus_infeasible_not_converged():
    case = (1.0, 0.1, 0.3, 1.0, 0.5)
    assert two_bus_closed_form(*case) is None
    yb, bt, sbus, v0 = two_bus(*case)
    res = oracle.System.from_ybus(yb, bt).solve(sbus, v0, tol=1e-8, max_iter=10, threads=1)
    assert not res.converged[0]
    assert res.status[0] in (1, 2, 3)


def test_max_iter_semantics():
    yb, bt, sbus, v0 = two_bus(1.0, 0.02, 0.06, 0.5, 0.2)
    s = oracle.System.from_ybus(yb, bt)
    r0 = s.solve(sbus, v0, max_iter=0, threads=1)
    assert not r0.converged[0] and r0.iters[0] == 0 and r0.status[0] == 1
    assert np.array_equal(r0.v, v0)
    r1 = s.solve(sbus, v0, max_iter=1, threads=1)
    assert r1.iters[0] == 1 and not r1.converged[0]
    rf = s.solve(sbus, v0, max_iter=10, threads=1)
    assert rf.converged[0] and 2 <= rf.iters[0] <= 6
    # a start that already satisfies the tolerance performs no update
    exact = rf.v.copy()
    rz = s.solve(sbus, exact, max_iter=10, threads=1)
    assert rz.converged[0] and rz.iters[0] == 0


# ------------------------------------------------------------------ brute force
@pytest.mark.parametrize("g", small_grids(), ids=lambda g: g.name)
def test_matches_dense_bruteforce(g):
    yb = gg.ybus(g)
    sc = gg.make_scenarios(g, 8, 77, "uniform20" if g.name.startswith("c0") else "mc")
    res = oracle.System.from_ybus(yb, g.bus_type).solve(sc.sbus, sc.v0, threads=2)
    for b in range(sc.batch):
        vm, va, k, ok, hist = dense_nr(yb, g.bus_type, sc.sbus[b], sc.v0[b])
        assert ok == bool(res.converged[b])
        assert k == res.iters[b]
        if ok:
            assert np.max(np.abs(vm - res.v[b, :, 0])) < 1e-12
            assert np.max(np.abs(va - res.v[b, :, 1])) < 1e-12
            h = res.hist[b, :k + 1]
            above = np.asarray(hist) > 1e-10      # below that both sit at the rounding floor
            assert np.allclose(h[above], np.asarray(hist)[above], rtol=1e-6)
            assert np.all(h[~above] < 1e-10)


# ------------------------------------------------------------------ Jacobian by finite differences
@pytest.mark.parametrize("g", small_grids()[:3], ids=lambda g: g.name)
def test_jacobian_finite_differences(g):
    yb = gg.ybus(g)
    s = oracle.System.from_ybus(yb, g.bus_type)
    rng = np.random.default_rng(5)
    v = gg.flat_start(g, 1)[0]
    v[:, 0] *= rng.uniform(0.95, 1.05, g.n)
    v[:, 1] = rng.uniform(-0.2, 0.2, g.n)
    sbus = gg.make_scenarios(g, 1, 3, "mc").sbus[0]
    J = s.jacobian_dense(v)
    pv, pq = s.unknown_buses()
    unk = [(b, 1) for b in pv] + [(b, 1) for b in pq] + [(b, 0) for b in pq]
    h = 1e-6
    Jfd = np.zeros_like(J)
    for c, (bus, comp) in enumerate(unk):
        vp = v.copy(); vp[bus, comp] += h
        vmn = v.copy(); vmn[bus, comp] -= h
        Fp, _ = s.mismatch(sbus, vp)
        Fm, _ = s.mismatch(sbus, vmn)
        Jfd[:, c] = (Fp - Fm) / (2 * h)
    scale = np.max(np.abs(J))
    assert np.max(np.abs(J - Jfd)) / scale < 1e-6
    # the structural pattern covers every numerically nonzero derivative
    rp, ci = s.jacobian_pattern()
    mask = np.zeros_like(J, bool)
    for r in range(s.N):
        mask[r, ci[rp[r]:rp[r + 1]]] = True
    assert np.all(np.abs(Jfd[~mask]) < 1e-7 * scale)


def test_mismatch_sign_and_content():
    # at the exact two-bus solution the mismatch vanishes; with zero voltage angle and
    # |V2| = 1 it equals calculated minus specified power
    case = (1.0, 0.02, 0.06, 0.5, 0.2)
    yb, bt, sbus, v0 = two_bus(*case)
    s = oracle.System.from_ybus(yb, bt)
    m, a = two_bus_closed_form(*case)
    F, nf = s.mismatch(sbus[0], np.array([[1.0, 0.0], [m, a]]))
    assert nf < 1e-12
    F, nf = s.mismatch(sbus[0], v0[0])
    y = 1.0 / (0.02 + 0.06j)
    s2 = 1.0 * np.conj(y * (1.0 - 1.0))
    assert np.allclose(F, [s2.real + 0.5, s2.imag + 0.2])


# ------------------------------------------------------------------ invariants at convergence
def branch_check(g, res, sbus):
    for b in range(res.v.shape[0]):
        if not res.converged[b]:
            continue
        v = res.v[b]
        sf, st = oracle.branch_flows(g, v)
        inj = np.zeros(g.n, complex)
        np.add.at(inj, g.f, sf)
        np.add.at(inj, g.t, st)
        pq = g.bus_type == gg.PQ
        pvpq = g.bus_type != gg.REF
        # injections from branch flows reproduce the specified ones
        assert np.max(np.abs(inj.real[pvpq] - sbus[b].real[pvpq])) < 1e-8
        assert np.max(np.abs(inj.imag[pq] - sbus[b].imag[pq])) < 1e-8
        # active balance: sum of specified pv/pq injections + slack = series losses
        V = v[:, 0] * np.exp(1j * v[:, 1])
        i_s = (V[g.f] - V[g.t]) / (g.r + 1j * g.x)
        losses = np.sum(g.r * np.abs(i_s) ** 2)
        ref = np.flatnonzero(g.bus_type == gg.REF)[0]
        lhs = np.sum(sbus[b].real[pvpq]) + inj.real[ref]
        assert abs(lhs - losses) < pvpq.sum() * 1e-8 + 1e-10
        assert losses >= 0
        # reactive balance: series reactive losses minus line charging
        q_ser = np.sum(g.x * np.abs(i_s) ** 2)
        q_ch = np.sum(0.5 * g.b * (np.abs(V[g.f]) ** 2 + np.abs(V[g.t]) ** 2))
        pvref = ~pq
        lhs_q = np.sum(sbus[b].imag[pq]) + np.sum(inj.imag[pvref])
        assert abs(lhs_q - (q_ser - q_ch)) < pq.sum() * 1e-8 + 1e-9


@pytest.mark.parametrize("g", small_grids(), ids=lambda g: g.name)
def test_power_balance_invariant(g):
    yb = gg.ybus(g)
    sc = gg.make_scenarios(g, 16, 99, "uniform20" if g.name.startswith("c0") else "mc")
    res = oracle.System.from_ybus(yb, g.bus_type).solve(sc.sbus, sc.v0, threads=4)
    assert res.converged.sum() >= 15
    branch_check(g, res, sc.sbus)


def test_quadratic_convergence_and_tolerance():
    g = gg.grid("c1_1350bus")
    yb = gg.ybus(g)
    sc = gg.make_scenarios(g, 24, 2001, "mc")
    res = oracle.System.from_ybus(yb, g.bus_type).solve(sc.sbus, sc.v0, threads=8)
    assert res.converged.mean() > 0.9
    for b in np.flatnonzero(res.converged):
        k = res.iters[b]
        h = res.hist[b]
        assert h[k] < 1e-8
        assert np.all(h[:k] >= 1e-8)
        for j in range(k):
            if h[j] < 1e-2:
                assert h[j + 1] <= 100.0 * h[j] ** 2 + 1e-13
    branch_check(g, res, sc.sbus)


# ------------------------------------------------------------------ linear algebra
def _random_sparse(N, density, rng, zero_diag_frac=0.0):
    A = np.where(rng.random((N, N)) < density, rng.normal(size=(N, N)), 0.0)
    A += np.diag(rng.uniform(1.0, 2.0, N) * np.sign(rng.normal(size=N)))
    if zero_diag_frac:
        idx = rng.choice(N, int(zero_diag_frac * N), replace=False)
        A[idx, idx] = 0.0
        # keep it nonsingular with an off-diagonal partner in each zeroed row
        for i in idx:
            j = (i + 1) % N
            A[i, j] = A[j, i] = 3.0
    return A


def _csr(A):
    rp = [0]; ci = []; v = []
    for r in range(A.shape[0]):
        nz = np.flatnonzero(A[r])
        ci += nz.tolist(); v += A[r, nz].tolist(); rp.append(len(ci))
    return np.array(rp), np.array(ci), np.array(v)


@pytest.mark.parametrize("seed,zf", [(1, 0.0), (2, 0.0), (3, 0.3), (4, 0.5)])
def test_sparse_lu_against_dense(seed, zf):
    rng = np.random.default_rng(seed)
    N = 60
    A = _random_sparse(N, 0.05, rng, zf)
    b = rng.normal(size=N)
    x = oracle.sparse_solve(*_csr(A), b)
    xr = np.linalg.solve(A, b)
    assert np.max(np.abs(x - xr)) / np.max(np.abs(xr)) < 1e-10
    assert np.max(np.abs(A @ x - b)) < 1e-10 * np.max(np.abs(A)) * np.max(np.abs(x))


def test_needs_pivoting_permutation_matrix():
    # an anti-diagonal matrix has no usable diagonal pivot at all
    N = 7
    A = np.fliplr(np.diag(np.arange(1.0, N + 1)))
    b = np.arange(N, dtype=float)
    assert np.allclose(oracle.sparse_solve(*_csr(A), b), np.linalg.solve(A, b), atol=1e-14)


def test_singular_detected():
    A = np.array([[1.0, 2.0], [2.0, 4.0]])
    with pytest.raises(np.linalg.LinAlgError):
        oracle.sparse_solve(*_csr(A), np.ones(2))


def test_jacobian_solve_residual():
    g = gg.grid("c1_1350bus")
    s = oracle.System.from_ybus(gg.ybus(g), g.bus_type)
    sc = gg.make_scenarios(g, 1, 5, "mc")
    J = s.jacobian(sc.v0[0])
    F, _ = s.mismatch(sc.sbus[0], sc.v0[0])
    x = s.jacobian_solve(J, F)
    import scipy.sparse as sp
    rp, ci = s.jacobian_pattern()
    Js = sp.csr_matrix((J, ci, rp), shape=(s.N, s.N))
    r = Js @ x - F
    assert np.max(np.abs(r)) / np.max(np.abs(F)) < 1e-12


# ------------------------------------------------------------------ ordering
def _sym_csr(n, edges):
    adj = [set([i]) for i in range(n)]
    for a, b in edges:
        adj[a].add(b); adj[b].add(a)
    rp = [0]; ci = []
    for i in range(n):
        ci += sorted(adj[i]); rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32)


def _fill(n, edges, order):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b); adj[b].add(a)
    gone = set(); fill = 0
    for v in order:
        nb = [u for u in adj[v] if u not in gone]
        for i in range(len(nb)):
            for j in range(i + 1, len(nb)):
                if nb[j] not in adj[nb[i]]:
                    adj[nb[i]].add(nb[j]); adj[nb[j]].add(nb[i]); fill += 1
        gone.add(v)
    return fill


def test_min_degree_path_and_star_and_tree_have_no_fill():
    # The oracle orders the unknowns of a Jacobian; test it through a pure-PQ chain
    # (J pattern = block tridiagonal) and a star, whose perfect orderings exist.
    for kind in ("path", "star", "tree"):
        n = 12
        if kind == "path":
            edges = [(i, i + 1) for i in range(n - 1)]
        elif kind == "star":
            edges = [(0, i) for i in range(1, n)]
        else:
            rng = np.random.default_rng(3)
            edges = [(i, int(rng.integers(0, i))) for i in range(1, n)]
        rp, ci = _sym_csr(n, edges)
        vals = np.ones(ci.shape[0])
        # build a CSR system whose sparse solve exercises the ordering; its fill must be 0
        ys = []
        for i in range(n):
            for p in range(rp[i], rp[i + 1]):
                ys.append(5.0 if ci[p] == i else -1.0)
        bt = np.full(n, gg.PQ, np.int8); bt[0 if kind != "star" else n - 1] = gg.REF
        s = oracle.System(rp, ci, np.array(ys, complex) * (1 - 3j), bt)
        order = s.order()
        assert sorted(order.tolist()) == list(range(s.N))
        jrp, jci = s.jacobian_pattern()
        jedges = [(r, c) for r in range(s.N) for c in jci[jrp[r]:jrp[r + 1]] if c > r]
        assert _fill(s.N, jedges, order) == 0, kind
