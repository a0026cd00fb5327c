"""Host-side checks of the C-ABI library (no GPU needed): every declared symbol is
exported, pf_analyze rejects malformed patterns, and the plan's symbolic analysis is the
structure the numerical kernels rely on.

Symbolic pins (independent of the plan's own code):
  * the L+U pattern equals the nonzero structure of a dense LU without pivoting of
    P J P^T with random values (brute force on small grids);
  * every column dependency k -> j (U(k, j) != 0) has level(k) < level(j);
  * the elimination order is a permutation and keeps a PQ bus's two unknowns adjacent;
  * the minimum-degree order produces much less fill than the natural order.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import gridgen as gg
import oracle
import paper_2101_02270_amd as pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "pf_analyze" in names and "pf_solve_batch" in names
    lib = ctypes.CDLL(pf.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(pf.EXPORTED)


def _pattern(g):
    yb = gg.ybus(g)
    return yb.row_ptr.copy(), yb.col_idx.copy(), g.bus_type.copy()


def _analyze_rc(rp, ci, bt, ordering=pf.PF_ORDER_MIN_DEGREE, perm=None):
    try:
        pf.Plan(rp, ci, bt, ordering=ordering, user_perm=perm)
        return 0, ""
    except pf.PfError as e:
        return -1, str(e)


def test_analyze_rejects_malformed_input():
    g = gg.grid("c0_14bus")
    rp, ci, bt = _pattern(g)
    assert _analyze_rc(rp, ci, bt)[0] == 0
    b2 = bt.copy(); b2[b2 == gg.REF] = gg.PQ
    assert "REF" in _analyze_rc(rp, ci, b2)[1]
    b3 = bt.copy(); b3[3] = gg.REF
    assert "REF" in _analyze_rc(rp, ci, b3)[1]
    b4 = bt.copy(); b4[2] = 7
    assert "type" in _analyze_rc(rp, ci, b4)[1]
    # drop the diagonal of row 5
    r5 = list(range(rp[5], rp[6]))
    d = [p for p in r5 if ci[p] == 5][0]
    ci2 = np.delete(ci, d); rp2 = rp.copy(); rp2[6:] -= 1
    assert "diagonal" in _analyze_rc(rp2, ci2, bt)[1]
    # unsorted columns in row 4
    ci3 = ci.copy(); a, b_ = rp[4], rp[5]
    ci3[a:b_] = ci3[a:b_][::-1]
    assert "unsorted" in _analyze_rc(rp, ci3, bt)[1]
    # structural asymmetry: remove one off-diagonal (i, k) but keep (k, i)
    i = 6
    off = [p for p in range(rp[i], rp[i + 1]) if ci[p] != i][0]
    ci4 = np.delete(ci, off); rp4 = rp.copy(); rp4[i + 1:] -= 1
    assert "symmetric" in _analyze_rc(rp4, ci4, bt)[1]
    # bad user permutation
    N = (bt == gg.PV).sum() + 2 * (bt == gg.PQ).sum()
    bad = np.arange(N); bad[0] = 1
    assert "permutation" in _analyze_rc(rp, ci, bt, pf.PF_ORDER_USER, bad)[1]


def test_isolated_bus_rejected_and_single_bus_accepted():
    rp = np.array([0, 1, 3, 5], np.int32)
    ci = np.array([0, 1, 2, 1, 2], np.int32)
    bt = np.array([gg.PQ, gg.REF, gg.PQ], np.int8)
    assert "isolated" in _analyze_rc(rp, ci, bt)[1]
    p = pf.Plan(np.array([0, 1], np.int32), np.array([0], np.int32), np.array([gg.REF], np.int8))
    assert p.N == 0 and p.nnz_lu == 0


def dense_symbolic(osys, perm):
    """Nonzero structure of a dense no-pivot LU of P J P^T with random values."""
    rp, ci = osys.jacobian_pattern()
    N = osys.N
    A = np.zeros((N, N))
    rng = np.random.default_rng(0)
    for r in range(N):
        A[r, ci[rp[r]:rp[r + 1]]] = rng.uniform(1, 2, rp[r + 1] - rp[r])
    A += np.eye(N) * N * 4               # keep the elimination well defined
    A = A[np.ix_(perm, perm)]
    S = A != 0
    for k in range(N):
        rows = np.flatnonzero(S[k + 1:, k]) + k + 1
        cols = np.flatnonzero(S[k, k + 1:]) + k + 1
        S[np.ix_(rows, cols)] = True
    return S


@pytest.mark.parametrize("name", ["c0_14bus", "c4_100bus"])
@pytest.mark.parametrize("ordering", [pf.PF_ORDER_MIN_DEGREE, pf.PF_ORDER_NATURAL])
def test_symbolic_pattern_matches_dense_elimination(name, ordering):
    g = gg.grid(name)
    yb = gg.ybus(g)
    plan = pf.Plan.from_ybus(yb, g.bus_type, ordering=ordering)
    osys = oracle.System.from_ybus(yb, g.bus_type)
    perm = plan.order()
    assert sorted(perm.tolist()) == list(range(plan.N))
    cp, ri, lv = plan.lu_pattern()
    S = np.zeros((plan.N, plan.N), bool)
    for j in range(plan.N):
        rows = ri[cp[j]:cp[j + 1]]
        assert np.all(np.diff(rows) > 0) and j in rows
        S[rows, j] = True
    assert np.array_equal(S, dense_symbolic(osys, perm))
    assert plan.nnz_lu >= plan.info["nnz_j"]
    # level validity: every dependency U(k, j) != 0, k < j has level(k) < level(j)
    for j in range(plan.N):
        for k in ri[cp[j]:cp[j + 1]]:
            if k < j:
                assert lv[k] < lv[j]
    assert plan.info["n_levels"] == lv.max() + 1


def test_min_degree_pairs_and_fill():
    g = gg.grid("c1_1350bus")
    yb = gg.ybus(g)
    md = pf.Plan.from_ybus(yb, g.bus_type)
    nat = pf.Plan.from_ybus(yb, g.bus_type, ordering=pf.PF_ORDER_NATURAL)
    assert md.nnz_lu < 0.25 * nat.nnz_lu
    perm = md.order()
    npvpq = int((g.bus_type != gg.REF).sum())
    pv, pq = np.flatnonzero(g.bus_type == gg.PV), np.flatnonzero(g.bus_type == gg.PQ)
    ubus = np.r_[pv, pq, pq]
    pos = np.empty_like(perm); pos[perm] = np.arange(perm.size)
    # the |V| unknown of every PQ bus sits right after its angle
    for k, bus in enumerate(pq):
        assert pos[npvpq + k] == pos[len(pv) + k] + 1
    assert ubus[perm[0]] in np.r_[pv, pq]


def test_plan_info_and_workspace():
    g = gg.grid("c1_1350bus")
    plan = pf.Plan.from_ybus(gg.ybus(g), g.bus_type)
    info = plan.info
    assert info["n_bus"] == g.n and info["n_unknowns"] == info["n_pv"] + 2 * info["n_pq"]
    assert info["flops_refactor"] > info["nnz_lu"]
    assert info["bytes_iter_fp32"] < info["bytes_iter_fp64"]
    w64 = plan.workspace_bytes(10000)
    w32 = plan.workspace_bytes(10000, precision=pf.PF_FP32_LU)
    assert w64 > 10000 * info["nnz_lu"] * 8 and 0 < w32 < w64
    assert plan.workspace_bytes(10000, tile=7) == 0


@pytest.mark.parametrize("name", ["c0_14bus", "c4_100bus", "c1_1350bus"])
def test_level_histogram_recomputed_from_pattern(name):
    """pf_plan_levels against a recomputation from the L+U pattern alone: the level of
    column j is one more than the highest level among the columns k with U(k, j) != 0,
    and the update of column j by k costs one multiply-add per L entry of column k."""
    g = gg.grid(name)
    plan = pf.Plan.from_ybus(gg.ybus(g), g.bus_type)
    cp, ri, _ = plan.lu_pattern()
    N = plan.N
    lev = np.zeros(N, np.int64)
    nl = np.array([int(np.sum(ri[cp[k]:cp[k + 1]] > k)) for k in range(N)])
    madd = np.zeros(N, np.int64)
    for j in range(N):
        ks = ri[cp[j]:cp[j + 1]]
        ks = ks[ks < j]
        if ks.size:
            lev[j] = lev[ks].max() + 1
            madd[j] = nl[ks].sum()
    cols, madds = plan.levels()
    assert cols.shape[0] == plan.info["n_levels"] == lev.max() + 1
    assert np.array_equal(cols, np.bincount(lev))
    assert np.array_equal(madds, np.bincount(lev, weights=madd).astype(np.int64))
    assert madds.sum() == plan.info["flops_refactor"]


def test_pattern_hash_identifies_pattern_and_order():
    g = gg.grid("c4_100bus")
    yb = gg.ybus(g)
    a = pf.Plan.from_ybus(yb, g.bus_type).info["pattern_hash"]
    b = pf.Plan.from_ybus(yb, g.bus_type).info["pattern_hash"]
    nat = pf.Plan.from_ybus(yb, g.bus_type, ordering=pf.PF_ORDER_NATURAL).info["pattern_hash"]
    g2 = gg.grid("c4_1000bus")
    other = pf.Plan.from_ybus(gg.ybus(g2), g2.bus_type).info["pattern_hash"]
    bt = g.bus_type.copy()
    bt[np.flatnonzero(bt == gg.PQ)[0]] = gg.PV
    retyped = pf.Plan.from_ybus(yb, bt).info["pattern_hash"]
    assert a == b and a != 0
    assert len({a, nat, other, retyped}) == 4


def test_queue_without_device_reports_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(pf.PfError):
        pf.Queue()


@pytest.mark.parametrize("name", ["c4_100bus", "c1_1350bus", "c2_9000bus"])
@pytest.mark.parametrize("order", [0, 1])
def test_schedule_is_topological_and_slots_are_handed_out_in_order(name, order):
    """The refactorization's deadlock-freedom rests on two properties of each panel order:
    every column-to-column update source (U(k, j) != 0, k < j) lies in an earlier panel,
    and the long panels' ranks increase along the order, so that with any number L of
    long slots the panel of rank r - L, whose publication frees the slot of rank r, comes
    earlier.  Checked from the LU pattern, independently of the plan's own construction."""
    g = gg.grid(name)
    plan = pf.Plan.from_ybus(gg.ybus(g), g.bus_type)
    cp, ri, _ = plan.lu_pattern()
    first, width, rank, prev = plan.schedule(order)
    N = plan.N
    assert np.array_equal(np.sort(np.concatenate([np.arange(f, f + w) for f, w in zip(first, width)])), np.arange(N))
    pos = np.empty(N, np.int64)
    for q, (f, w) in enumerate(zip(first, width)):
        pos[f:f + w] = q
    for j in range(N):
        rows = ri[cp[j]:cp[j + 1]]
        srcs = rows[rows < j]                       # U part of column j: its update sources
        srcs = srcs[pos[srcs] != pos[j]]            # the pair's first column is internal
        assert (pos[srcs] < pos[j]).all(), j
    info = plan.info
    long_q = np.flatnonzero(rank >= 0)
    rows_of = (cp[first + 1] - cp[first])
    assert (rows_of[long_q] > info["slot_rows"]).all()
    assert (rows_of[rank < 0] <= info["slot_rows"]).all()
    assert np.array_equal(rank[long_q], np.arange(len(long_q)))       # ranks in order
    assert (prev[rank < 0] == -1).all()
    if len(long_q):
        assert prev[long_q[0]] == -1
        assert np.array_equal(prev[long_q[1:]], first[long_q[:-1]])   # previous long panel


def test_automatic_launch_configuration():
    """pf_resolve_opts (host logic): explicit choices are kept, invalid ones rejected, and
    the automatic choice picks the configurations measured fastest for the two workload
    shapes (many instances of a 1350-bus grid; few of a 9000-bus grid)."""
    g1 = gg.grid("c1_1350bus")
    p1 = pf.Plan.from_ybus(gg.ybus(g1), g1.bus_type)
    # per-phase FP64 on two or more generations of 16-instance tiles with four long slots:
    # 16 instances x 8 waves (23.0 ms against 23.9 ms for 8 x 16 on 10,000 instances);
    # fewer instances keep the latency model's 8 x 16
    assert (p1.resolve(10000)["tile"], p1.resolve(10000)["waves"], p1.resolve(10000)["long_slots"]) == (16, 8, 4)
    assert (p1.resolve(4000)["tile"], p1.resolve(4000)["waves"]) == (8, 16)
    assert (p1.resolve(10000, launch=pf.PF_LAUNCH_FUSED)["tile"], p1.resolve(10000, launch=pf.PF_LAUNCH_FUSED)["waves"]) == (8, 16)
    # grids of at least 10,000 LU entries: per-phase launches; small grids: one fused launch
    assert p1.resolve(10000)["launch"] == pf.PF_LAUNCH_PHASES
    assert p1.resolve(10000, launch=pf.PF_LAUNCH_FUSED)["launch"] == pf.PF_LAUNCH_FUSED
    g0 = gg.grid("c0_14bus")
    p0 = pf.Plan.from_ybus(gg.ybus(g0), g0.bus_type)
    assert p0.resolve(64)["launch"] == pf.PF_LAUNCH_FUSED
    r = p1.resolve(10000, precision=pf.PF_FP32_LU)
    assert (r["tile"], r["waves"]) == (16, 16)
    r = p1.resolve(10000, tile=4, waves=2, schedule=1)
    assert (r["tile"], r["waves"], r["schedule"]) == (4, 2, 1)
    g2 = gg.grid("c2_9000bus")
    p2 = pf.Plan.from_ybus(gg.ybus(g2), g2.bus_type)
    r = p2.resolve(2000)
    assert (r["tile"], r["waves"]) == (8, 16)
    assert r["launch"] == pf.PF_LAUNCH_PHASES
    # long slots: as many as keep the resident workgroups the batch can use.  Measured on
    # 10,000 scenarios of the 1350-bus grid: FP64 (8, 8) 31.4 / 29.1 / 27.6 ms with 2 / 3 /
    # 4 slots, (8, 16) with 8 slots 26.2 ms; FP32-LU (16, 8) 23.9 ms, (16, 16) with 8
    # slots 20.2 ms.  2,000 scenarios of the 9000-bus grid: FP64 (8, 16) 87.2 / 74.8 ms
    # with 2 / 3 slots (3 is the most that fit), FP32-LU (8, 16) 57.9 / 54.7 / 53.8 / 53.1 ms
    # with 6 / 8 / 10 / 11 (11 is the most that fit).
    assert p1.resolve(10000, launch=pf.PF_LAUNCH_FUSED)["long_slots"] == 8
    assert p1.resolve(4000)["long_slots"] == 8
    assert p1.resolve(10000, precision=pf.PF_FP32_LU)["long_slots"] == 8
    assert p2.resolve(2000)["long_slots"] == 3
    assert p2.resolve(2000, precision=pf.PF_FP32_LU)["long_slots"] == 11
    r = p1.resolve(10000, tile=8, waves=8)
    assert r["long_slots"] == 4                                  # two workgroups per CU kept
    assert p1.resolve(10000, long_slots=2)["long_slots"] == 2
    g0 = gg.grid("c0_14bus")
    assert pf.Plan.from_ybus(gg.ybus(g0), g0.bus_type).resolve(64)["long_slots"] == 0    # no long panel
    g4 = gg.grid("c4_100bus")
    p4 = pf.Plan.from_ybus(gg.ybus(g4), g4.bus_type)
    n_long_panels = int((p4.schedule(0)[2] >= 0).sum())
    assert p4.resolve(100, long_slots=12)["long_slots"] == min(12, n_long_panels)      # capped
    for bad in (dict(tile=32), dict(waves=3), dict(schedule=2), dict(precision=7), dict(long_slots=13),
                dict(long_slots=-1)):
        with pytest.raises(pf.PfError):
            p1.resolve(100, **bad)


@pytest.mark.parametrize("name", ["c1_1350bus", "c2_9000bus", "c4_3000bus"])
@pytest.mark.parametrize("order", [0, 1])
def test_long_panel_ring_never_reuses_rows_in_use(name, order):
    """The long panels' working columns share an LDS ring of n_long * 2 * max_col rows.
    A panel may start once every rank in its wait range has published; a panel that
    started has seen every rank its waits published before.  Safety: for every pair of
    long panels r' < r whose rows overlap, r' must be among the ranks guaranteed published
    when r starts (its wait range, and, transitively, theirs).  Liveness: waits only name
    earlier ranks.  Checked for every budget from the ring's own rows and offsets."""
    g = gg.grid(name)
    plan = pf.Plan.from_ybus(gg.ybus(g), g.bus_type)
    cp, _, _ = plan.lu_pattern()
    first, width, rank, _ = plan.schedule(order)
    long_q = np.flatnonzero(rank >= 0)
    size_expected = width[long_q] * (cp[first[long_q] + 1] - cp[first[long_q]])
    max_col = plan.info["max_col"]
    for n_long in range(1, 13):
        off, rows, lo, hi = plan.ring(order, n_long)
        cap = n_long * 2 * max_col
        assert np.array_equal(rows, size_expected)
        assert (off >= 0).all() and (off + rows <= cap).all()
        guaranteed = []
        for r in range(len(off)):
            assert lo[r] > hi[r] or (0 <= lo[r] and hi[r] < r)       # waits name earlier ranks only
            g_r = set()
            for b in range(lo[r], hi[r] + 1):
                g_r.add(b)
                g_r |= guaranteed[b]
            guaranteed.append(g_r)
            for rp in range(r):
                if off[rp] < off[r] + rows[r] and off[r] < off[rp] + rows[rp]:
                    assert rp in g_r, (n_long, r, rp)


def test_tune_cache_file_round_trip(tmp_path):
    """pf_tune_cache_save / _load: entries written to a text file come back with every key
    field and configuration intact (a second save is identical), a file that is not a cache
    is refused without touching the cache, and a missing file is an error."""
    pf.tune_cache_clear()
    assert pf.tune_cache_size() == 0
    src = tmp_path / "in.txt"
    src.write_text("pf_tune_cache 1\n"
                   "00000000000000aa 00000000000000bb 0 8 10000 10 0x1.5798ee2308c3ap-27 0 8 16 0 8 2 0 0x1.7p+4\n"
                   "00000000000000aa 00000000000000bb 1 0 2000 10 0x1.5798ee2308c3ap-27 1 16 16 1 11 1 1 0x1.1p+5\n")
    pf.tune_cache_load(str(src))
    assert pf.tune_cache_size() == 2
    out1, out2 = tmp_path / "a.txt", tmp_path / "b.txt"
    pf.tune_cache_save(str(out1))
    pf.tune_cache_clear()
    pf.tune_cache_load(str(out1))
    pf.tune_cache_save(str(out2))
    assert out1.read_text() == out2.read_text()
    rows = [ln.split() for ln in out1.read_text().splitlines()[1:]]
    assert [r[2:6] for r in rows] == [["0", "8", "10000", "10"], ["1", "0", "2000", "10"]]
    assert float.fromhex(rows[0][6]) == 1e-8 and float.fromhex(rows[1][14]) == 34.0
    assert rows[1][7:14] == ["1", "16", "16", "1", "11", "1", "1"]
    bad = tmp_path / "bad.txt"
    bad.write_text("pf_tune_cache 1\n00aa 00bb 0 8\n")
    with pytest.raises(pf.PfError, match="not a pf_tune cache"):
        pf.tune_cache_load(str(bad))
    assert pf.tune_cache_size() == 2
    with pytest.raises(pf.PfError):
        pf.tune_cache_load(str(tmp_path / "missing.txt"))
    pf.tune_cache_clear()
