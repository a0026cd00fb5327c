"""Seeded synthetic power grids and load/infeed scenarios.

This module only *draws inputs*: network topology, branch parameters, bus types, base
injections and Monte Carlo scenarios, plus the bus admittance matrix assembled from the
branch list (the input the batched solver receives, as in the paper's problem statement,
Sec. 3 / Eq. 1).  It contains no part of the power-flow method itself (no mismatch, no
Jacobian, no factorization), so both the CPU oracle and the GPU path can consume exactly
the same arrays.

Conventions (MATPOWER, as the paper follows):
  * bus types: PQ = 1, PV = 2, REF = 3;
  * pi-model branches: series admittance y_s = 1/(r + jx), total line charging b split
    b/2 at each end; no taps, phase shifters or bus shunts;
  * injections in per unit on the system base: PQ buses carry -(P_L + jQ_L), PV buses
    +P_G (Q unused), the REF bus is unused;
  * flat start: theta = 0 everywhere, |V| = 1 at PQ buses and the set-point at PV/REF.

Every random draw goes through ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Tuple

import numpy as np

PQ, PV, REF = 1, 2, 3


@dataclass
class Grid:
    name: str
    n: int
    f: np.ndarray          # int32 [m] from-bus of each branch
    t: np.ndarray          # int32 [m] to-bus of each branch
    r: np.ndarray          # float64 [m] series resistance (pu)
    x: np.ndarray          # float64 [m] series reactance (pu)
    b: np.ndarray          # float64 [m] total line charging susceptance (pu)
    bus_type: np.ndarray   # int8 [n]
    p_load: np.ndarray     # float64 [n] base active load (PQ buses only)
    q_load: np.ndarray     # float64 [n] base reactive load (PQ buses only)
    p_gen: np.ndarray      # float64 [n] base active generation (PV buses only)
    v_set: np.ndarray      # float64 [n] |V| set-point (PV and REF), 1.0 elsewhere
    scale: float = 1.0     # stress factor already applied to b and v_set; scales injections
    meta: Dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.f.shape[0])


@dataclass
class Ybus:
    """Bus admittance matrix in CSR form with sorted, unique column indices."""
    n: int
    row_ptr: np.ndarray    # int32 [n+1]
    col_idx: np.ndarray    # int32 [nnz]
    val: np.ndarray        # complex128 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])


@dataclass
class Scenarios:
    sbus: np.ndarray       # complex128 [B][n] specified injections
    v0: np.ndarray         # float64 [B][n][2] initial (|V|, theta)

    @property
    def batch(self) -> int:
        return int(self.sbus.shape[0])


# --------------------------------------------------------------------------- topology
def _tree_random_attachment(n: int, rng: np.random.Generator) -> List[Tuple[int, int]]:
    order = rng.permutation(n)
    edges = []
    for pos in range(1, n):
        parent = order[rng.integers(0, pos)]
        edges.append((int(order[pos]), int(parent)))
    return edges


def _geometric_edges(n: int, m: int, rng: np.random.Generator) -> Tuple[np.ndarray, List[Tuple[int, int]]]:
    """Spanning tree by nearest-earlier-node attachment, then chords drawn from
    6-nearest-neighbour pairs until the grid has m branches."""
    from scipy.spatial import cKDTree

    pts = rng.random((n, 2))
    order = rng.permutation(n)
    edges = set()
    placed = pts[order[:1]]
    for pos in range(1, n):
        node = order[pos]
        d2 = np.sum((placed - pts[node]) ** 2, axis=1)
        parent = order[int(np.argmin(d2))]
        edges.add((min(node, parent), max(node, parent)))
        placed = pts[order[: pos + 1]]
    tree = cKDTree(pts)
    _, nbr = tree.query(pts, k=7)
    cand = set()
    for i in range(n):
        for j in nbr[i, 1:]:
            j = int(j)
            if i != j:
                e = (min(i, j), max(i, j))
                if e not in edges:
                    cand.add(e)
    cand = sorted(cand)
    need = m - len(edges)
    if need > len(cand):
        raise ValueError("not enough nearest-neighbour chords for the requested degree")
    if need > 0:
        pick = rng.choice(len(cand), size=need, replace=False)
        for p in sorted(pick):
            edges.add(cand[p])
    return pts, sorted(edges)


def _finish_grid(name, n, edges, bus_type, rng, stress, meta, infeed_mean=1.0) -> Grid:
    m = len(edges)
    f = np.array([e[0] for e in edges], dtype=np.int32)
    t = np.array([e[1] for e in edges], dtype=np.int32)
    r = rng.uniform(0.01, 0.1, m)
    x = r * rng.uniform(2.0, 5.0, m)
    b = rng.uniform(0.0, 0.05, m)
    p_load = np.zeros(n)
    q_load = np.zeros(n)
    p_gen = np.zeros(n)
    v_set = np.ones(n)
    pq = np.flatnonzero(bus_type == PQ)
    pv = np.flatnonzero(bus_type == PV)
    ref = np.flatnonzero(bus_type == REF)
    p_load[pq] = rng.uniform(0.0, 0.5, pq.size)
    q_load[pq] = p_load[pq] * rng.uniform(0.2, 0.5, pq.size)
    p_gen[pv] = rng.uniform(0.2, 1.0, pv.size)
    v_set[pv] = rng.uniform(1.00, 1.05, pv.size)
    v_set[ref] = rng.uniform(1.00, 1.05, ref.size)
    # balance the expected generation (base P_G times the mean infeed factor of the
    # scenario distribution) against the total load, before any global scaling
    if pv.size and p_gen.sum() > 0:
        p_gen *= p_load.sum() / (infeed_mean * p_gen.sum())
    # stress factor: scales every departure from the trivial unloaded case (injections,
    # line charging and set-point deviations from 1 pu) by the same amount
    b = b * stress
    v_set = 1.0 + (v_set - 1.0) * stress
    meta = dict(meta, stress=float(stress))
    return Grid(name=name, n=n, f=f, t=t, r=r, x=x, b=b, bus_type=bus_type,
                p_load=p_load, q_load=q_load, p_gen=p_gen, v_set=v_set,
                scale=float(stress), meta=meta)


def make_tree_grid(n_pv: int, n_pq: int, n_chords: int, seed: int, stress: float = 1.0,
                   name: str = "tree") -> Grid:
    """Random spanning tree (random attachment) plus distinct random chords; bus 0 is REF."""
    rng = np.random.default_rng(seed)
    n = 1 + n_pv + n_pq
    tree = _tree_random_attachment(n, rng)
    edges = {(min(a, c), max(a, c)) for a, c in tree}
    while len(edges) < n - 1 + n_chords:
        a, c = (int(v) for v in rng.integers(0, n, 2))
        if a != c:
            edges.add((min(a, c), max(a, c)))
    bus_type = np.full(n, PQ, dtype=np.int8)
    bus_type[0] = REF
    pv = 1 + rng.choice(n - 1, size=n_pv, replace=False)
    bus_type[pv] = PV
    return _finish_grid(name, n, sorted(edges), bus_type, rng, stress,
                        {"topology": "tree+chords", "seed": seed}, infeed_mean=1.0)


def make_geometric_grid(n: int, avg_degree: float, pv_frac: float, seed: int,
                        stress: float = 1.0, name: str = "geo", infeed_mean: float = 0.6) -> Grid:
    """Meshed transmission-like grid on random points in the unit square.  The REF bus is
    the bus nearest the centre, relabelled to index 0."""
    rng = np.random.default_rng(seed)
    m = int(round(avg_degree * n / 2.0))
    pts, edges = _geometric_edges(n, m, rng)
    centre = int(np.argmin(np.sum((pts - 0.5) ** 2, axis=1)))
    relabel = np.arange(n)
    relabel[0], relabel[centre] = centre, 0
    inv = np.empty(n, dtype=np.int64)
    inv[relabel] = np.arange(n)
    edges = sorted({(min(inv[a], inv[c]), max(inv[a], inv[c])) for a, c in edges})
    edges = [(int(a), int(c)) for a, c in edges]
    bus_type = np.full(n, PQ, dtype=np.int8)
    bus_type[0] = REF
    n_pv = int(round(pv_frac * n))
    pv = 1 + rng.choice(n - 1, size=n_pv, replace=False)
    bus_type[pv] = PV
    return _finish_grid(name, n, edges, bus_type, rng, stress,
                        {"topology": "geometric", "seed": seed, "avg_degree": avg_degree},
                        infeed_mean=infeed_mean)


# --------------------------------------------------------------------------- admittance
def ybus(grid: Grid) -> Ybus:
    """Assemble the pi-model bus admittance matrix (CSR, sorted columns)."""
    n = grid.n
    ys = 1.0 / (grid.r + 1j * grid.x)
    ysh = 0.5j * grid.b
    rows = np.concatenate([grid.f, grid.t, grid.f, grid.t])
    cols = np.concatenate([grid.f, grid.t, grid.t, grid.f])
    vals = np.concatenate([ys + ysh, ys + ysh, -ys, -ys])
    key = rows.astype(np.int64) * n + cols
    uniq, inv = np.unique(key, return_inverse=True)
    acc = np.zeros(uniq.size, dtype=np.complex128)
    np.add.at(acc, inv, vals)
    r_idx = (uniq // n).astype(np.int32)
    c_idx = (uniq % n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(row_ptr, r_idx + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return Ybus(n=n, row_ptr=row_ptr, col_idx=c_idx, val=acc)


def ybus_outage(grid: Grid, k: int) -> Ybus:
    """Ybus of the grid with branch k out of service, on the full grid's pattern: the
    branch's pi-model contributions are subtracted, so its off-diagonal entries become
    explicit zeros (N-1 contingency cases share one sparsity pattern)."""
    full = ybus(grid)
    return Ybus(n=grid.n, row_ptr=full.row_ptr, col_idx=full.col_idx,
                val=ybus_outage_values(grid, full, np.array([k]))[0])


def ybus_outage_values(grid: Grid, full: Ybus, outages) -> np.ndarray:
    """complex128 [len(outages)][nnz]: the full Ybus values with branch outages[i] removed."""
    def pos(i, j):
        row = full.col_idx[full.row_ptr[i]:full.row_ptr[i + 1]]
        return full.row_ptr[i] + int(np.searchsorted(row, j))
    out = np.repeat(full.val[None, :], len(outages), axis=0)
    for i, k in enumerate(np.asarray(outages, dtype=np.int64)):
        f, t = int(grid.f[k]), int(grid.t[k])
        ys = 1.0 / (grid.r[k] + 1j * grid.x[k])
        ysh = 0.5j * grid.b[k]
        out[i, pos(f, f)] -= ys + ysh
        out[i, pos(t, t)] -= ys + ysh
        out[i, pos(f, t)] = 0.0
        out[i, pos(t, f)] = 0.0
    return out


def non_bridge_branches(grid: Grid) -> np.ndarray:
    """Branches whose outage leaves the grid connected (so every N-1 case keeps a
    solvable power flow structure)."""
    out = []
    for k in range(grid.f.size):
        adj = [[] for _ in range(grid.n)]
        for e in range(grid.f.size):
            if e != k:
                adj[grid.f[e]].append(grid.t[e])
                adj[grid.t[e]].append(grid.f[e])
        seen = np.zeros(grid.n, dtype=bool)
        stack = [0]
        seen[0] = True
        while stack:
            u = stack.pop()
            for w in adj[u]:
                if not seen[w]:
                    seen[w] = True
                    stack.append(w)
        if seen.all():
            out.append(k)
    return np.asarray(out, dtype=np.int64)


# --------------------------------------------------------------------------- scenarios
def flat_start(grid: Grid, batch: int) -> np.ndarray:
    v0 = np.zeros((batch, grid.n, 2))
    v0[:, :, 0] = np.where(grid.bus_type == PQ, 1.0, grid.v_set)[None, :]
    return v0


def make_scenarios(grid: Grid, count: int, seed: int, kind: str = "mc") -> Scenarios:
    """Monte Carlo scenarios.

    kind="uniform20": every load and generator scaled by its own N(1, 0.2) factor,
    clipped to [0.5, 1.5] (the 14-bus case).
    kind="mc": loads scaled per bus by N(1, 0.15) clipped to [0.5, 1.5]; PV infeed scaled
    per bus by Beta(2, 2) * 1.2 (renewable-like).
    """
    rng = np.random.default_rng(seed)
    n = grid.n
    pq = grid.bus_type == PQ
    pv = grid.bus_type == PV
    if kind == "uniform20":
        fl = np.clip(rng.normal(1.0, 0.2, (count, n)), 0.5, 1.5)
        fg = np.clip(rng.normal(1.0, 0.2, (count, n)), 0.5, 1.5)
    elif kind == "mc":
        fl = np.clip(rng.normal(1.0, 0.15, (count, n)), 0.5, 1.5)
        fg = rng.beta(2.0, 2.0, (count, n)) * 1.2
    else:
        raise ValueError(kind)
    s = grid.scale
    p = np.where(pv[None, :], s * grid.p_gen[None, :] * fg, 0.0)
    p = p - np.where(pq[None, :], s * grid.p_load[None, :] * fl, 0.0)
    q = -np.where(pq[None, :], s * grid.q_load[None, :] * fl, 0.0)
    sbus = p + 1j * q
    return Scenarios(sbus=sbus.astype(np.complex128), v0=flat_start(grid, count))


MEAN_INFEED = {"uniform20": 1.0, "mc": 0.6}   # E[N(1,0.2) clipped] = 1, E[Beta(2,2)*1.2] = 0.6


def base_case(grid: Grid, kind: str = "mc") -> Scenarios:
    """The base case: every scenario factor at its mean (loads x1, infeed x its mean)."""
    pq = grid.bus_type == PQ
    pv = grid.bus_type == PV
    s = grid.scale
    g = MEAN_INFEED[kind]
    p = np.where(pv, s * g * grid.p_gen, 0.0) - np.where(pq, s * grid.p_load, 0.0)
    q = -np.where(pq, s * grid.q_load, 0.0)
    return Scenarios(sbus=(p + 1j * q)[None, :].astype(np.complex128), v0=flat_start(grid, 1))


# --------------------------------------------------------------------------- workloads
# Stress factors kappa = 0.8**k: for each grid the largest power of 0.8 such that the base
# case converges from flat start in at most 5 Newton iterations and at least 99.5 % of
# three 400-scenario samples converge within 10 (the tests re-check the property against
# the CPU oracle on another sample).
GRID_SPECS = {
    "c0_14bus": dict(kind="tree", n_pv=4, n_pq=9, n_chords=7, seed=1000, stress=1.0),
    "c1_1350bus": dict(kind="geo", n=1350, avg_degree=2.8, pv_frac=0.15, seed=1001, stress=0.8 ** 13),
    "c2_9000bus": dict(kind="geo", n=9000, avg_degree=2.6, pv_frac=0.20, seed=1002, stress=0.8 ** 17),
    "c4_100bus": dict(kind="geo", n=100, avg_degree=2.8, pv_frac=0.15, seed=1041, stress=0.8 ** 9),
    "c4_1000bus": dict(kind="geo", n=1000, avg_degree=2.8, pv_frac=0.15, seed=1042, stress=0.8 ** 11),
    "c4_3000bus": dict(kind="geo", n=3000, avg_degree=2.8, pv_frac=0.15, seed=1043, stress=0.8 ** 15),
    "c4_9000bus": dict(kind="geo", n=9000, avg_degree=2.6, pv_frac=0.20, seed=1044, stress=0.8 ** 17),
}

# (grid, scenario count, scenario seed, scenario kind)
WORKLOADS = {
    "c0": [("c0_14bus", 64, 2000, "uniform20")],
    "c1": [("c1_1350bus", 10000, 2001, "mc")],
    "c2": [("c2_9000bus", 2000, 2002, "mc")],
    "c3_train": [("c1_1350bus", 50000, 3001, "mc")],
    "c3_eval": [("c1_1350bus", 10000, 3002, "mc")],
    "c4": [("c4_100bus", 4000, 2041, "mc"), ("c4_1000bus", 2000, 2042, "mc"),
           ("c4_3000bus", 1000, 2043, "mc"), ("c4_9000bus", 200, 2044, "mc")],
}

_GRID_CACHE: Dict[str, Grid] = {}


def grid(name: str) -> Grid:
    if name not in _GRID_CACHE:
        spec = dict(GRID_SPECS[name])
        kind = spec.pop("kind")
        if kind == "tree":
            _GRID_CACHE[name] = make_tree_grid(name=name, **spec)
        else:
            _GRID_CACHE[name] = make_geometric_grid(name=name, **spec)
    return _GRID_CACHE[name]


def workload(key: str, count: int | None = None):
    """Yield (grid, ybus, scenarios) for every grid of a named workload.  ``count`` caps
    the scenario count (the first ``count`` scenarios of the full seeded set)."""
    out = []
    for gname, cnt, seed, kind in WORKLOADS[key]:
        g = grid(gname)
        sc = make_scenarios(g, cnt, seed, kind)
        if count is not None and count < cnt:
            sc = Scenarios(sbus=sc.sbus[:count].copy(), v0=sc.v0[:count].copy())
        out.append((g, ybus(g), sc))
    return out
