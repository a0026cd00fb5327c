// One-time analysis of a Ybus pattern (Sec. 4.1 of the paper: the pre-order, the
// symbolic LU pattern and the static lookups are computed once and reused by every
// refactorization of every instance that shares the pattern).
//
//   * unknowns/equations: [angle of pv buses, angle of pq buses, |V| of pq buses], each
//     ascending by bus index (Eq. 2); equation r and unknown r belong to the same bus, so
//     the Jacobian pattern is structurally symmetric;
//   * pre-order: weighted minimum degree on the bus graph (a PQ bus carries two unknowns,
//     a PV bus one); both unknowns of a PQ bus are placed next to each other, so columns
//     come in pairs with identical patterns;
//   * symbolic factorization of A = P J P^T with diagonal pivots (the refactorization
//     keeps the permutation fixed, Sec. 4.1), via the elimination tree;
//   * the left-looking update lists (column j receives an update from every k < j with
//     U(k, j) != 0, Sec. 4.2 Alg. 2), with direct relative indexing of the targets;
//   * level sets of the column DAG (Sec. 4.3.1) and of the row DAG of the backward
//     substitution (Sec. 4.3.3).
#include <algorithm>
#include <cstring>
#include <numeric>

#include "pf_internal.h"

namespace pf {

namespace {

bool validate(int n, int nnzy, const int32_t *rp, const int32_t *ci, const int8_t *bt,
              std::string &err)
{
    if (n < 1) { err = "n_bus must be positive"; return false; }
    if (!rp || !ci || !bt) { err = "null pattern or bus_type pointer"; return false; }
    if (rp[0] != 0 || rp[n] != nnzy) { err = "row_ptr must start at 0 and end at nnz_y"; return false; }
    int nref = 0;
    for (int i = 0; i < n; i++) {
        if (bt[i] < PF_BUS_PQ || bt[i] > PF_BUS_REF) { err = "bus type out of range at bus " + std::to_string(i); return false; }
        if (bt[i] == PF_BUS_REF) nref++;
        if (rp[i + 1] < rp[i]) { err = "row_ptr not monotone"; return false; }
        bool diag = false;
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] < 0 || ci[p] >= n) { err = "column index out of range in row " + std::to_string(i); return false; }
            if (p > rp[i] && ci[p] <= ci[p - 1]) { err = "unsorted or duplicate columns in row " + std::to_string(i); return false; }
            if (ci[p] == i) diag = true;
        }
        if (!diag) { err = "row " + std::to_string(i) + " has no diagonal entry"; return false; }
        if (n > 1 && rp[i + 1] - rp[i] < 2) { err = "bus " + std::to_string(i) + " is isolated"; return false; }
    }
    if (nref != 1) { err = "exactly one REF bus is required (found " + std::to_string(nref) + ")"; return false; }
    for (int i = 0; i < n; i++)
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            int k = ci[p];
            if (!std::binary_search(ci + rp[k], ci + rp[k + 1], i)) {
                err = "pattern is not structurally symmetric at (" + std::to_string(i) + "," + std::to_string(k) + ")";
                return false;
            }
        }
    return true;
}

// Weighted minimum degree on the bus graph without the REF bus.  The degree of a bus is
// the number of unknowns of its current neighbours in the elimination graph; ties go to
// the smaller bus index.  Returns the buses in elimination order.
std::vector<int> bus_min_degree(const HostPlan &h)
{
    const int n = h.n;
    std::vector<std::vector<int>> adj(n);
    std::vector<int> w(n, 0);
    for (int i = 0; i < n; i++) {
        if (h.bus_type[i] == PF_BUS_REF) continue;
        w[i] = h.bus_type[i] == PF_BUS_PQ ? 2 : 1;
        for (int p = h.yrp[i]; p < h.yrp[i + 1]; p++) {
            int k = h.yci[p];
            if (k != i && h.bus_type[k] != PF_BUS_REF) adj[i].push_back(k);
        }
    }
    std::vector<long> deg(n, 0);
    std::vector<char> alive(n, 0);
    for (int i = 0; i < n; i++)
        if (w[i]) {
            alive[i] = 1;
            for (int k : adj[i]) deg[i] += w[k];
        }
    std::vector<int> out;
    out.reserve(n);
    std::vector<int> merged;
    for (;;) {
        int v = -1;
        for (int i = 0; i < n; i++)
            if (alive[i] && (v < 0 || deg[i] < deg[v])) v = i;
        if (v < 0) break;
        out.push_back(v);
        alive[v] = 0;
        const std::vector<int> nb = adj[v];
        for (int u : nb) {
            // adj[u] <- (adj[u] U nb) \ {u, v}
            merged.clear();
            std::set_union(adj[u].begin(), adj[u].end(), nb.begin(), nb.end(), std::back_inserter(merged));
            adj[u].clear();
            long d = 0;
            for (int x : merged)
                if (x != u && x != v) { adj[u].push_back(x); d += w[x]; }
            deg[u] = d;
        }
        adj[v].clear();
    }
    return out;
}

}  // namespace

int analyze(int n, int nnzy, const int32_t *row_ptr, const int32_t *col_idx,
            const int8_t *bus_type, int ordering, const int32_t *user_perm, HostPlan &h,
            std::string &err)
{
    if (!validate(n, nnzy, row_ptr, col_idx, bus_type, err)) return PF_EINVAL;
    h = HostPlan();
    h.n = n;
    h.nnzy = nnzy;
    h.yrp.assign(row_ptr, row_ptr + n + 1);
    h.yci.assign(col_idx, col_idx + nnzy);
    h.bus_type.assign(bus_type, bus_type + n);
    h.yrow.resize(nnzy);
    for (int i = 0; i < n; i++)
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; p++) h.yrow[p] = i;

    // ---- unknown numbering (Eq. 2)
    std::vector<int> th(n, -1), vm(n, -1);
    for (int i = 0; i < n; i++) {
        if (bus_type[i] == PF_BUS_PV) h.npv++;
        if (bus_type[i] == PF_BUS_PQ) h.npq++;
        if (bus_type[i] == PF_BUS_REF) h.ref = i;
    }
    h.npvpq = h.npv + h.npq;
    h.N = h.npvpq + h.npq;
    const int N = h.N;
    h.ubus.resize(N);
    int u = 0;
    for (int i = 0; i < n; i++) if (bus_type[i] == PF_BUS_PV) { th[i] = u; h.ubus[u++] = i; }
    for (int i = 0; i < n; i++) if (bus_type[i] == PF_BUS_PQ) { th[i] = u; h.ubus[u++] = i; }
    for (int i = 0; i < n; i++) if (bus_type[i] == PF_BUS_PQ) { vm[i] = u; h.ubus[u++] = i; }

    // ---- pre-order
    h.perm.resize(N);
    if (ordering == PF_ORDER_NATURAL) {
        std::iota(h.perm.begin(), h.perm.end(), 0);
    } else if (ordering == PF_ORDER_MIN_DEGREE) {
        int j = 0;
        for (int bus : bus_min_degree(h)) {
            h.perm[j++] = th[bus];
            if (vm[bus] >= 0) h.perm[j++] = vm[bus];
        }
        if (j != N) { err = "internal: ordering lost unknowns"; return PF_EINVAL; }
    } else if (ordering == PF_ORDER_USER) {
        if (!user_perm) { err = "PF_ORDER_USER needs user_perm"; return PF_EINVAL; }
        std::vector<char> seen(N, 0);
        for (int j = 0; j < N; j++) {
            int x = user_perm[j];
            if (x < 0 || x >= N || seen[x]) { err = "user_perm is not a permutation of the unknowns"; return PF_EINVAL; }
            seen[x] = 1;
            h.perm[j] = x;
        }
    } else {
        err = "unknown ordering";
        return PF_EINVAL;
    }
    h.pinv.resize(N);
    for (int j = 0; j < N; j++) h.pinv[h.perm[j]] = j;

    // ---- lower pattern of A = P J P^T, then symbolic LU via the elimination tree
    auto unknowns_of = [&](int bus, int *out) {
        int c = 0;
        if (th[bus] >= 0) out[c++] = th[bus];
        if (vm[bus] >= 0) out[c++] = vm[bus];
        return c;
    };
    std::vector<std::vector<int>> L(N);
    std::vector<std::vector<int>> children(N);
    std::vector<int> tmp, merged;
    for (int j = 0; j < N; j++) {
        int bus = h.ubus[h.perm[j]];
        tmp.clear();
        for (int p = h.yrp[bus]; p < h.yrp[bus + 1]; p++) {
            int uk[2];
            int c = unknowns_of(h.yci[p], uk);
            for (int a = 0; a < c; a++) {
                int r = h.pinv[uk[a]];
                if (r > j) tmp.push_back(r);
            }
        }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        for (int c : children[j]) {
            merged.clear();
            std::set_union(tmp.begin(), tmp.end(), L[c].begin(), L[c].end(), std::back_inserter(merged));
            tmp.clear();
            for (int r : merged) if (r != j) tmp.push_back(r);
        }
        L[j] = tmp;
        if (!L[j].empty()) children[L[j][0]].push_back(j);
    }
    std::vector<std::vector<int>> Up(N);   // Upat(j): k < j with j in L(k), ascending
    for (int k = 0; k < N; k++)
        for (int i : L[k]) Up[i].push_back(k);

    // ---- storage: column j = [U rows ascending, diagonal, L rows ascending]
    h.col_ptr.assign(N + 1, 0);
    h.col_diag.resize(N);
    for (int j = 0; j < N; j++) {
        h.col_diag[j] = (int)Up[j].size();
        h.col_ptr[j + 1] = h.col_ptr[j] + (int)(Up[j].size() + 1 + L[j].size());
        h.max_col = std::max(h.max_col, h.col_ptr[j + 1] - h.col_ptr[j]);
    }
    const int nnzlu = h.col_ptr[N];
    if (h.max_col >= (1 << 16)) { err = "an LU column exceeds 65535 entries"; return PF_EINVAL; }
    h.row_idx.resize(nnzlu);
    for (int j = 0; j < N; j++) {
        int e = h.col_ptr[j];
        for (int k : Up[j]) h.row_idx[e++] = k;
        h.row_idx[e++] = j;
        for (int i : L[j]) h.row_idx[e++] = i;
    }

    // ---- Jacobian descriptors: which Ybus entry and which derivative fills each slot
    h.desc.resize(nnzlu);
    for (int j = 0; j < N; j++) {
        int uc = h.perm[j];
        int bc = h.ubus[uc];
        int wrt_v = uc >= h.npvpq;
        for (int e = h.col_ptr[j]; e < h.col_ptr[j + 1]; e++) {
            int ue = h.perm[h.row_idx[e]];
            int be = h.ubus[ue];
            int is_q = ue >= h.npvpq;
            const int32_t *b0 = h.yci.data() + h.yrp[be], *b1 = h.yci.data() + h.yrp[be + 1];
            const int32_t *it = std::lower_bound(b0, b1, bc);
            if (it != b1 && *it == bc) {
                h.desc[e] = JacDesc{(int32_t)(it - h.yci.data()), be, bc, (is_q << 1) | wrt_v};
            } else {
                h.desc[e] = JacDesc{-1, be, bc, 0};
            }
        }
    }

    h.jpos.assign(h.nnzy, JPos{-1, -1, -1, -1});
    h.isj.assign(nnzlu, 0);
    for (int e = 0; e < nnzlu; e++) {
        const JacDesc &d = h.desc[e];
        if (d.p < 0) continue;
        h.isj[e] = 1;
        int32_t *slots = &h.jpos[d.p].pt;
        slots[d.kind] = e;
    }

    // ---- left-looking update lists with relative targets
    std::vector<int> where(N, -1);
    h.upd_ptr.assign(N + 1, 0);
    for (int j = 0; j < N; j++) {
        int cs = h.col_ptr[j];
        for (int e = cs; e < h.col_ptr[j + 1]; e++) where[h.row_idx[e]] = e - cs;
        for (int k : Up[j]) {
            Update up;
            const int lcnt = (int)L[k].size();
            up.krel_lcnt = where[k] | (lcnt << 16);
            up.lbeg = h.col_ptr[k] + h.col_diag[k] + 1;
            up.roff = (int)h.rel.size();
            up.k = k;
            for (int i : L[k]) {
                if (where[i] < 0) { err = "internal: symbolic pattern not closed"; return PF_EINVAL; }
                h.rel.push_back(where[i]);
            }
            h.upd.push_back(up);
            h.flops += lcnt;
        }
        h.upd_ptr[j + 1] = (int)h.upd.size();
        for (int e = cs; e < h.col_ptr[j + 1]; e++) where[h.row_idx[e]] = -1;
    }

    // ---- refactorization levels: level(j) = 1 + max level(k), k in Upat(j)
    h.level.assign(N, 0);
    int nlev = 0;
    for (int j = 0; j < N; j++) {
        int lv = 0;
        for (int k : Up[j]) lv = std::max(lv, h.level[k] + 1);
        h.level[j] = lv;
        nlev = std::max(nlev, lv + 1);
    }
    h.lev_ptr.assign(nlev + 1, 0);
    for (int j = 0; j < N; j++) h.lev_ptr[h.level[j] + 1]++;
    for (int l = 0; l < nlev; l++) h.lev_ptr[l + 1] += h.lev_ptr[l];
    h.lev_cols.resize(N);
    {
        std::vector<int> fillp(h.lev_ptr.begin(), h.lev_ptr.end() - 1);
        for (int j = 0; j < N; j++) h.lev_cols[fillp[h.level[j]]++] = j;
    }

    // ---- backward substitution rows: z_j = (y_j - sum_i U(j,i) z_i) / U(j,j), i in L(j)
    h.bs_ptr.assign(N + 1, 0);
    for (int j = 0; j < N; j++) {
        for (int i : L[j]) {
            // position of row j inside the U part of column i
            const std::vector<int> &ui = Up[i];
            int r = (int)(std::lower_bound(ui.begin(), ui.end(), j) - ui.begin());
            h.bs_pos.push_back(h.col_ptr[i] + r);
            h.bs_col.push_back(i);
        }
        h.bs_ptr[j + 1] = (int)h.bs_pos.size();
    }
    std::vector<int> blev(N, 0);
    int nb = 0;
    for (int j = N - 1; j >= 0; j--) {
        int lv = 0;
        for (int i : L[j]) lv = std::max(lv, blev[i] + 1);
        blev[j] = lv;
        nb = std::max(nb, lv + 1);
    }
    h.bs_lev_ptr.assign(nb + 1, 0);
    for (int j = 0; j < N; j++) h.bs_lev_ptr[blev[j] + 1]++;
    for (int l = 0; l < nb; l++) h.bs_lev_ptr[l + 1] += h.bs_lev_ptr[l];
    h.bs_lev_rows.resize(N);
    {
        std::vector<int> fillp(h.bs_lev_ptr.begin(), h.bs_lev_ptr.end() - 1);
        for (int j = 0; j < N; j++) h.bs_lev_rows[fillp[blev[j]]++] = j;
    }

    // ---- panels: (angle, |V|) pairs of one PQ bus with identical row lists
    h.panel_ptr.clear();
    for (int j = 0; j < N;) {
        h.panel_ptr.push_back(j);
        bool pair = false;
        if (j + 1 < N) {
            const int u0 = h.perm[j], u1 = h.perm[j + 1];
            if (u0 < h.npvpq && u1 >= h.npvpq && h.ubus[u0] == h.ubus[u1]) {
                const int n0 = h.col_ptr[j + 1] - h.col_ptr[j], n1 = h.col_ptr[j + 2] - h.col_ptr[j + 1];
                pair = n0 == n1 && h.col_diag[j + 1] == h.col_diag[j] + 1 &&
                       std::equal(h.row_idx.begin() + h.col_ptr[j], h.row_idx.begin() + h.col_ptr[j + 1],
                                  h.row_idx.begin() + h.col_ptr[j + 1]);
            }
        }
        j += pair ? 2 : 1;
    }
    h.panel_ptr.push_back(N);
    {
        const int np = (int)h.panel_ptr.size() - 1;
        std::vector<int> lk(np), bk(np);
        for (int q = 0; q < np; q++) {
            lk[q] = h.level[h.panel_ptr[q]];
            bk[q] = blev[h.panel_ptr[q + 1] - 1];
        }
        h.lu_seq.resize(np);
        h.bs_seq.resize(np);
        std::iota(h.lu_seq.begin(), h.lu_seq.end(), 0);
        std::iota(h.bs_seq.begin(), h.bs_seq.end(), 0);
        std::stable_sort(h.lu_seq.begin(), h.lu_seq.end(), [&](int a, int b) { return lk[a] < lk[b]; });
        std::stable_sort(h.bs_seq.begin(), h.bs_seq.end(), [&](int a, int b) {
            return bk[a] != bk[b] ? bk[a] < bk[b] : a > b;
        });

        // short working columns cover all but the longest ~4% of panels (at least 16 rows,
        // a multiple of 8); the rest share the launch's long slots
        std::vector<int> rows(np);
        for (int q = 0; q < np; q++) rows[q] = h.col_ptr[h.panel_ptr[q] + 1] - h.col_ptr[h.panel_ptr[q]];
        std::vector<int> sorted_rows(rows);
        std::sort(sorted_rows.begin(), sorted_rows.end());
        const int p96 = np ? sorted_rows[std::min(np - 1, (int)(0.96 * np))] : 0;
        h.slot_rows = std::max(16, (p96 + 7) / 8 * 8);
        if (h.slot_rows >= h.max_col) h.slot_rows = h.max_col;
        h.n_longp = 0;
        for (int q = 0; q < np; q++) h.n_longp += rows[q] > h.slot_rows;
        h.long_rank.assign((size_t)2 * np, -1);
        h.long_first.assign((size_t)2 * h.n_longp, -1);
        for (int order = 0; order < 2; order++) {
            int r = 0;
            for (int q = 0; q < np; q++) {
                const int pi = order == 0 ? h.lu_seq[q] : q;
                if (rows[pi] <= h.slot_rows) continue;
                h.long_rank[(size_t)order * np + pi] = r;
                h.long_first[(size_t)order * h.n_longp + r] = h.panel_ptr[pi];
                r++;
            }
        }
        if (h.n_longp >= (1 << 15)) { err = "too many long panels"; return PF_EINVAL; }
        // the LDS ring of the long panels, for every budget: rows are handed out in rank
        // order; a panel that does not fit before the end starts again at row 0; the ranks
        // that last held any of its rows must have published before it starts
        h.ring.assign((size_t)kMaxLong * 2 * h.n_longp, RingSlot{0, 1});
        std::vector<int> last;
        for (int nl = 1; nl <= kMaxLong; nl++) {
            const int cap = nl * 2 * h.max_col;
            for (int order = 0; order < 2; order++) {
                last.assign(cap, -1);
                int at = 0;
                for (int r = 0; r < h.n_longp; r++) {
                    const int j = h.long_first[(size_t)order * h.n_longp + r];
                    const int w = *std::upper_bound(h.panel_ptr.begin(), h.panel_ptr.end(), j) - j;
                    const int size = w * (h.col_ptr[j + 1] - h.col_ptr[j]);
                    if (at + size > cap) at = 0;
                    int lo = h.n_longp, hi = -1;
                    for (int u = at; u < at + size; u++) {
                        if (last[u] >= 0) { lo = std::min(lo, last[u]); hi = std::max(hi, last[u]); }
                        last[u] = r;
                    }
                    if (hi < 0) { lo = 1; hi = 0; }
                    h.ring[(((size_t)nl - 1) * 2 + order) * h.n_longp + r] = RingSlot{at, lo | (hi << 16)};
                    at += size;
                }
            }
        }
    }

    // ---- per-position panel descriptors of both orders
    {
        const int np = (int)h.panel_ptr.size() - 1;
        h.lu_desc.resize((size_t)2 * np);
        h.bs_desc.resize((size_t)2 * np);
        for (int order = 0; order < 2; order++)
            for (int q = 0; q < np; q++) {
                {
                    const int pi = order == 0 ? h.lu_seq[q] : q;
                    const int j = h.panel_ptr[pi];
                    const int two = h.panel_ptr[pi + 1] - j == 2;
                    h.lu_desc[(size_t)order * np + q] =
                        LuPanel{j | (two << 30), h.col_ptr[j], h.col_ptr[j + 1] - h.col_ptr[j], h.col_diag[j],
                                h.upd_ptr[j], h.upd_ptr[j + 1], h.long_rank[(size_t)order * np + pi], 0};
                }
                {
                    const int pi = order == 0 ? h.bs_seq[q] : np - 1 - q;
                    const int j = h.panel_ptr[pi];
                    const int two = h.panel_ptr[pi + 1] - j == 2;
                    const int jl = two ? j + 1 : j;
                    h.bs_desc[(size_t)order * np + q] =
                        BsPanel{j | (two << 30), h.col_ptr[j], two ? h.col_ptr[j + 1] : h.col_ptr[j], h.col_diag[j],
                                h.bs_ptr[jl], h.bs_ptr[jl + 1], 0, 0};
                }
            }
    }

    // ---- right-hand side and update maps
    h.bus_peq.assign(n, -1);
    h.bus_qeq.assign(n, -1);
    for (int i = 0; i < n; i++) {
        if (th[i] >= 0) h.bus_peq[i] = h.pinv[th[i]];
        if (vm[i] >= 0) h.bus_qeq[i] = h.pinv[vm[i]];
    }
    h.pos_upd.resize(N);
    for (int j = 0; j < N; j++) {
        int uu = h.perm[j];
        h.pos_upd[j] = h.ubus[uu] * 2 + (uu >= h.npvpq ? 1 : 0);
    }
    for (BsPanel &d : h.bs_desc) d.pu = h.pos_upd[d.j2 & ((1 << 30) - 1)];
    return PF_OK;
}

}  // namespace pf
