// Internal data structures shared by the host analysis and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pf.h"

namespace pf {

// Jacobian entry descriptor of one L+U-I slot: the Ybus entry p = (i, k) it derives
// from, the buses i (equation) and k (unknown), and the kind: bit 1 = Q equation (else
// P), bit 0 = derivative w.r.t. |V| (else angle).  p = -1 marks a fill slot.
struct JacDesc {
    int32_t p, i, k, kind;
};

// LU positions of the four Jacobian entries that one Ybus entry (i, k) produces.
struct JPos {
    int32_t pt, pv, qt, qv;
};

// One column-to-column update of the left-looking refactorization: column j receives
// LU(r, j) -= LU(k, j) * LU(r, k) for every r in the L part of column k.
struct Update {
    int32_t krel_lcnt;  // position of row k inside column j | (number of L entries of k) << 16
    int32_t lbeg;       // absolute entry index of the first L entry of column k
    int32_t roff;       // offset into rel[]: relative target positions in column j
    int32_t k;          // source column
};

// Everything one refactorization panel needs, in processing order (one load per panel):
// first column with the pair flag in bit 30, first entry and entry count of the column,
// position of the diagonal inside it, the column's update range, and its rank among the
// order's long panels (-1: short; see HostPlan::long_rank).
struct LuPanel {
    int32_t j2, cs, cnt, dr, u0, u1, lrank, pad;
};

// The same for back substitution: first row with the pair flag in bit 30, first entries of
// the panel's columns, diagonal position, range of the last row's U entries in bs_col /
// bs_pos, and the update target (bus * 2 + is |V|) of the first row.
struct BsPanel {
    int32_t j2, cs, cs1, dr, q0, q1, pu, pad;
};


// Most shared long working-column slots of a launch: the LDS budget of the long panels is
// n_long (1..kMaxLong) times a pair of columns of max_col rows.
constexpr int kMaxLong = 12;

// A long panel's place in the LDS ring (see HostPlan::ring): its first row, and the range
// lo (bits 0-15) .. hi (bits 16-31) of earlier long ranks it waits for (lo > hi: none).
struct RingSlot {
    int32_t off, blk;
};

// Everything pf_analyze derives from the pattern, on the host.
struct HostPlan {
    int n = 0, nnzy = 0, npv = 0, npq = 0, npvpq = 0, N = 0, ref = -1;
    std::vector<int32_t> yrp, yci, yrow;          // Ybus pattern; row of every entry
    std::vector<int8_t> bus_type;
    std::vector<int32_t> ubus;                    // unknown -> bus
    std::vector<int32_t> perm, pinv;              // position j of A -> unknown; inverse
    // L+U-I storage, column-major by position j: U rows ascending, diagonal, L rows ascending
    std::vector<int32_t> col_ptr;                 // N+1
    std::vector<int32_t> col_diag;                // N, relative position of the diagonal
    std::vector<int32_t> row_idx;                 // nnz_lu
    std::vector<JacDesc> desc;                    // nnz_lu Jacobian descriptors
    // per Ybus entry (i, k): LU positions of dP_i/dangle_k, dP_i/d|V_k|, dQ_i/dangle_k,
    // dQ_i/d|V_k| (-1 where the equation or unknown does not exist); per LU position: 1 if
    // it holds a Jacobian entry, 0 for fill
    std::vector<JPos> jpos;
    std::vector<uint8_t> isj;
    // refactorization updates, per column j in ascending k
    std::vector<int32_t> upd_ptr;                 // N+1
    std::vector<Update> upd;
    std::vector<int32_t> rel;                     // relative targets (one per multiply-add)
    // level schedules
    std::vector<int32_t> lev_ptr, lev_cols;       // refactorization levels (columns)
    std::vector<int32_t> level;                   // level of each column
    std::vector<int32_t> bs_lev_ptr, bs_lev_rows; // backward-substitution levels (rows)
    // backward substitution: for row j, the entries U(j, i), i > j
    std::vector<int32_t> bs_ptr, bs_pos, bs_col;
    // panels: a PQ bus's angle and |V| columns (adjacent, same row list) form a 2-column
    // supernode; every other column is a panel of its own
    std::vector<int32_t> panel_ptr;               // first column of each panel, then N
    // processing orders of the panels: by refactorization level (a topological order of
    // the column DAG) and by back-substitution level (topological for the row DAG)
    std::vector<int32_t> lu_seq, bs_seq;
    // working columns of the refactorization: a panel of at most slot_rows rows uses its
    // wavefront's own pair of short columns; a longer panel takes rows of the launch's
    // shared LDS ring (its budget is chosen per launch from the LDS left over).  For each
    // of the two panel orders (level, elimination): the rank of each panel among the
    // order's long panels (-1 for a short panel) and the first column of the long panel of
    // each rank; ranks follow the order, so the ring is handed out in topological order.
    int slot_rows = 0, n_longp = 0;
    std::vector<int32_t> long_rank;               // [2][n_panels]
    std::vector<int32_t> long_first;              // [2][n_longp]
    // The long panels' working columns are packed into an LDS ring of n_long * 2 * max_col
    // rows, each panel taking exactly its own rows (one column, or both of a pair), handed
    // out in rank order and wrapping to the start when the end is reached.  For each
    // budget n_long, order and rank: the panel's first row in the ring and the range of
    // earlier ranks (lo, hi) whose rows it reuses; it starts once every rank in that range
    // has published.  ring[((n_long - 1) * 2 + order) * n_longp + rank] = {offset,
    // lo | hi << 16}, lo > hi when no rank precedes it there.
    std::vector<RingSlot> ring;                   // [kMaxLong][2][n_longp]
    // per order (0: level, 1: elimination) and position in that order
    std::vector<LuPanel> lu_desc;                 // [2][n_panels]
    std::vector<BsPanel> bs_desc;                 // [2][n_panels]
    // right-hand side and update maps
    std::vector<int32_t> bus_peq, bus_qeq;        // bus -> position of its P / Q equation, -1
    std::vector<int32_t> pos_upd;                 // position j -> bus * 2 + (unknown is |V|)
    int max_col = 0;
    int64_t flops = 0;
};

// Device copy of what the kernels read of the plan: one allocation, pointers into it.
struct DevPlan {
    int n, nnzy, N, nnzlu, max_col;
    const int32_t *yrp, *yci;
    const JPos *jpos;
    const uint8_t *isj;
    const int32_t *rel;
    const Update *upd;
    const int32_t *bs_pos, *bs_col;
    const int32_t *bus_peq, *bus_qeq;
    const LuPanel *lu_desc;
    const BsPanel *bs_desc;
    const RingSlot *ring;
    int n_panels, slot_rows, n_longp;
};

struct Plan {
    HostPlan h;
    DevPlan d{};
    void *dev_mem = nullptr;
    size_t dev_bytes = 0;
    const int32_t *perm_dev = nullptr;
    int device = 0;
};

// host analysis (pf_plan.cpp)
int analyze(int n, int nnzy, const int32_t *row_ptr, const int32_t *col_idx,
            const int8_t *bus_type, int ordering, const int32_t *user_perm, HostPlan &out,
            std::string &err);

void set_error(const std::string &msg);

// batched CPU engine (pf_cpu.cpp): host arrays, threads = 0 uses every online core
int cpu_solve(const HostPlan &h, int32_t batch, const double *ybus, const double *sbus, const double *v0, double tol,
              int32_t max_iter, int32_t threads, double *v_out, int32_t *iters_out, uint8_t *conv_out,
              int8_t *status_out, std::string &err);

}  // namespace pf
