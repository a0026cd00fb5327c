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

// One column-to-column update of the left-looking refactorization: column j receives
// LU(r, j) -= LU(k, j) * LU(r, k) for every r in the L part of column k.
struct Update {
    int32_t krel_lcnt;  // position of row k inside column j | (number of L entries of k) << 16
    int32_t lbeg;       // absolute entry index of the first L entry of column k
    int32_t roff;       // offset into rel[]: relative target positions in column j
    int32_t k;          // source column
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
    // right-hand side and update maps
    std::vector<int32_t> bus_peq, bus_qeq;        // bus -> position of its P / Q equation, -1
    std::vector<int32_t> pos_upd;                 // position j -> bus * 2 + (unknown is |V|)
    int max_col = 0;
    int64_t flops = 0;
};

// Device copy of the plan: one allocation, pointers into it.
struct DevPlan {
    int n, nnzy, N, nnzlu, n_levels, n_bs_levels, max_col, npvpq;
    const int32_t *yrp, *yci, *yrow;
    const int8_t *bus_type;
    const int32_t *col_ptr, *col_diag;
    const JacDesc *desc;
    const int32_t *upd_ptr, *rel;
    const Update *upd;
    const int32_t *lev_ptr, *lev_cols, *bs_lev_ptr, *bs_lev_rows;
    const int32_t *bs_ptr, *bs_pos, *bs_col;
    const int32_t *bus_peq, *bus_qeq, *pos_upd;
    const int32_t *panel_ptr, *lu_seq, *bs_seq;
    int n_panels;
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

}  // namespace pf
