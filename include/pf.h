/*
 * pf.h -- C ABI of the batched Newton-Raphson AC power-flow solver for AMD MI355X (gfx950).
 *
 * The solver runs many power flows that share one bus admittance matrix (Ybus) sparsity
 * pattern, the setting of Wang, Wende-von Berg and Braun, "Fast parallel Newton-Raphson
 * power flow solver for large number of system calculations with CPU and GPU" (Sec. 3):
 * each instance finds V such that the calculated nodal power S = V o conj(Ybus V)
 * (Eq. 1) matches the specified injections, by Newton iterations of
 *   mismatch -> Jacobian update -> LU refactorization -> forward/backward substitution
 *   -> voltage update                                                  (Sec. 3, Eq. 2)
 * with a fill-reducing pre-order and the symbolic LU pattern analysed once per pattern
 * (Sec. 4.1, Eq. 3).
 *
 * Conventions common to every call:
 *   * All indices are int32 and 0-based.  Bus types use the MATPOWER codes below.
 *   * Complex numbers are interleaved (re, im) pairs of doubles.
 *   * Host pointers are marked [host]; bulk data are [device] pointers (for instance the
 *     data_ptr of framework tensors).  The caller owns every buffer; the library owns
 *     only the opaque plan.
 *   * Calls that take a stream (hipStream_t passed as void*, NULL = the null stream) are
 *     stream-ordered and asynchronous: outputs are valid after the stream synchronises.
 *   * Return codes: PF_OK or a negative PF_E* code; pf_last_error() gives a message
 *     (thread-local) for the last failing call.  No exception crosses the ABI.
 *   * Per-instance numerical failure is not an error: it is reported per instance through
 *     converged_out = 0 and status_out.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_plan_s *pf_plan;

enum { PF_BUS_PQ = 1, PF_BUS_PV = 2, PF_BUS_REF = 3 };
enum { PF_ORDER_NATURAL = 0, PF_ORDER_MIN_DEGREE = 1, PF_ORDER_USER = 2 };
enum { PF_FP64 = 0, PF_FP32_LU = 1 };
enum { PF_OK = 0, PF_EINVAL = -1, PF_ENOMEM = -2, PF_EDEVICE = -3, PF_ESTRUCT = -4 };
/* Per-instance status.  PF_ST_INTERNAL: the kernel's bounded dataflow wait expired (a
   library defect, never expected); the instance's result is invalid. */
enum { PF_ST_CONVERGED = 0, PF_ST_MAXITER = 1, PF_ST_NONFINITE = 2, PF_ST_PIVOT = 3,
       PF_ST_INTERNAL = -1 };

/* Sizes of an analysed pattern. */
typedef struct {
    int32_t n_bus, n_pv, n_pq;      /* buses; n_bus - n_pv - n_pq = 1 (the REF bus)        */
    int32_t n_unknowns;             /* N = n_pv + 2 n_pq: [angle pv,pq ; |V| pq]  (Eq. 2) */
    int32_t nnz_y, nnz_j, nnz_lu;   /* Ybus, Jacobian, L+U-I pattern sizes                 */
    int32_t n_levels;               /* column levels of the refactorization DAG (Sec. 4.3) */
    int32_t n_bs_levels;            /* row levels of the backward substitution             */
    int32_t max_col;                /* longest column of L+U-I                              */
    int64_t n_updates;              /* column-to-column updates (k, j), U(k,j) != 0        */
    int64_t flops_refactor;         /* multiply-adds of one refactorization                */
    int64_t bytes_iter_fp64;        /* compulsory HBM bytes per instance-iteration, FP64   */
    int64_t bytes_iter_fp32;        /* the same with the LU data in FP32                    */
} pf_plan_info_t;

/* Solver options; pass NULL for the defaults. */
typedef struct {
    int32_t precision;     /* PF_FP64 (default) or PF_FP32_LU: Jacobian, LU refactor and
                              substitutions in FP32; mismatch, convergence test and
                              voltage update in FP64 (inexact Newton)                      */
    int32_t tile;          /* instances per workgroup (8, 16 or 32); 0 = automatic          */
    int32_t waves;         /* wavefronts per workgroup (1..8); 0 = automatic                */
    int32_t reserved[5];
} pf_solve_opts;

/*
 * pf_analyze -- one-time analysis of a Ybus pattern (Sec. 4.1: pre-order, symbolic LU
 * and static lookups are built once and reused by every refactorization).
 *   n_bus, nnz_y       sizes of the pattern
 *   row_ptr [host]     n_bus + 1 entries, CSR row pointers
 *   col_idx [host]     nnz_y entries, strictly increasing within each row
 *   bus_type [host]    n_bus entries, PF_BUS_PQ / PF_BUS_PV / PF_BUS_REF
 *   ordering           PF_ORDER_NATURAL, PF_ORDER_MIN_DEGREE or PF_ORDER_USER
 *   user_perm [host]   for PF_ORDER_USER: N entries, user_perm[j] = unknown eliminated
 *                      j-th; NULL otherwise
 *   out                receives the plan (device memory is allocated on the current device)
 * Rejects with PF_EINVAL: not exactly one REF bus, a bus type out of range, a row without
 * its diagonal, unsorted or duplicate columns, a pattern that is not structurally
 * symmetric, an isolated bus, an invalid user permutation.
 */
int pf_analyze(int32_t n_bus, int32_t nnz_y, const int32_t *row_ptr, const int32_t *col_idx,
               const int8_t *bus_type, int32_t ordering, const int32_t *user_perm, pf_plan *out);

/* Sizes of the plan (host struct). */
int pf_plan_info(pf_plan plan, pf_plan_info_t *out);

/* Elimination order [host, N entries]: perm[j] = unknown in position j of A = P J P^T. */
int pf_plan_order(pf_plan plan, int32_t *perm);

/*
 * Pattern of L+U-I in the plan's storage order [host]: col_ptr (N+1), row_idx (nnz_lu)
 * give, for each column j of A, its rows ascending (U rows, the diagonal, then L rows);
 * level [N] gives each column's refactorization level (0-based).
 */
int pf_plan_lu_pattern(pf_plan plan, int32_t *col_ptr, int32_t *row_idx, int32_t *level);

/* Workspace bytes pf_solve_batch needs for `batch` instances with `opts` (NULL = default). */
size_t pf_workspace_bytes(pf_plan plan, int32_t batch, const pf_solve_opts *opts);

/*
 * pf_solve_batch -- `batch` Newton-Raphson power flows on the plan's pattern (Sec. 3).
 *   ybus [device]      nnz_y complex Ybus values in the pattern's order
 *   ybus_batched       must be 0 (one Ybus shared by every instance)
 *   sbus [device]      [batch][n_bus] complex specified injections (pu): P at PV and PQ
 *                      buses, Q at PQ buses are used; the rest is ignored
 *   v0 [device]        [batch][n_bus][2] initial (|V|, angle in rad); |V| at PV and REF
 *                      buses and the REF angle are the fixed set-points
 *   tol, max_iter      stop when max |mismatch| < tol (tested before every update), or
 *                      after max_iter updates
 *   workspace [device] at least pf_workspace_bytes(plan, batch, opts) bytes, 256-B aligned
 *   v_out [device]     [batch][n_bus][2] final (|V|, angle)
 *   iters_out [device] [batch] voltage updates performed
 *   converged_out [device] [batch] 1 if the tolerance was met
 *   status_out [device] [batch] PF_ST_* (may be NULL)
 * Every instance runs independently; a non-finite value or a zero pivot in one instance
 * affects no other.
 */
int pf_solve_batch(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched,
                   const double *sbus, const double *v0, double tol, int32_t max_iter,
                   const pf_solve_opts *opts, void *workspace, size_t workspace_bytes,
                   double *v_out, int32_t *iters_out, uint8_t *converged_out,
                   int8_t *status_out, void *stream);

/*
 * Single-step entry points for checking the stages of one Newton iteration at a given V
 * (same kernels, same workspace contract as pf_solve_batch):
 *   pf_eval_mismatch: f_out [device] [batch][N] mismatch in unknown order
 *                     ([dP pv,pq ; dQ pq], calculated minus specified, Alg. 1) and
 *                     normf_out [device] [batch] its infinity norm.
 *   pf_eval_factor:   lu_out [device] [batch][nnz_lu] values of L+U-I of A = P J(V) P^T
 *                     in the order of pf_plan_lu_pattern (unit diagonal of L implied).
 *   pf_eval_step:     dx_out [device] [batch][N] solution of J(V) dx = F(V) in unknown
 *                     order (so that V_new = V - dx).
 */
int pf_eval_mismatch(pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                     const double *v, const pf_solve_opts *opts, void *workspace,
                     size_t workspace_bytes, double *f_out, double *normf_out, void *stream);
int pf_eval_factor(pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                   const double *v, const pf_solve_opts *opts, void *workspace,
                   size_t workspace_bytes, double *lu_out, void *stream);
int pf_eval_step(pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                 const double *v, const pf_solve_opts *opts, void *workspace,
                 size_t workspace_bytes, double *dx_out, void *stream);

/* Release the plan and its device memory. */
void pf_plan_destroy(pf_plan plan);

/* Message for the last failing call on this thread ("" if none). */
const char *pf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
