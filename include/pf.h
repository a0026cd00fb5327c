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
    int32_t n_panels;               /* panels: single columns and angle/|V| column pairs    */
    int32_t slot_rows;              /* rows of a wavefront's short working columns          */
    int32_t max_col;                /* longest column of L+U-I                              */
    int64_t n_updates;              /* column-to-column updates (k, j), U(k,j) != 0        */
    int64_t flops_refactor;         /* multiply-adds of one refactorization                */
    int64_t bytes_iter_fp64;        /* compulsory HBM bytes per instance-iteration, FP64   */
    int64_t bytes_iter_fp32;        /* the same with the LU data in FP32                    */
    uint64_t pattern_hash;          /* FNV-1a of sizes, bus types, Ybus pattern and order   */
} pf_plan_info_t;

/* Solver options; pass NULL for the defaults. */
typedef struct {
    int32_t precision;     /* PF_FP64 (default) or PF_FP32_LU: Jacobian, LU refactor and
                              substitutions in FP32; mismatch, convergence test and
                              voltage update in FP64 (inexact Newton)                      */
    int32_t tile;          /* instances per workgroup: 4, 8 or 16 (FP64), 8, 16 or 32
                              (FP32-LU); 0 = automatic                                     */
    int32_t waves;         /* wavefronts per workgroup (2, 4, 8 or 16); 0 = automatic       */
    int32_t schedule;      /* order in which wavefronts take the panels (single columns and
                              the angle/|V| column pairs of PQ buses): 0 = by level of the
                              column DAG (default), 1 = elimination order; both are
                              topological, results differ only by rounding order          */
    int32_t long_slots;    /* shared LDS working columns for the panels longer than
                              info.slot_rows (1..12): more let more of the serial tail of the
                              elimination overlap, at the cost of LDS; 0 = automatic (the
                              most that keep the resident workgroups the batch can use)    */
    int32_t launch;        /* PF_LAUNCH_AUTO (0), PF_LAUNCH_FUSED (1): one launch runs every
                              Newton iteration of a tile; PF_LAUNCH_PHASES (2): one launch per
                              phase and iteration (mismatch/Jacobian over all buses and
                              instances, refactorization per tile, back substitution per
                              tile), each with its own register budget.  Same results.
                              pf_solve_batch only; the other entry points run fused        */
    int32_t reorder;       /* PF_REORDER_AUTO (0): per-phase solves of several generations of
                              tiles run the first update over the whole batch, then order
                              the instances by the size of their first step, largest first:
                              the hardest finish in one fused launch of small tiles that
                              keep their CUs (their long iteration chains run at one tile's
                              latency beside the rest; with a fallback start the hardest
                              run their restart beside their first attempt, with the
                              results of the one-lane rule), the others in dense tiles.  Needs
                              the workspace size pf_workspace_bytes gives, else the
                              caller's order is kept.  PF_REORDER_OFF (1): keep the
                              caller's order.  An instance's results depend on its place
                              only through the rounding of the back substitution's sums,
                              whose split over lanes follows the tile size               */
    int32_t reserved;
} pf_solve_opts;
enum { PF_LAUNCH_AUTO = 0, PF_LAUNCH_FUSED = 1, PF_LAUNCH_PHASES = 2 };
enum { PF_REORDER_AUTO = 0, PF_REORDER_OFF = 1 };

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

/*
 * Level histogram of the refactorization's column DAG (Sec. 4.3.1: columns of one level
 * are independent; few columns per level make the serial region) [host, info.n_levels
 * entries each]: cols_per_level[l] columns at level l, and madds_per_level[l] (may be NULL)
 * the multiply-adds of their column updates (their sum is info.flops_refactor).
 */
int pf_plan_levels(pf_plan plan, int32_t *cols_per_level, int64_t *madds_per_level);

/* Elimination order [host, N entries]: perm[j] = unknown in position j of A = P J P^T. */
int pf_plan_order(pf_plan plan, int32_t *perm);

/*
 * Pattern of L+U-I in the plan's storage order [host]: col_ptr (N+1), row_idx (nnz_lu)
 * give, for each column j of A, its rows ascending (U rows, the diagonal, then L rows);
 * level [N] gives each column's refactorization level (0-based).
 */
int pf_plan_lu_pattern(pf_plan plan, int32_t *col_ptr, int32_t *row_idx, int32_t *level);

/*
 * The refactorization schedule of one panel order (order 0: by level, 1: elimination
 * order) [host, n_panels = info.n_panels entries each]: first[q] is the first column of
 * the q-th panel in that order and width[q] its column count (1, or 2 for the angle/|V|
 * pair of a PQ bus); long_rank[q] is -1 for a panel that uses its wavefront's short
 * working columns (at most info.slot_rows rows), else its rank among the order's long
 * panels, and prev_long[q] the first column of the long panel one rank earlier (-1: none).
 * A launch with L long slots (pf_solve_opts.long_slots) gives the long panel of rank r
 * slot r mod L once the one of rank r - L has published.  The kernel relies on: every
 * update source of a panel lies in an earlier panel of the order, and ranks increase
 * along the order (so every slot wait names an earlier panel).
 */
int pf_plan_schedule(pf_plan plan, int32_t order, int32_t *first, int32_t *width, int32_t *long_rank,
                     int32_t *prev_long);

/* Workspace bytes pf_solve_batch needs for `batch` instances with `opts` (NULL = default),
 * including the per-phase reorder area (16 B per instance and a few KB of counts). */
size_t pf_workspace_bytes(pf_plan plan, int32_t batch, const pf_solve_opts *opts);

/*
 * pf_plan_ring: where the refactorization keeps the working columns of each long panel
 * (more than slot_rows rows) for panel order `order` (0 level, 1 elimination) and an LDS
 * budget of n_long (1..12) pairs of max_col rows: an LDS ring of n_long * 2 * max_col
 * rows, handed out in rank order, wrapping to row 0 when a panel does not fit before the
 * end.  For each long rank r (0 .. n_long_panels - 1): offset[r] its first row, rows[r]
 * its row count (one column, or both columns of a pair), and the rank range
 * wait_lo[r] .. wait_hi[r] of earlier long panels that last held any of those rows and
 * must have published before it starts (empty when wait_lo > wait_hi).  Host arrays of
 * n_long_panels entries; PF_EINVAL for invalid arguments.
 */
int pf_plan_ring(pf_plan plan, int32_t order, int32_t n_long, int32_t *offset, int32_t *rows, int32_t *wait_lo,
                 int32_t *wait_hi);

/*
 * pf_resolve_opts: the configuration pf_solve_batch would use for batch instances with opts
 * (NULL = defaults): zero tile/waves/long_slots are replaced by the automatic choice, and
 * long_slots is capped at the number of long panels (0 when there are none).  PF_EINVAL
 * for invalid options or when nothing fits in LDS.
 */
int pf_resolve_opts(pf_plan plan, int32_t batch, const pf_solve_opts *opts, pf_solve_opts *out);

/*
 * pf_solve_batch -- `batch` Newton-Raphson power flows on the plan's pattern (Sec. 3).
 *   ybus [device]      nnz_y complex Ybus values in the pattern's order, shared by every
 *                      instance (ybus_batched = 0), or batch x nnz_y values, one set per
 *                      instance on the same pattern (ybus_batched = 1: N-1 contingency
 *                      cases, where an outaged branch leaves explicit zeros; Sec. 3,
 *                      the figure of the batched profile data, part c)
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
/*
 * pf_solve_batch_noalloc: pf_solve_batch without a workspace argument and without any
 * device allocation, for callers that cannot allocate (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  The workspace is a fixed 128 MiB
 * device array inside the library (one per device, held until the process ends); a call
 * whose pf_workspace_bytes(plan, batch, opts) exceeds it fails with PF_EINVAL and a
 * message, so split larger batches.  The plan must already be resident on the current
 * device (pf_analyze uploads it when a device is present), otherwise PF_EINVAL.  Same
 * kernels, inputs, outputs, stream ordering and results as pf_solve_batch.  Every call
 * on one device shares that array: calls that overlap in time on one device (two streams,
 * two threads) race and must be serialised by the caller.
 */
int pf_solve_batch_noalloc(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched,
                           const double *sbus, const double *v0, double tol, int32_t max_iter,
                           const pf_solve_opts *opts, double *v_out, int32_t *iters_out, uint8_t *converged_out,
                           int8_t *status_out, void *stream);

/*
 * pf_solve_batch_warm: pf_solve_batch from the start v0 (e.g. a learned prediction) with
 * an in-kernel fallback: an instance whose attempt from v0 fails (non-finite mismatch, an
 * update that does not reduce max|F|, or a zero pivot) restarts once from v_fallback
 * [device, B x n_bus x 2, same layout as v0; typically the flat start].  max_iter bounds
 * the voltage updates of each attempt, so the restart runs exactly as a plain solve from
 * v_fallback would (every instance that solve converges also converges here); iters_out
 * counts the updates of both attempts; status and converged describe the final attempt.
 * Other arguments and errors as pf_solve_batch.
 */
int pf_solve_batch_warm(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched,
                        const double *sbus, const double *v0, const double *v_fallback, double tol,
                        int32_t max_iter, const pf_solve_opts *opts, void *workspace,
                        size_t workspace_bytes, double *v_out, int32_t *iters_out, uint8_t *converged_out,
                        int8_t *status_out, void *stream);

int pf_eval_mismatch(pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                     const double *v, const pf_solve_opts *opts, void *workspace,
                     size_t workspace_bytes, double *f_out, double *normf_out, void *stream);
int pf_eval_factor(pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                   const double *v, const pf_solve_opts *opts, void *workspace,
                   size_t workspace_bytes, double *lu_out, void *stream);
int pf_eval_step(pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                 const double *v, const pf_solve_opts *opts, void *workspace,
                 size_t workspace_bytes, double *dx_out, void *stream);

/*
 * Learned warm start (an addition to the paper's method: a small network maps the
 * specified injections to initial voltages; Newton still iterates to the same tolerance,
 * so the network only changes the iteration count).  BF16 operands, FP32 accumulation;
 * all matrices row-major [device].
 *
 * pf_mlp_gemm: C[M][N] = op(A) op(B) with op(A) = A ([M][K]) or A^T (A stored [K][M]) when
 *   trans_a, op(B) = B ([K][N]) or B^T (B stored [N][K]) when trans_b; epilogue
 *   z = C + bias[n] (bias may be NULL) written to z_out (FP32, may be NULL), and
 *   act = GELU(z) (exact erf form) when gelu else z, written as BF16 and/or FP32 (either
 *   may be NULL).  Runs on the matrix cores.
 * pf_mlp_act_backward: dz = d_act * GELU'(z) (or d_act when !gelu), rounded to BF16, and
 *   db[n] = sum over rows of dz (FP32, may be NULL); [M][N].
 * pf_mlp_mse: grad = 2 (pred - target) / count; loss_parts[n_parts] partial sums of
 *   (pred - target)^2 / count (their sum is the loss).
 * pf_mlp_adam: one Adam step (bias-corrected, step >= 1) on FP32 master weights w with
 *   moments m, v; the BF16 copy w_bf16 (may be NULL) is refreshed.
 * pf_mlp_to_bf16: y = x rounded to nearest-even BF16.
 * pf_mlp_features: x_bf16 [batch][2 nf_bus] = z-scored (P, Q) of PQ buses and (P, |V| set-
 *   point) of PV buses listed in feat_bus (sbus, v0 as in pf_solve_batch; mu, sigma
 *   [2 nf_bus]).
 * pf_mlp_warm_v0: v0 [batch][n_bus][2] from the network output out [batch][2 nf_bus]
 *   ((|V|, angle) per feature bus, de-normalised with mu, sigma); PV |V| and the REF bus
 *   keep the set-points of v_set ([batch][n_bus][2]); non-finite outputs fall back to v_set.
 */
int pf_mlp_gemm(int32_t M, int32_t N, int32_t K, int32_t trans_a, int32_t trans_b, const uint16_t *a,
                const uint16_t *b, const float *bias, int32_t gelu, float *z_out, uint16_t *act_bf16_out,
                float *act_f32_out, void *stream);
int pf_mlp_act_backward(int32_t M, int32_t N, const float *d_act, const float *z, int32_t gelu,
                        uint16_t *dz_bf16, float *db, void *stream);
int pf_mlp_mse(int64_t count, const float *pred, const float *target, float *grad, float *loss_parts,
               int32_t n_parts, void *stream);
int pf_mlp_adam(int64_t n, float *w, uint16_t *w_bf16, const float *grad, float *m, float *v, float lr,
                float beta1, float beta2, float eps, int32_t step, void *stream);
int pf_mlp_to_bf16(int64_t n, const float *x, uint16_t *y, void *stream);
int pf_mlp_features(int32_t batch, int32_t n_bus, const double *sbus, const double *v0,
                    const int8_t *bus_type, const int32_t *feat_bus, int32_t nf_bus, const float *mu,
                    const float *sigma, uint16_t *x_bf16, void *stream);
int pf_mlp_warm_v0(int32_t batch, int32_t n_bus, const float *out, const int32_t *feat_bus,
                   int32_t nf_bus, const float *mu, const float *sigma, const int8_t *bus_type,
                   const double *v_set, double *v0, void *stream);

/*
 * Multi-pattern queue (an addition to the paper's method, which solves one grid per
 * launch): instances of several grids, each with its own plan and configuration, run in
 * one replayable graph.  Items that share precision, tile and waves form one persistent
 * kernel whose workgroups take tiles from a device counter, largest cost per tile first.
 *
 * pf_queue_create: an empty queue bound to the current device.
 * pf_queue_add: appends one item; arguments as in pf_solve_batch (opts selects precision,
 *   tile, waves, schedule and long slots, e.g. from pf_tune).  Each item keeps its own
 *   long-slot count; a group's kernel reserves the largest LDS of its items.
 *   done_ticks_out [device, may be NULL]
 *   receives, per instance, the device wall-clock ticks from the start of the run to the
 *   moment the instance's results were written (pf_queue_info gives the tick rate).  All
 *   pointers are borrowed: they must stay valid, and keep their addresses, for every
 *   later pf_queue_run.  An item with batch 0 is accepted and ignored.  Adding to a queue
 *   that has run makes the next run rebuild it.
 * pf_queue_run: enqueues the whole queue on stream (NULL = default stream).  The first run
 *   after an addition allocates the queue's workspace (device memory owned by the queue),
 *   uploads the items and builds the graph; later runs only replay it.  Runs of one queue
 *   share its workspace and counters and must not overlap.
 * pf_queue_destroy: waits for the device, then frees the graph and workspace.
 */
typedef struct pf_queue_s *pf_queue;
typedef struct {
    int32_t n_items, n_groups;     /* items added; persistent kernels of the built graph    */
    int32_t built;                 /* 1 when the graph is current                           */
    int32_t grid[18];              /* workgroups of each persistent kernel                  */
    int64_t n_tiles, n_instances;  /* over all items                                       */
    size_t workspace_bytes;        /* device memory held by the queue                      */
    double wall_clock_hz;          /* rate of the done_ticks clock                          */
} pf_queue_info_t;

int pf_queue_create(pf_queue *out);
int pf_queue_add(pf_queue queue, pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                 const double *v0, double tol, int32_t max_iter, const pf_solve_opts *opts, double *v_out,
                 int32_t *iters_out, uint8_t *converged_out, int8_t *status_out, uint64_t *done_ticks_out);
int pf_queue_run(pf_queue queue, void *stream);
int pf_queue_info(pf_queue queue, pf_queue_info_t *out);
void pf_queue_destroy(pf_queue queue);

/*
 * pf_tune: times every configuration (tile, waves, schedule, and long slots: the automatic
 * count for this batch and 2, 4, 8, each distinct count once) that fits in LDS on the given
 * instances (the same arguments as pf_solve_batch), in the single-launch form the queue
 * runs (launch = PF_LAUNCH_FUSED in best_out), with reps timed solves after one
 * untimed one, and returns the one with the most converged flows per second in best_out
 * (its mean ms per solve in best_ms_out, may be NULL).  A candidate whose untimed solve
 * converges fewer instances than the default configuration's, or reports PF_ST_INTERNAL,
 * is not timed.  waves = 0 tries every workgroup size, otherwise only that one.  Results
 * are cached in the process, keyed by the plan's pattern hash, device, precision, waves,
 * batch, tol and max_iter; flags & PF_TUNE_FORCE re-times a cached key.  Allocates and
 * frees its own device buffers; synchronises with stream.
 */
enum { PF_TUNE_FORCE = 1 };
int pf_tune(pf_plan plan, int32_t batch, const double *ybus, const double *sbus, const double *v0, double tol,
            int32_t max_iter, int32_t precision, int32_t waves, int32_t reps, int32_t flags,
            pf_solve_opts *best_out, double *best_ms_out, void *stream);

/*
 * The tuner's cache across processes.  A key is the plan's pattern hash, the device model
 * (its architecture name and CU count, not its ordinal), precision, waves, batch, max_iter
 * and tol, so a cache saved on one device applies to every device of the same kind.
 *   pf_tune_cache_save   writes every cached entry to the text file at path (replaced):
 *                        a header line, then one line per entry (key, configuration, ms)
 *   pf_tune_cache_load   adds the entries of such a file to the cache (an entry with the
 *                        same key is replaced); PF_EINVAL, cache unchanged, when the file
 *                        is missing or not such a file
 *   pf_tune_cache_clear  empties the cache;  pf_tune_cache_size: the number of entries
 * Host only; no device is needed.
 */
int pf_tune_cache_save(const char *path);
int pf_tune_cache_load(const char *path);
int pf_tune_cache_clear(void);
int32_t pf_tune_cache_size(void);

/*
 * pf_branch_flows: branch power flows and losses at voltages v (e.g. a solve's v_out), the
 * quantities a batch of scenarios is run for.  Pi-model branches: series admittance
 * 1/(r + jx), total line charging b_total split half per end.
 *   from_bus, to_bus [device]  n_branch bus indices (outside [0, n_bus): NaN flows)
 *   r, x, b_total [device]     n_branch per-unit parameters
 *   v [device]                 batch x n_bus x 2 (|V|, angle), as pf_solve_batch's v_out
 *   s_from, s_to [device]      out, batch x n_branch x 2 complex S at each end (pu)
 *   loss [device]              out, batch x 2 complex sum of S_from + S_to, or NULL
 * Stream-ordered; the caller owns every buffer.
 */
int pf_branch_flows(int32_t n_bus, int32_t n_branch, const int32_t *from_bus, const int32_t *to_bus,
                    const double *r, const double *x, const double *b_total, int32_t batch, const double *v,
                    double *s_from, double *s_to, double *loss, void *stream);

/*
 * pf_solve_host: pf_solve_batch for a batch that lives in host memory.  The batch is
 * solved in chunks of `chunk` instances on two internal streams, so that one chunk's
 * copies overlap the other's solve; all chunks use the configuration pf_resolve_opts gives
 * for `chunk` instances.  ybus [device] as in pf_solve_batch (shared values); sbus_host,
 * v0_host [host, batch x n_bus x 2] in; v_out_host [host, same shape], iters_host,
 * converged_host, status_host (may be NULL) [host, batch] out.  Host buffers should be
 * pinned (hipHostMalloc) for the copies to overlap; pageable memory works but copies
 * synchronously.  The work starts after what is already queued on stream; the call
 * returns when every result is in host memory.  Allocates and frees its own device
 * buffers and streams (default priority).
 */
int pf_solve_host(pf_plan plan, int32_t batch, const double *ybus, const double *sbus_host, const double *v0_host,
                  double tol, int32_t max_iter, const pf_solve_opts *opts, int32_t chunk, double *v_out_host,
                  int32_t *iters_host, uint8_t *converged_host, int8_t *status_host, void *stream);

/*
 * pf_cpu_solve_batch: the batched CPU engine (Sec. 4.2, Alg. 2 run over mini-batches; Sec.
 * 3.1): the same Newton iterations as pf_solve_batch in FP64 on the host, with the plan's
 * pre-order, pattern and update lists.  The batch is cut into mini-batches of 8 instances
 * stored side by side ([element][8]), so every inner loop is a SIMD operation over the
 * mini-batch (AVX-512, AVX2 or plain code, chosen at run time for the host CPU), and
 * `threads` worker threads (0 = every online core) take mini-batches from a shared
 * counter.  A separate engine for CPU hosts and a baseline for the GPU path: no GPU entry
 * point calls it.
 *   ybus [host]    nnz_y complex values (shared by the batch)
 *   sbus, v0 [host], v_out [host], iters_out, converged_out, status_out (may be NULL)
 *   [host]         as pf_solve_batch
 * Synchronous; needs no device.  PF_EINVAL for invalid arguments, PF_ENOMEM when a
 * thread's scratch (about 16 (nnz_lu + 6 n) * 8 bytes) cannot be allocated.
 */
int pf_cpu_solve_batch(pf_plan plan, int32_t batch, const double *ybus, const double *sbus, const double *v0,
                       double tol, int32_t max_iter, int32_t threads, double *v_out, int32_t *iters_out,
                       uint8_t *converged_out, int8_t *status_out);

/*
 * Second chance for instances whose refactorization failed (Sec. 3.2: a task that does not
 * converge because of numerical trouble in the LU refactorization is solved again with a
 * pivoting numerical factorization; Sec. 4.1: partial pivoting updates the row permutation
 * of Eq. 3 to avoid tiny pivots).  The GPU refactorization keeps the symmetric pre-order
 * and diagonal pivots and reports such an instance as PF_ST_PIVOT (a pivot that is not
 * finite, not above 1e-300 in magnitude, or below 1e-14 (FP64) / 1e-7 (FP32-LU) times the
 * largest magnitude in its column of A = P J P^T) or, when a bad step made the mismatch
 * non-finite, PF_ST_NONFINITE.
 *
 * pf_cpu_solve_pivoting: Newton-Raphson in FP64 on the host with a fresh left-looking
 * Gilbert-Peierls LU with threshold partial pivoting every iteration (the diagonal row is
 * kept while its magnitude is at least 0.1 times the column's largest candidate; fill
 * follows the pivots), same stopping rules and outputs as pf_solve_batch.
 *   ybus [host]  nnz_y complex values, or batch x nnz_y when ybus_batched
 *   sbus, v0, v_out, iters_out, converged_out, status_out (may be NULL) [host] as
 *                pf_solve_batch; threads = 0 uses every online core.
 * Synchronous; needs no device.  PF_EINVAL for invalid arguments, PF_ENOMEM.
 *
 * pf_solve_fallback: after a pf_solve_batch(_warm) call with the same arguments (device
 * pointers, same stream), waits for the stream, reads status_out and re-solves every
 * instance reporting PF_ST_PIVOT or PF_ST_NONFINITE from its v0 as pf_cpu_solve_pivoting
 * does, on the host (only those instances' inputs are copied), then writes its V,
 * iteration count, flag and status back over the GPU result.  status_out is required.
 * *n_resolved (may be NULL) receives the number of instances re-solved.  Synchronous with
 * respect to the host; PF_EDEVICE when a copy or the synchronisation fails.
 */
int pf_cpu_solve_pivoting(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched,
                          const double *sbus, const double *v0, double tol, int32_t max_iter, int32_t threads,
                          double *v_out, int32_t *iters_out, uint8_t *converged_out, int8_t *status_out);
int pf_solve_fallback(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched, const double *sbus,
                      const double *v0, double tol, int32_t max_iter, int32_t threads, double *v_out,
                      int32_t *iters_out, uint8_t *converged_out, int8_t *status_out, int32_t *n_resolved,
                      void *stream);

/* Release the plan and its device memory. */
void pf_plan_destroy(pf_plan plan);

/* Message for the last failing call on this thread ("" if none). */
const char *pf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
