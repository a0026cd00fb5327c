// Batched Newton-Raphson power flow on gfx950: one fused kernel per launch.
//
// A workgroup owns a tile of T instances and runs their whole Newton loop (Sec. 3 of
// the paper) without leaving the kernel:
//   M   rectangular V, then one pass over every Ybus row: I = Y V, S = V o conj(I)
//       (Eq. 1), F = calculated - specified (Alg. 1), and from the same Y_ik V_k products
//       the four Jacobian entries of each Ybus entry (Sec. 3.1.2), written straight into
//       their positions of the permuted matrix A = P J P^T; the per-instance infinity
//       norm by wavefront shuffles and an LDS reduction, and the convergence decision;
//   LU  a sync-free dataflow form of the left-looking refactorization (Sec. 4.2-4.3):
//       wavefronts take panels (a column, or the angle/|V| column pair of a PQ bus) in a
//       topological order, round-robin; each loads its Jacobian values into LDS working
//       columns, applies the update of every column k with U(k,j) != 0 in ascending k as
//       soon as k is published (the sparse multiply-add of Alg. 3 with direct indexing),
//       carries the forward substitution of the right-hand side along, normalises the L
//       part, writes the columns back and publishes them.  This extends the paper's
//       second stage (partial updates of unfinished columns) to every column: no level
//       barriers remain and the serial tail pipelines across wavefronts;
//   BS  backward substitution in the same dataflow style (a row waits for the rows it
//       reads), and the voltage update V <- V - dx for instances still iterating.
// Each entry of every per-instance array is stored tile-interleaved: element e of
// instance t of a tile lives at [e][t], so a wavefront reading entry e for the tile's
// instances issues one contiguous T * sizeof(real) access (the paper's batched layout,
// Sec. 3.1, at tile granularity).  Inside a wavefront the 64 lanes are T instances x
// (64 / T) sub-lanes that split the rows of a column (the paper's extra multiply-add
// parallelism).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "pf_internal.h"
#include "pf_math.h"

namespace pf {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

enum Mode { MODE_SOLVE = 0, MODE_MISMATCH = 1, MODE_FACTOR = 2, MODE_STEP = 3 };

constexpr int kMBlock = 256;     // threads of a mismatch-kernel workgroup (per-phase launches)
// admittance entries whose operands the per-phase mismatch kernel loads together
// (1350-bus grid, 10,000 instances, FP64 solves in the given order: 27.1 ms one at a time,
// 25.4 with two, 25.5 with three, 26.5 with four, 27.5 with eight: more entries hold more
// registers, and fewer wavefronts fit)
constexpr int kMRow = 2;
constexpr size_t kBsZBytes = 48 * 1024;   // wide per-phase back substitution: LDS for z of the tail
constexpr int kPhasesMinLu = 10000;       // automatic launch form: per-phase from this many LU entries
constexpr int UPD_GROUP = 3;     // column updates whose operand loads are issued together
constexpr int L_ROWS = 2;        // rows of each source column per lane loaded with its group
// the same, and the panel rows prefetched per lane, in the per-phase refactorization kernel
// (measured there: four updates per group 1-2% faster than three or five; three or four
// source rows per lane, or three prefetched panel rows, 1-5% slower)
constexpr int kWideGroup = 4, kWideLRows = 2, kWideARows = 2;

struct KArgs {
    DevPlan p;
    const int32_t *perm;        // position -> unknown (device)
    const double *ybus;         // [nnzy][2], or [B][nnzy][2] with ybus_stride = 2 nnzy
    size_t ybus_stride;         // doubles between instances' Ybus values (0: shared)
    const double *sbus;         // [B][n][2]
    const double *v0;           // [B][n][2]
    const double *v_fb;         // [B][n][2] restart point after a failed first attempt (may be null)
    double tol;
    int max_iter, batch, mode;
    int n_long;                 // LDS budget of the long panels' ring, in pairs of max_col rows
    char *ws;
    size_t tile_bytes, off_y, off_vec;   // byte offsets inside one tile's block
    size_t off_ctl, off_part;   // per-phase launches: instance states and tile flags; mismatch maxima
    int nbb;                    // per-phase launches: bus blocks of the mismatch kernel
    double *v_out;
    int32_t *iters_out;
    uint8_t *conv_out;
    int8_t *status_out;
    double *aux_out;            // F, LU or dx for the single-step modes
    double *aux2_out;           // max |F| for MODE_MISMATCH
    unsigned long long *done_ticks;        // per-instance completion tick (may be null)
    const unsigned long long *t0;          // start tick the completion ticks are relative to
    int sched;                  // 0: level order, 1: elimination order
    // per-phase launches: the instance held by each slot (tile * T + lane) when the batch has
    // been reordered; null = slot b holds instance b
    const int32_t *inst;
    // a fused launch that resumes a reordered batch: |V| and angle rows and control words
    // parked after its first update, in instance order; with paired attempts, the first
    // pair_slots slots hold two per instance (a multiple of the tile size)
    const double *vpark;
    const int4 *cpark;
    int pair_slots;
    // per-phase back substitution: LDS bytes for z of the highest positions
    int bs_zbytes;
};

__device__ __forceinline__ int inst_of(const KArgs &a, int slot) { return a.inst ? a.inst[slot] : slot; }

// Waits until every vector memory load this wavefront has issued has returned (vmcnt(0);
// the encoding leaves the other counters unconstrained).  The memory counter also counts
// stores, so a wait for a register loaded in an earlier loop iteration (whose distance
// in operations the compiler cannot count) becomes a wait for everything, stores
// included.  Placed where only loads are outstanding, this wait lets the compiler see
// that nothing loaded is pending at the loop's back edge.
__device__ __forceinline__ void wait_loads_returned() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Publication flags of the dataflow phases: one LDS byte per column (row).  A producer
// makes its global writes visible to the workgroup (release fence) and then every lane of
// the wavefront stores the same flag byte (plain stores, no atomics, so the loops stay free
// of lane-divergent regions).  A consumer polls the byte uniformly across the wavefront
// and acquires.
//
// Every wait is bounded by progress, not by time: each wavefront counts its own
// publications in an LDS word (only that wavefront writes it, so plain stores suffice), and
// a waiter restarts its poll count whenever the sum over the workgroup's wavefronts has
// moved.  Only kNoProgressPolls polls in a row with no publication anywhere in the
// workgroup (about 0.1 s; a panel publishes within microseconds) raise the tile's error
// flag and end the wait, so a wrong schedule can only produce an error status, never a
// hang, while a slow but progressing tile always completes.
constexpr unsigned kNoProgressPolls = 1u << 22;
constexpr unsigned kProgressCheck = 256;       // polls between reads of the progress words

template <int NW>
__device__ __forceinline__ int progress_sum(const int *prog)
{
    int s = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) s += __hip_atomic_load(&prog[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return __builtin_amdgcn_readfirstlane(s);
}

// The slow path of a wait: called after a poll found the condition unmet.  Returns true
// when the wait must end (error raised here or by another wavefront).
template <int NW>
__device__ __forceinline__ bool wait_tick(unsigned &spins, int &seen, const int *prog, int *err)
{
    const int e = __builtin_amdgcn_readfirstlane(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (e) return true;
    if ((++spins & (kProgressCheck - 1)) == 0) {
        const int now = progress_sum<NW>(prog);
        if (now != seen) {
            seen = now;
            spins = 0;
        } else if (spins >= kNoProgressPolls) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return true;
        }
    }
    __builtin_amdgcn_s_sleep(1);
    return false;
}

template <int NW>
__device__ __forceinline__ void wait_published(unsigned char *flags, int j, const int *prog, int *err)
{
    unsigned spins = 0;
    int seen = -1;
    for (;;) {
        const int f = __builtin_amdgcn_readfirstlane(
            (int)__hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (f || wait_tick<NW>(spins, seen, prog, err)) break;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The same wait for an LDS counter to reach a value (counters only grow).
template <int NW>
__device__ __forceinline__ void wait_count(int *ctr, int target, const int *prog, int *err)
{
    unsigned spins = 0;
    int seen = -1;
    for (;;) {
        const int v = __builtin_amdgcn_readfirstlane(__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (v >= target || wait_tick<NW>(spins, seen, prog, err)) break;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// A wavefront records one more publication in its progress word.
__device__ __forceinline__ void note_progress(int *prog, int wave, int &count)
{
    __hip_atomic_store(&prog[wave], ++count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Per-tile state shared by the phases of the Newton loop: the tile's arrays, the LDS
// working areas and flags, and the lane's place in the workgroup.
template <typename R>
struct TileCtx {
    const KArgs &a;
    int tid, wave, lane, t, s;
    bool valid;
    R *LU, *Yv;
    double *Vm, *Va;
    R *short_base, *long_base, *ysl, *ysl1, *cmx, *cmx1;
    unsigned char *done, *ldone;
    int *err, *s_prog, *s_piv;
    const int *s_active, *s_reset;
    int &nprog;                         // this wavefront's publications so far
    R *zlds;                            // back substitution: z of positions >= zb in LDS
    int zb;                             // (zb = N: none)
};

// ---- refactorization with the forward substitution carried along (Sec. 4.2-4.3): the
// Jacobian values are in the tile's LU array and the right-hand sides in Yv; on return every
// panel has published (or the tile's error flag is set) and s_piv marks failed pivots.
// WIDE: the per-phase kernel, which has registers to spare, keeps more loads in flight
// (four rows per sub-lane per round trip for a long panel's own rows and for a source
// column's rows beyond the group load); the fused kernel is at its register limit.
template <typename R, int T, int NW, bool WIDE>
__device__ __forceinline__ void lu_phase(TileCtx<R> &cx)
{
    constexpr int SL = 64 / T;
    constexpr int NT = NW * 64;
    // panel rows per lane whose loads are issued together; updates per operand group and
    // rows of each source column per lane loaded with it (more in the per-phase kernel)
    constexpr int A_ROWS = WIDE ? kWideARows : 2;
    constexpr int UG = WIDE ? kWideGroup : UPD_GROUP;
    constexpr int LR = WIDE ? kWideLRows : L_ROWS;
    const KArgs &a = cx.a;
    const DevPlan &P = a.p;
    const int tid = cx.tid, wave = cx.wave, lane = cx.lane, t = cx.t, s = cx.s;
    const bool valid = cx.valid;
    const int N = P.N;
    R *const LU = cx.LU;
    R *const Yv = cx.Yv;
    R *const short_base = cx.short_base, *const long_base = cx.long_base;
    R *const ysl = cx.ysl, *const ysl1 = cx.ysl1, *const cmx = cx.cmx, *const cmx1 = cx.cmx1;
    unsigned char *const done = cx.done, *const ldone = cx.ldone;
    int *const err = cx.err, *const s_prog = cx.s_prog, *const s_piv = cx.s_piv;
    int &nprog = cx.nprog;
    for (int w = tid; w < N + P.n_longp; w += NT)
        __hip_atomic_store(&done[w], (unsigned char)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    // Panels (one column, or the angle/|V| pair of a PQ bus sharing one row list) in
    // level order, round-robin over the wavefronts.  The order is topological, so the
    // earliest unfinished panel always has every source published and some wavefront
    // always makes progress; level order keeps independent panels side by side.
    // The loads of a panel's Jacobian values and right-hand sides do not depend on any
    // other panel (only the panel itself rewrites its columns and rows), so they are
    // software-pipelined: while a wavefront works on one panel, the loads of its next
    // panel are in flight.  A_ROWS rows per lane travel this way; longer panels load
    // their remaining rows when they start.
    //
    // Metadata travels in vector registers instead of scalar loads (a scalar load is
    // counted together with LDS operations, so every LDS wait would also wait for it):
    // one load brings the descriptors of the wavefront's next 8 panels (lane l holds
    // word l % 8 of descriptor l / 8) and one load 16 update records of a panel (lane l
    // holds word l % 4 of record l / 4); fields are read with readlane.  A panel's first
    // 16 records arrive with its prefetch; a panel with more loads each further chunk
    // one chunk ahead of its use, so no update group waits for its own records.
    const LuPanel *lud = P.lu_desc + (size_t)a.sched * P.n_panels;
    auto desc_chunk = [&](int c) -> int {
        const int qq = wave + NW * (8 * c + (lane >> 3));
        return reinterpret_cast<const int *>(lud)[(size_t)qq * 8 + (lane & 7)];   // padded table
    };
    auto desc_from = [&](int chunk, int k) -> LuPanel {
        LuPanel d;
        int *w = reinterpret_cast<int *>(&d);
#pragma unroll
        for (int f = 0; f < 8; f++) w[f] = __builtin_amdgcn_readlane(chunk, k * 8 + f);
        return d;
    };
    // records [ua, ua + 16); only those below the panel's end are read back (the table
    // is padded by one chunk)
    auto upd_chunk_at = [&](int ua) -> int { return reinterpret_cast<const int *>(P.upd)[(size_t)ua * 4 + lane]; };
    auto upd_chunk = [&](const LuPanel &d) -> int { return upd_chunk_at(d.u0); };
    R pa0[A_ROWS], pa1[A_ROWS], py0 = 0, py1 = 0;
    unsigned char pf[A_ROWS];
    int pupd = 0;
    auto prefetch = [&](const LuPanel &d) {
        pupd = upd_chunk(d);
        const int jn = d.j2 & ((1 << 30) - 1);
        const bool tw = (d.j2 >> 30) & 1;
#pragma unroll
        for (int r = 0; r < A_ROWS; r++) {
            const int e = min(s + r * SL, d.cnt - 1);      // rows past the end re-read the last
            pf[r] = P.isj[d.cs + e];
            pa0[r] = LU[(size_t)(d.cs + e) * T + t];
            pa1[r] = LU[(size_t)(d.cs + (tw ? d.cnt : 0) + e) * T + t];
        }
        py0 = Yv[jn * T + t];
        py1 = Yv[(jn + (tw ? 1 : 0)) * T + t];
    };
    int dch0 = desc_chunk(0), dch1 = desc_chunk(1);
    LuPanel pdc = desc_from(dch0, 0);         // the current panel's descriptor, kept in
    if (wave < P.n_panels) prefetch(pdc);     // scalar registers across iterations
    wait_loads_returned();
    for (int q = wave, qi = 0; q < P.n_panels; q += NW, qi++) {
        const int kq = qi & 7;
        const LuPanel pd = pdc;
        const int ucur = pupd;
        const int j = pd.j2 & ((1 << 30) - 1);
        const bool two = (pd.j2 >> 30) & 1;
        const int cs = pd.cs, cnt = pd.cnt, dr = pd.dr;
        const bool more = q + NW < P.n_panels;
        const LuPanel pdn = kq < 7 ? desc_from(dch0, kq + 1) : desc_from(dch1, 0);
        if (kq == 7) {
            dch0 = dch1;
            dch1 = desc_chunk((qi >> 3) + 2);
        }
        R *xw, *xw1;
        if (pd.lrank < 0) {
            xw = short_base + (size_t)wave * 2 * P.slot_rows * T;
            xw1 = xw + (size_t)P.slot_rows * T;
        } else {
            // a long panel takes its own rows of the ring once every earlier long panel
            // that last held any of them has published (ranks follow the topological
            // order); the entry is read with a per-lane address so that it is a vector
            // load (a scalar load would share its counter with the LDS operations)
            const int rw = reinterpret_cast<const int *>(
                P.ring + ((size_t)(a.n_long - 1) * 2 + a.sched) * P.n_longp + pd.lrank)[lane & 1];
            const int roff = __builtin_amdgcn_readlane(rw, 0), rblk = __builtin_amdgcn_readlane(rw, 1);
            for (int rr = rblk & 0xffff; rr <= (rblk >> 16); rr++) wait_published<NW>(ldone, rr, s_prog, err);
            xw = long_base + (size_t)roff * T;
            xw1 = xw + (size_t)cnt * T;
        }
        // the panel's Jacobian values (written by the mismatch pass; fill positions read
        // as zero; both columns of a pair share the row list and the fill pattern) and
        // right-hand sides
        {
            R cm0 = 0, cm1 = 0;
#pragma unroll
            for (int r = 0; r < A_ROWS; r++) {
                const int e = s + r * SL;
                if (e < cnt) {
                    const R a0 = pf[r] ? pa0[r] : (R)0, a1 = pf[r] ? pa1[r] : (R)0;
                    xw[e * T + t] = a0;
                    if (two) xw1[e * T + t] = a1;
                    cm0 = fmax(cm0, fabs(a0));
                    cm1 = fmax(cm1, fabs(a1));
                }
            }
            if (s == 0) {
                ysl[t] = py0;
                if (two) ysl1[t] = py1;
            }
            if constexpr (WIDE) {
                // rows past the end read the following entries of the tile's block and the
                // padded flag table, and are discarded
                for (int e0 = s + A_ROWS * SL; e0 < cnt; e0 += 4 * SL) {
                    R v0[4], v1[4];
                    bool fe[4];
#pragma unroll
                    for (int x = 0; x < 4; x++) {
                        const int e = e0 + x * SL;
                        fe[x] = P.isj[cs + e];
                        v0[x] = LU[(size_t)(cs + e) * T + t];
                        v1[x] = LU[(size_t)(cs + (two ? cnt : 0) + e) * T + t];
                    }
#pragma unroll
                    for (int x = 0; x < 4; x++) {
                        const int e = e0 + x * SL;
                        if (e < cnt) {
                            const R a0 = fe[x] ? v0[x] : (R)0, a1 = fe[x] ? v1[x] : (R)0;
                            xw[e * T + t] = a0;
                            if (two) xw1[e * T + t] = a1;
                            cm0 = fmax(cm0, fabs(a0));
                            cm1 = fmax(cm1, fabs(a1));
                        }
                    }
                }
            } else {
                for (int e = s + A_ROWS * SL; e < cnt; e += SL) {
                    const bool fe = P.isj[cs + e];
                    const R v0 = LU[(size_t)(cs + e) * T + t];
                    const R v1 = two ? LU[(size_t)(cs + cnt + e) * T + t] : (R)0;
                    const R a0 = fe ? v0 : (R)0, a1 = fe ? v1 : (R)0;
                    xw[e * T + t] = a0;
                    if (two) xw1[e * T + t] = a1;
                    cm0 = fmax(cm0, fabs(a0));
                    cm1 = fmax(cm1, fabs(a1));
                }
            }
            // the column maxima over the instance's sub-lanes, kept in LDS until the pivots
#pragma unroll
            for (int off = T; off < 64; off <<= 1) {
                cm0 = fmax(cm0, __shfl_xor(cm0, off));
                cm1 = fmax(cm1, __shfl_xor(cm1, off));
            }
            if (s == 0) {
                cmx[t] = cm0;
                cmx1[t] = cm1;
            }
        }
        if (more) prefetch(pdn);
        pdc = pdn;
        // Updates in ascending source order.  After waiting for the first pending source,
        // the run of following updates whose sources are already published (up to
        // UG, within one chunk of records) has its operand loads issued together
        // (LR rows of each source column per lane), then the updates are applied one
        // after another in LDS (the order of the arithmetic is unchanged).  Rows beyond
        // LR per lane (the long source columns of the dense tail) are loaded two at a
        // time.
        const int u0 = pd.u0, u1 = pd.u1;
        int ubase = u0, uc0 = ucur, uc1 = 0;
        if (u1 - u0 > 16) uc1 = upd_chunk_at(u0 + 16);
        auto upd_rec = [&](int u) -> Update {
            const int r = u - ubase;
            Update x;
            x.krel_lcnt = __builtin_amdgcn_readlane(uc0, 4 * r);
            x.lbeg = __builtin_amdgcn_readlane(uc0, 4 * r + 1);
            x.roff = __builtin_amdgcn_readlane(uc0, 4 * r + 2);
            x.k = __builtin_amdgcn_readlane(uc0, 4 * r + 3);
            return x;
        };
        for (int ub = u0; ub < u1;) {
            if (ub - ubase >= 16) {
                ubase += 16;
                uc0 = uc1;
                if (u1 - ubase > 16) uc1 = upd_chunk_at(ubase + 16);
            }
            Update ups[UG];
            ups[0] = upd_rec(ub);
            wait_published<NW>(done, ups[0].k, s_prog, err);
            int gcnt = 1;
#pragma unroll
            for (int g = 1; g < UG; g++) {
                if (gcnt == g && ub + g < u1 && ub + g - ubase < 16) {
                    ups[g] = upd_rec(ub + g);
                    const int f = __builtin_amdgcn_readfirstlane((int)__hip_atomic_load(
                        &done[ups[g].k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                    if (f) gcnt = g + 1;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            R lv[UG][LR], yk[UG];
            int rv[UG][LR];
#pragma unroll
            for (int g = 0; g < UG; g++) {
                yk[g] = 0;
#pragma unroll
                for (int e = 0; e < LR; e++) { lv[g][e] = 0; rv[g][e] = -1; }
                if (g < gcnt) {
                    const int lcnt = ups[g].krel_lcnt >> 16;
#pragma unroll
                    for (int e = 0; e < LR; e++)
                        if (s + e * SL < lcnt) {
                            lv[g][e] = LU[(size_t)(ups[g].lbeg + s + e * SL) * T + t];
                            rv[g][e] = P.rel[ups[g].roff + s + e * SL];
                        }
                    yk[g] = Yv[ups[g].k * T + t];
                }
            }
            wave_sync();
#pragma unroll
            for (int g = 0; g < UG; g++) {
                if (g < gcnt) {
                    const Update up = ups[g];
                    const int krel = up.krel_lcnt & 0xffff, lcnt = up.krel_lcnt >> 16;
                    const R m0 = xw[krel * T + t];
                    const R m1 = two ? xw1[krel * T + t] : (R)0;
                    const R ykg = yk[g];
                    // row tr of the panel's columns (and its right-hand side) minus the
                    // multipliers times the source column's entry l
                    auto apply = [&](int tr, R l) {
                        xw[tr * T + t] = fma(-m0, l, xw[tr * T + t]);
                        if (two) xw1[tr * T + t] = fma(-m1, l, xw1[tr * T + t]);
                        if (tr == dr) ysl[t] = fma(-l, ykg, ysl[t]);
                        else if (two && tr == dr + 1) ysl1[t] = fma(-l, ykg, ysl1[t]);
                    };
#pragma unroll
                    for (int e = 0; e < LR; e++)
                        if (rv[g][e] >= 0) apply(rv[g][e], lv[g][e]);
                    if constexpr (WIDE) {
                        // rows past the column's end read the following entries and the
                        // padded target table, and are discarded
                        for (int r = s + LR * SL; r < lcnt; r += 4 * SL) {
                            R lx[4];
                            int tx[4];
#pragma unroll
                            for (int x = 0; x < 4; x++) {
                                lx[x] = LU[(size_t)(up.lbeg + r + x * SL) * T + t];
                                tx[x] = P.rel[up.roff + r + x * SL];
                            }
#pragma unroll
                            for (int x = 0; x < 4; x++)
                                if (r + x * SL < lcnt) apply(tx[x], lx[x]);
                        }
                    } else {
                        for (int r = s + LR * SL; r < lcnt; r += 2 * SL) {
                            const bool h2 = r + SL < lcnt;
                            const R l = LU[(size_t)(up.lbeg + r) * T + t];
                            const int tr = P.rel[up.roff + r];
                            const R l2 = h2 ? LU[(size_t)(up.lbeg + r + SL) * T + t] : (R)0;
                            const int tr2 = h2 ? P.rel[up.roff + r + SL] : 0;
                            apply(tr, l);
                            if (h2) apply(tr2, l2);
                        }
                    }
                    wave_sync();
                }
            }
            ub += gcnt;
        }
        wave_sync();
        // a pivot that is not finite, not above 1e-300, or tiny against its column of A
        // (1e-14 of the largest magnitude in FP64, 1e-7 in FP32) fails the instance
        constexpr R kRelPivot = sizeof(R) == 8 ? (R)1e-14 : (R)1e-7;
        const R d = xw[dr * T + t];
        if (s == 0 && valid && !(fabs((double)d) > 1e-300 && isfinite((double)d) && fabs(d) >= kRelPivot * cmx[t]))
            s_piv[t] = 1;
        const R rd = (R)1 / d;          // one reciprocal per pivot, not a division per row
        for (int e = dr + 1 + s; e < cnt; e += SL) xw[e * T + t] = xw[e * T + t] * rd;
        wave_sync();
        if (two) {
            // the pair's second column receives the update of the first (its last source)
            const R m = xw1[dr * T + t];
            for (int e = dr + 1 + s; e < cnt; e += SL) xw1[e * T + t] = fma(-m, xw[e * T + t], xw1[e * T + t]);
            wave_sync();
            if (s == 0) ysl1[t] = fma(-xw[(dr + 1) * T + t], ysl[t], ysl1[t]);
            const R d1 = xw1[(dr + 1) * T + t];
            if (s == 0 && valid &&
                !(fabs((double)d1) > 1e-300 && isfinite((double)d1) && fabs(d1) >= kRelPivot * cmx1[t]))
                s_piv[t] = 1;
            const R rd1 = (R)1 / d1;
            for (int e = dr + 2 + s; e < cnt; e += SL) xw1[e * T + t] = xw1[e * T + t] * rd1;
            wave_sync();
        }
        wait_loads_returned();
        for (int e = s; e < cnt; e += SL) {
            LU[(size_t)(cs + e) * T + t] = xw[e * T + t];
            if (two) LU[(size_t)(cs + cnt + e) * T + t] = xw1[e * T + t];
        }
        if (s == 0) {
            Yv[j * T + t] = ysl[t];
            if (two) Yv[(j + 1) * T + t] = ysl1[t];
        }
        wave_sync();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __hip_atomic_store(&done[j], (unsigned char)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (two) __hip_atomic_store(&done[j + 1], (unsigned char)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (pd.lrank >= 0) __hip_atomic_store(&ldone[pd.lrank], (unsigned char)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        note_progress(s_prog, wave, nprog);
    }
}

// ---- backward substitution and, with upd_v, the voltage update of active instances
// (Sec. 4.3.3, in the same dataflow style); the factors are in LU, y in Yv.
// WIDE: the per-phase kernel prefetches each row's next entry chunk (indices, then U
// values) ahead of its wait; the fused kernel is at its register limit.
template <typename R, int T, int NW, bool WIDE>
__device__ __forceinline__ void bs_phase(TileCtx<R> &cx, const bool upd_v)
{
    constexpr int SL = 64 / T;
    const KArgs &a = cx.a;
    const DevPlan &P = a.p;
    const int tid = cx.tid, wave = cx.wave, lane = cx.lane, t = cx.t, s = cx.s;
    (void)tid;
    const int N = P.N;
    R *const LU = cx.LU;
    R *const Yv = cx.Yv;
    double *const Vm = cx.Vm, *const Va = cx.Va;
    unsigned char *const done = cx.done;
    int *const err = cx.err, *const s_prog = cx.s_prog;
    const int *const s_active = cx.s_active, *const s_reset = cx.s_reset;
    int &nprog = cx.nprog;
    R *const zlds = cx.zlds;
    const int zb = cx.zb;
    (void)err; (void)N;
    const BsPanel *bsd = P.bs_desc + (size_t)a.sched * P.n_panels;
    auto bs_chunk = [&](int c) -> int {
        const int qq = wave + NW * (8 * c + (lane >> 3));
        return reinterpret_cast<const int *>(bsd)[(size_t)qq * 8 + (lane & 7)];   // padded table
    };
    int bch0 = bs_chunk(0), bch1 = bs_chunk(1);
    // FP32-LU: the first entry chunk of the wavefront's next row is loaded while the
    // current row runs, so a row starts with its poll (measured 1-3% faster; in the FP64
    // kernels the extra registers cost more than the round trip saved)
    constexpr bool kBsAhead = sizeof(R) == 4 && !WIDE;
    int nc_all = 0, npq_all = 0;
    if constexpr (kBsAhead) {
        const int q0f = __builtin_amdgcn_readlane(bch0, 4);
        nc_all = P.bs_col[q0f + s];       // padded tables
        npq_all = P.bs_pos[q0f + s];
    }
    wait_loads_returned();
    for (int q = wave, qi = 0; q < P.n_panels; q += NW, qi++) {
        const int kq = qi & 7;
        BsPanel pd;
        {
            int *w = reinterpret_cast<int *>(&pd);
#pragma unroll
            for (int f = 0; f < 8; f++) w[f] = __builtin_amdgcn_readlane(bch0, kq * 8 + f);
        }
        int c0_all = 0, pq0_all = 0;
        if constexpr (kBsAhead) {
            c0_all = nc_all;
            pq0_all = npq_all;
            const int q0n = kq < 7 ? __builtin_amdgcn_readlane(bch0, (kq + 1) * 8 + 4)
                                   : __builtin_amdgcn_readlane(bch1, 4);
            nc_all = P.bs_col[q0n + s];
            npq_all = P.bs_pos[q0n + s];
        }
        if (kq == 7) {
            bch0 = bch1;
            bch1 = bs_chunk((qi >> 3) + 2);
        }
        const int j = pd.j2 & ((1 << 30) - 1);
        const bool two = (pd.j2 >> 30) & 1;
        const int cs = pd.cs, dr = pd.dr, cs1 = pd.cs1;
        const int pu = pd.pu;
        const int bus = pu >> 1;
        // operands that no other row changes, loaded before the wait so that their
        // latency overlaps it: right-hand sides, diagonal (and for a pair the coupling
        // U(j, j+1)), and the voltages to update
        const R y0 = Yv[j * T + t];
        const R d0 = LU[(size_t)(cs + dr) * T + t];
        const R y1 = two ? Yv[(j + 1) * T + t] : (R)0;
        const R d1 = two ? LU[(size_t)(cs1 + dr + 1) * T + t] : (R)1;
        const R u01 = two ? LU[(size_t)(cs1 + dr) * T + t] : (R)0;
        const double vm_old = Vm[bus * T + t], va_old = Va[bus * T + t];
        R acc0 = 0, acc1 = 0;
        const int q0 = pd.q0, q1 = pd.q1;
        // SL entries of the row at a time: each lane loads its entry's column and
        // position, the wavefront waits until all those rows are published, then the
        // operands are loaded.  The FP64 kernels keep the plain loop below: the same
        // body written once as a lambda for both branches compiles, in FP64, to a
        // measurably slower register allocation (7% on the 1350-bus workload).
        if constexpr (kBsAhead) {
            auto chunk = [&](int qb, int c_all, int pq_all) {
                const int q = qb + s;
                const bool in = q < q1;
                const int c = in ? c_all : -1;
                const int pq = in ? pq_all : 1;
                unsigned spins = 0;
                int seen = -1;
                for (;;) {
                    const bool ok = c < 0 || __hip_atomic_load(&done[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (__all(ok) || wait_tick<NW>(spins, seen, s_prog, err)) break;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const R z = Yv[(in ? c : j) * T + t];
                const R l1 = LU[(size_t)pq * T + t];
                const R l0 = LU[(size_t)(pq - 1) * T + t];
                if (in) {
                    if (two) {
                        acc1 = fma(l1, z, acc1);
                        acc0 = fma(l0, z, acc0);
                    } else {
                        acc0 = fma(l1, z, acc0);
                    }
                }
            };
            if (q0 < q1) chunk(q0, c0_all, pq0_all);
            for (int qb = q0 + SL; qb < q1; qb += SL) chunk(qb, P.bs_col[qb + s], P.bs_pos[qb + s]);
        } else if constexpr (WIDE) {
            // U values and column indices do not depend on other rows: the indices of the
            // next two chunks and the U values of the next are in flight while the current
            // chunk waits for its rows (padded tables; positions clamped to 1); z of the
            // positions held in LDS is read from there
            int ca = P.bs_col[q0 + s], pa = max(P.bs_pos[q0 + s], 1);
            R ua1 = LU[(size_t)pa * T + t], ua0 = LU[(size_t)(pa - 1) * T + t];
            int cb = P.bs_col[q0 + SL + s], pb = P.bs_pos[q0 + SL + s];
            for (int qb = q0; qb < q1; qb += SL) {
                const bool in = qb + s < q1;
                const int c = in ? ca : -1;
                const R l1 = ua1, l0 = ua0;
                ca = cb;
                pa = max(pb, 1);
                ua1 = LU[(size_t)pa * T + t];
                ua0 = LU[(size_t)(pa - 1) * T + t];
                cb = P.bs_col[qb + 2 * SL + s];
                pb = P.bs_pos[qb + 2 * SL + s];
                unsigned spins = 0;
                int seen = -1;
                for (;;) {
                    const bool ok = c < 0 || __hip_atomic_load(&done[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (__all(ok) || wait_tick<NW>(spins, seen, s_prog, err)) break;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const int cz = in ? c : j;
                const R z = cz >= zb ? zlds[(cz - zb) * T + t] : Yv[cz * T + t];
                if (in) {
                    if (two) {
                        acc1 = fma(l1, z, acc1);
                        acc0 = fma(l0, z, acc0);
                    } else {
                        acc0 = fma(l1, z, acc0);
                    }
                }
            }
        } else {
            for (int qb = q0; qb < q1; qb += SL) {
                const int q = qb + s;
                const bool in = q < q1;
                const int c_all = P.bs_col[q], pq_all = P.bs_pos[q];   // padded tables
                const int c = in ? c_all : -1;
                const int pq = in ? pq_all : 1;
                unsigned spins = 0;
                int seen = -1;
                for (;;) {
                    const bool ok = c < 0 || __hip_atomic_load(&done[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (__all(ok) || wait_tick<NW>(spins, seen, s_prog, err)) break;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const R z = Yv[(in ? c : j) * T + t];
                const R l1 = LU[(size_t)pq * T + t];
                const R l0 = LU[(size_t)(pq - 1) * T + t];
                if (in) {
                    if (two) {
                        acc1 = fma(l1, z, acc1);
                        acc0 = fma(l0, z, acc0);
                    } else {
                        acc0 = fma(l1, z, acc0);
                    }
                }
            }
        }
#pragma unroll
        for (int off = T; off < 64; off <<= 1) {
            acc0 += __shfl_xor(acc0, off);
            acc1 += __shfl_xor(acc1, off);
        }
        wait_loads_returned();
        if constexpr (WIDE) {
            R z0 = 0, zl = 0;
            if (s == 0) {
                if (two) {
                    zl = (y1 - acc1) / d1;
                    acc0 = fma(u01, zl, acc0);
                }
                z0 = (y0 - acc0) / d0;
                if (j >= zb) zlds[(j - zb) * T + t] = z0;
                if (two && j + 1 >= zb) zlds[(j + 1 - zb) * T + t] = zl;
            }
            // a row held in LDS is read only from there, so it publishes before its global
            // stores; the others publish after them (a pair straddling zb counts as the
            // latter: its first row is read from global memory)
            const bool lds_only = j >= zb;
            auto store_z = [&]() {
                if (s == 0) {
                    if (two) Yv[(j + 1) * T + t] = zl;
                    Yv[j * T + t] = z0;
                    if (upd_v && s_active[t] && !s_reset[t]) {
                        if (two) {
                            Va[bus * T + t] = va_old - (double)z0;
                            Vm[bus * T + t] = vm_old - (double)zl;
                        } else if (pu & 1) {
                            Vm[bus * T + t] = vm_old - (double)z0;
                        } else {
                            Va[bus * T + t] = va_old - (double)z0;
                        }
                    }
                }
            };
            if (!lds_only) store_z();
            wave_sync();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __hip_atomic_store(&done[j], (unsigned char)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (two) __hip_atomic_store(&done[j + 1], (unsigned char)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (lds_only) store_z();
        } else {
            if (s == 0) {
                R zl = 0;
                if (two) {
                    zl = (y1 - acc1) / d1;
                    Yv[(j + 1) * T + t] = zl;
                    acc0 = fma(u01, zl, acc0);
                }
                const R z0 = (y0 - acc0) / d0;
                Yv[j * T + t] = z0;
                if (upd_v && s_active[t] && !s_reset[t]) {
                    if (two) {
                        Va[bus * T + t] = va_old - (double)z0;
                        Vm[bus * T + t] = vm_old - (double)zl;
                    } else if (pu & 1) {
                        Vm[bus * T + t] = vm_old - (double)z0;
                    } else {
                        Va[bus * T + t] = va_old - (double)z0;
                    }
                }
            }
            wave_sync();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __hip_atomic_store(&done[j], (unsigned char)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (two) __hip_atomic_store(&done[j + 1], (unsigned char)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        note_progress(s_prog, wave, nprog);
    }
}

// One bus's row of I = Y V (Eq. 1) for instance lane t: ir + j ii = sum_k Y_ik V_k in entry
// order, the diagonal entry's admittance and index, and, with build, the off-diagonal
// Jacobian entries of the bus's equations written into the LU array (Sec. 3.1.2): with
// w = V_i conj(Y_ik V_k), dS_i/dangle_k = -j w and dS_i/d|V_k| = w / |V_k|.  The row goes in
// groups of G entries whose operands are all loaded before any of the group's stores (a
// store could alias a later load, so entry by entry the loads would wait for them); the
// fused kernel, at its register limit, takes G = 1.
template <typename R, int T, int G>
__device__ __forceinline__ void bus_row(const DevPlan &P, const double2 *yrow, const double2 *Vc, const double *Vm,
                                        R *LU, int i, int t, double2 vv, bool build, double &ir, double &ii,
                                        double2 &ydg, int &qdg)
{
    ir = 0.0;
    ii = 0.0;
    ydg = make_double2(0.0, 0.0);
    qdg = -1;
    const int q1 = P.yrp[i + 1];
    for (int qb = P.yrp[i]; qb < q1; qb += G) {
        int kx[G];
        double2 yx[G], vx[G];
        double vmk[G];
        JPos jx[G];
#pragma unroll
        for (int x = 0; x < G; x++) {
            const int q = min(qb + x, q1 - 1);
            kx[x] = P.yci[q];
            yx[x] = yrow[q];
            if (build) jx[x] = P.jpos[q];
        }
#pragma unroll
        for (int x = 0; x < G; x++) {
            vx[x] = Vc[kx[x] * T + t];
            if (build) vmk[x] = Vm[kx[x] * T + t];
        }
#pragma unroll
        for (int x = 0; x < G; x++) {
            if (qb + x >= q1) break;
            const int k = kx[x];
            const double2 y = yx[x], v = vx[x];
            const double cr = y.x * v.x - y.y * v.y, ci = y.x * v.y + y.y * v.x;     // Y_ik V_k
            ir += cr;
            ii += ci;
            if (k == i) {
                ydg = y;
                qdg = qb + x;
            } else if (build) {
                const JPos jp = jx[x];
                const double inv = 1.0 / vmk[x];
                const double wr = vv.x * cr + vv.y * ci, wi = vv.y * cr - vv.x * ci;
                if (jp.pt >= 0) LU[(size_t)jp.pt * T + t] = (R)wi;
                if (jp.pv >= 0) LU[(size_t)jp.pv * T + t] = (R)(wr * inv);
                if (jp.qt >= 0) LU[(size_t)jp.qt * T + t] = (R)(-wr);
                if (jp.qv >= 0) LU[(size_t)jp.qv * T + t] = (R)(wi * inv);
            }
        }
    }
}

// The whole Newton loop of one tile (T instances) by one workgroup.  Called by the
// one-tile-per-workgroup kernel and by the persistent multi-pattern queue kernel.  With
// RESUME the tile's slots hold instances a.inst[slot] of a reordered batch, which continue
// from their parked state (see split_park_kernel).  With PAIR (a warm-started batch) the
// first a.pair_slots slots hold two per instance, a.inst[slot / 2]: the even slot continues
// the attempt from the given start, the odd slot runs the restart from the fallback point
// at the same time instead of after it; an attempt that would restart stops there, the odd
// slot stops once the even one has ended otherwise, and the slot that the one-lane rule
// would have ended in writes the results (iterations: the updates of both attempts).  The
// slots after those hold one instance each, a.inst[pair_slots / 2 + slot - pair_slots].
constexpr int kStRestart = 100;     // internal: an attempt handed over to its restart

template <typename R, int T, int NW, bool RESUME = false, bool PAIR = false>
__device__ __forceinline__ void nr_tile_body(const KArgs &a, const int tile)
{
    constexpr int SL = 64 / T;          // sub-lanes per instance inside a wavefront
    constexpr int NT = NW * 64;
    constexpr int SLOTS = NT / T;       // bus slots per workgroup
    constexpr int A_ROWS = 2;            // panel rows per lane whose loads are issued together

    extern __shared__ char smem_raw[];
    __shared__ double s_red[NW][T];
    __shared__ int s_bad[NW][T];
    __shared__ int s_active[T], s_status[T], s_iters[T], s_piv[T];
    __shared__ int s_retry[T], s_reset[T], s_nupd[T], s_base[T];
    __shared__ double s_prevf[T];
    __shared__ double s_normf[T];
    __shared__ int s_any, s_err;
    __shared__ int s_prog[NW];          // publications made by each wavefront (progress bound)

    const DevPlan &P = a.p;
    const int tid = threadIdx.x;
    // wavefront index as a scalar: every plan lookup keyed by it becomes a scalar load and
    // every loop over panels a scalar loop
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int t = lane % T;
    const int s = lane / T;
    const int slot = tid / T;
    const int b = tile * T + t;
    const bool valid = b < a.batch;
    const bool paired = PAIR && b < a.pair_slots;
    const int rank = paired ? b >> 1 : PAIR ? (a.pair_slots >> 1) + b - a.pair_slots : b;
    const int bi = RESUME ? (valid ? a.inst[rank] : 0) : b;       // the slot's instance
    const bool flat_lane = paired && (t & 1);   // the flat-start attempt of a paired instance
    const int n = P.n;
    const int N = P.N;

    char *base = a.ws + (size_t)tile * a.tile_bytes;
    R *LU = reinterpret_cast<R *>(base);
    R *Yv = reinterpret_cast<R *>(base + a.off_y);
    double *vec = reinterpret_cast<double *>(base + a.off_vec);
    const size_t nT = (size_t)n * T;
    double *Vm = vec, *Va = vec + nT, *Ps = vec + 2 * nT, *Qs = vec + 3 * nT;
    double2 *Vc = reinterpret_cast<double2 *>(vec + 4 * nT);     // V = |V| e^{j angle}

    // LDS: per wavefront a short working-column pair (slot_rows rows each), the long panels'
    // ring (n_long * 2 * max_col rows), per wavefront two right-hand-side slots and two
    // column maxima, then one publication byte per column and one per long panel
    R *const short_base = reinterpret_cast<R *>(smem_raw);
    R *const long_base = short_base + (size_t)NW * 2 * P.slot_rows * T;
    R *ysl = long_base + (size_t)a.n_long * 2 * P.max_col * T + (size_t)wave * 2 * T;
    R *ysl1 = ysl + T;
    // per wavefront the largest magnitudes of its current panel's columns of A (relative
    // pivot test)
    R *cmx = long_base + (size_t)a.n_long * 2 * P.max_col * T + (size_t)NW * 2 * T + (size_t)wave * 2 * T;
    R *cmx1 = cmx + T;
    unsigned char *done = reinterpret_cast<unsigned char *>(
        long_base + (size_t)a.n_long * 2 * P.max_col * T + (size_t)NW * 4 * T);
    unsigned char *ldone = done + N;
    int *err = &s_err;
    int nprog = 0;                      // this wavefront's publications so far
    TileCtx<R> cx{a, tid, wave, lane, t, s, valid, LU, Yv, Vm, Va, short_base, long_base, ysl, ysl1, cmx, cmx1,
                  done, ldone, err, s_prog, s_piv, s_active, s_reset, nprog, nullptr, N};

    // ---- boundary layout [B][n][2] -> tile layout [n][T]
    const double *vsrc = flat_lane ? a.v_fb : RESUME ? a.vpark : a.v0;
    for (int i = slot; i < n; i += SLOTS) {
        double vm = 1.0, va = 0.0, ps = 0.0, qs = 0.0;
        if (valid) {
            const size_t o = ((size_t)bi * n + i) * 2;
            vm = vsrc[o]; va = vsrc[o + 1];
            ps = a.sbus[o]; qs = a.sbus[o + 1];
        }
        Vm[i * T + t] = vm; Va[i * T + t] = va;
        Ps[i * T + t] = ps; Qs[i * T + t] = qs;
    }
    if (tid < T) {
        s_active[t] = valid ? 1 : 0;
        s_status[t] = PF_ST_MAXITER;
        s_iters[t] = 0;
        s_retry[t] = 0; s_reset[t] = 0; s_nupd[t] = 0; s_base[t] = 0;
        s_prevf[t] = INFINITY;
        if (RESUME && valid) {
            // {status, iterations, updates, active}, {retried, restart pending, updates when
            // the attempt began}, {last max |F| (two words), tile error}
            const int4 c = a.cpark[(size_t)bi * 3], w = a.cpark[(size_t)bi * 3 + 1], x = a.cpark[(size_t)bi * 3 + 2];
            if (!flat_lane) {
                s_status[t] = c.x; s_iters[t] = c.y; s_nupd[t] = c.z; s_active[t] = c.w;
                s_retry[t] = w.x; s_reset[t] = w.y; s_base[t] = w.z;
                s_prevf[t] = __hiloint2double(x.y, x.x);
            } else {
                // a plain solve from the fallback point (no restart of its own); needless
                // when the instance has already stopped or already restarted
                s_retry[t] = 1;
                s_active[t] = c.w && !w.x;
            }
        }
    }
    if (tid == 0) {
        int e0 = 0;
        if (RESUME)
            for (int q = 0; q < T; q++)
                if (tile * T + q < a.batch) {
                    const int bq = tile * T + q;
                    const int rq = !PAIR ? bq : bq < a.pair_slots ? bq >> 1 : (a.pair_slots >> 1) + bq - a.pair_slots;
                    e0 |= a.cpark[(size_t)a.inst[rq] * 3 + 2].z;
                }
        s_err = e0;
    }
    if (tid < NW) s_prog[tid] = 0;
    __syncthreads();

    for (int it = 0;; ++it) {
        // an instance whose first attempt failed restarts from the fallback point
        if (a.v_fb) {
            if (s_reset[t] && valid)
                for (int i = slot; i < n; i += SLOTS) {
                    const size_t o = ((size_t)bi * n + i) * 2;
                    Vm[i * T + t] = a.v_fb[o];
                    Va[i * T + t] = a.v_fb[o + 1];
                }
            __syncthreads();
            if (tid < T) s_reset[t] = 0;
        }
        // ============================ M: mismatch and convergence test
        for (int i = slot; i < n; i += SLOTS) {
            double sn, cs;
            const double vm = Vm[i * T + t];
            sincos_angle(Va[i * T + t], &sn, &cs);
            Vc[i * T + t] = make_double2(vm * cs, vm * sn);
        }
        __syncthreads();
        // I = Y V, S = V conj(I) and F per bus; the same pass over the Ybus row writes the
        // Jacobian entries of the row's equations into the LU array (Sec. 3.1.2): with
        // w = V_i conj(Y_ik V_k), off-diagonal dS_i/dangle_k = -j w, dS_i/d|V_k| = w / |V_k|;
        // diagonal dS_i/dangle_i = j (S_i - |V_i|^2 conj Y_ii), dS_i/d|V_i| = S_i / |V_i| +
        // |V_i| conj Y_ii.  P rows take the real part, Q rows the imaginary part.
        const bool build = a.mode != MODE_MISMATCH;
        // this instance's Ybus values (padding lanes of the last tile read instance 0's)
        const double2 *yrow = reinterpret_cast<const double2 *>(a.ybus + (valid ? (size_t)bi * a.ybus_stride : 0));
        double mx = 0.0;
        int bad = 0;
        for (int i = slot; i < n; i += SLOTS) {
            const double2 vv = Vc[i * T + t];
            double ir, ii;
            double2 ydg;
            int qdg;
            bus_row<R, T, 1>(P, yrow, Vc, Vm, LU, i, t, vv, build, ir, ii, ydg, qdg);
            const double sr = vv.x * ir + vv.y * ii, si = vv.y * ir - vv.x * ii;       // S_i
            if (build && qdg >= 0) {
                const JPos jp = P.jpos[qdg];
                const double vmi = Vm[i * T + t];
                const double m2 = vmi * vmi;
                if (jp.pt >= 0) LU[(size_t)jp.pt * T + t] = (R)(-si - m2 * ydg.y);
                if (jp.pv >= 0) LU[(size_t)jp.pv * T + t] = (R)(sr / vmi + vmi * ydg.x);
                if (jp.qt >= 0) LU[(size_t)jp.qt * T + t] = (R)(sr - m2 * ydg.x);
                if (jp.qv >= 0) LU[(size_t)jp.qv * T + t] = (R)(si / vmi - vmi * ydg.y);
            }
            const int pe = P.bus_peq[i], qe = P.bus_qeq[i];
            if (pe >= 0) {
                const double f = sr - Ps[i * T + t];
                Yv[pe * T + t] = (R)f;
                if (!isfinite(f)) bad = 1; else mx = fmax(mx, fabs(f));
                if (a.mode == MODE_MISMATCH && valid) a.aux_out[(size_t)b * N + a.perm[pe]] = f;
            }
            if (qe >= 0) {
                const double f = si - Qs[i * T + t];
                Yv[qe * T + t] = (R)f;
                if (!isfinite(f)) bad = 1; else mx = fmax(mx, fabs(f));
                if (a.mode == MODE_MISMATCH && valid) a.aux_out[(size_t)b * N + a.perm[qe]] = f;
            }
        }
#pragma unroll
        for (int off = T; off < 64; off <<= 1) {
            mx = fmax(mx, __shfl_xor(mx, off));
            bad |= __shfl_xor(bad, off);
        }
        if (s == 0) { s_red[wave][t] = mx; s_bad[wave][t] = bad; }
        __syncthreads();
        if (tid < T) {
            double nf = 0.0;
            int nb = 0;
#pragma unroll
            for (int w = 0; w < NW; w++) { nf = fmax(nf, s_red[w][t]); nb |= s_bad[w][t]; }
            s_normf[t] = nb ? NAN : nf;
            s_piv[t] = 0;
            if (s_active[t] && a.mode == MODE_SOLVE) {
                // iters counts voltage updates over both attempts; max_iter bounds the
                // updates of each attempt (s_base: the count when the current one began), so
                // a restart from the fallback point runs exactly as a plain solve from there
                int fail = 0;
                if (nb) fail = PF_ST_NONFINITE;
                else if (nf < a.tol) { s_status[t] = PF_ST_CONVERGED; s_active[t] = 0; s_iters[t] = s_nupd[t]; }
                else if (s_nupd[t] - s_base[t] >= a.max_iter) fail = PF_ST_MAXITER;
                // an attempt that has a fallback gives up as soon as an update fails to
                // reduce the mismatch (Newton from a good start contracts every step)
                else if (a.v_fb && !s_retry[t] && !(nf < s_prevf[t])) fail = PF_ST_MAXITER;
                s_prevf[t] = nf;
                if (fail) {
                    if (a.v_fb && !s_retry[t]) {
                        if (paired) { s_status[t] = kStRestart; s_active[t] = 0; s_iters[t] = s_nupd[t]; }
                        else { s_retry[t] = 1; s_reset[t] = 1; s_base[t] = s_nupd[t]; }
                    } else { s_status[t] = fail; s_active[t] = 0; s_iters[t] = s_nupd[t]; }
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            int any = 0;
            for (int q = 0; q < T; q++) {
                // a flat-start attempt is needless once its warm attempt has ended otherwise
                if (PAIR && (q & 1) && tile * T + q < a.pair_slots && !s_active[q - 1] && s_status[q - 1] != kStRestart)
                    s_active[q] = 0;
                any |= s_active[q];
            }
            s_any = any;
        }
        __syncthreads();
        if (a.mode == MODE_MISMATCH) {
            if (tid < T && valid) a.aux2_out[b] = s_normf[t];
            return;
        }
        if (!s_any) {
            if (a.mode != MODE_SOLVE) return;
            break;
        }
        // every instance ends within 2 max_iter + 3 passes (the updates of both attempts,
        // the restart pass and the final tests); a tile still running well past that has
        // lost its state and reports an internal error instead of looping on
        if (it > 2 * a.max_iter + 4) {
            if (tid == 0) s_err = 1;
            __syncthreads();
            break;
        }

        // ============================ LU: Jacobian -> refactorization -> forward substitution
        lu_phase<R, T, NW, false>(cx);
        __syncthreads();
        if (tid < T && s_piv[t] && s_active[t] && !s_reset[t] && a.mode == MODE_SOLVE) {
            if (a.v_fb && !s_retry[t]) {
                if (paired) { s_status[t] = kStRestart; s_active[t] = 0; s_iters[t] = s_nupd[t]; }
                else { s_retry[t] = 1; s_reset[t] = 1; s_base[t] = s_nupd[t]; }
            } else { s_status[t] = PF_ST_PIVOT; s_active[t] = 0; s_iters[t] = s_nupd[t]; }
        }
        if (a.mode == MODE_FACTOR) {
            const size_t nnz = (size_t)P.nnzlu;
            if (valid)
                for (size_t e = slot; e < nnz; e += SLOTS) a.aux_out[(size_t)b * nnz + e] = (double)LU[e * T + t];
            return;
        }
        for (int w = tid; w < N; w += NT)
            __hip_atomic_store(&done[w], (unsigned char)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();

        // ============================ BS: backward substitution and voltage update
        // Panels in back-substitution level order.  For a pair (j, j+1) the rows share their
        // column set i > j+1, and U(j, i), U(j+1, i) sit next to each other in column i.
        const bool upd_v = (a.mode == MODE_SOLVE);
        bs_phase<R, T, NW, false>(cx, upd_v);
        __syncthreads();
        if (a.mode == MODE_STEP) {
            if (valid)
                for (int j = slot; j < N; j += SLOTS) a.aux_out[(size_t)b * N + a.perm[j]] = (double)Yv[j * T + t];
            return;
        }
        if (tid < T && s_active[t] && !s_reset[t]) s_nupd[t]++;
    }

    // ---- tile layout -> boundary layout (of a pair, the slot whose attempt ended the solve)
    const bool chosen = !paired || (flat_lane ? s_status[t ^ 1] == kStRestart : s_status[t] != kStRestart);
    if (valid && chosen) {
        for (int i = slot; i < n; i += SLOTS) {
            const size_t o = ((size_t)bi * n + i) * 2;
            a.v_out[o] = Vm[i * T + t];
            a.v_out[o + 1] = Va[i * T + t];
        }
        if (s == 0 && wave == 0) {
            if (a.done_ticks) a.done_ticks[bi] = wall_clock64() - *a.t0;
            const int st = s_err ? PF_ST_INTERNAL : s_status[t];
            a.iters_out[bi] = s_iters[t] + (flat_lane ? s_iters[t ^ 1] : 0);
            a.conv_out[bi] = st == PF_ST_CONVERGED ? 1 : 0;
            if (a.status_out) a.status_out[bi] = (int8_t)st;
        }
    }
}

// Four waves per SIMD: the refactorization is bound by dependent memory round trips, so
// resident wavefronts matter more than the few registers spilled at this bound.
template <typename R, int T, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void nr_tile_kernel(KArgs a)
{
    nr_tile_body<R, T, NW>(a, blockIdx.x);
}

// The head of a reordered batch: its hardest instances finish their Newton iterations in one
// launch whose workgroups keep their CUs until done, at one tile's latency per iteration.
template <typename R, int T, int NW, bool PAIR>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void nr_head_kernel(KArgs a)
{
    nr_tile_body<R, T, NW, true, PAIR>(a, blockIdx.x);
}

// Persistent launch over a queue of work items (one per pattern / batch): workgroups pop
// tiles from a global counter until every item's tiles are done.  prefix[i] is the first
// tile of item i (prefix[nitems] = total); items are ordered by the caller.
// Persistent launch over a queue of work items (one per pattern / batch) that share one
// precision, tile size and workgroup size: workgroups pop tiles from a global counter until
// every item's tiles are done.  prefix[i] is the first tile of item i (prefix[nitems] =
// total).  Every wave leaves the loop once the counter has passed the last tile, so the
// grid always drains.
template <typename R, int T, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void nr_queue_kernel(
    const KArgs *__restrict__ items, const int *__restrict__ prefix, int nitems, int *counter)
{
    __shared__ int s_tile;
    const int total = prefix[nitems];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
        __syncthreads();
        const int tg = __builtin_amdgcn_readfirstlane(s_tile);
        if (tg >= total) break;
        int it = 0;
        while (it + 1 < nitems && prefix[it + 1] <= tg) it++;
        nr_tile_body<R, T, NW>(items[it], tg - prefix[it]);
    }
}

// Resets the queue's tile counters and records the launch's start tick; a kernel rather than
// a memset so that it can sit inside a graph.
__global__ void queue_reset_kernel(int *counters, int n, unsigned long long *t0)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0;
    if (threadIdx.x == 0) *t0 = wall_clock64();
}

// ------------------------------------------------------------------ per-phase launches
// The same Newton iterations as nr_tile_body, one launch per phase and iteration, so that
// each phase runs with its own register budget and launch shape: the mismatch and Jacobian
// (a3, a4) over every (bus, instance) of the batch at full occupancy, the refactorization
// (a5, a6 forward) and the back substitution with the voltage update (a6, a7) per tile.
// The loop stays on the host as a fixed sequence of launches; an instance's state
// (status, iterations, updates, active) and its tile's flags live in the tile's block of
// the workspace, and a tile whose instances have all stopped returns at once.

// The per-phase kernels use the refactorization's wider load batches (measured on 2,000
// scenarios of the 9000-bus grid: FP64 64.7 -> 61.0 ms, FP32-LU 44.1 -> 44.2 ms); the back
// substitution's prefetch and LDS copy of z are slower there (66.6 / 47.7 ms with them)
// and stay off.
template <typename R> constexpr bool kWideLu = true;
template <typename R> constexpr bool kWideBs = false;

// A tile's control block: per instance {status, iterations, updates, active}, the tile's
// flags {any active, internal error}, per instance the fallback start's state {retried,
// restart pending, updates when the current attempt began}, and the last max |F|.
template <int T>
__device__ __forceinline__ int4 *tile_ctl(const KArgs &a, int tile)
{
    return reinterpret_cast<int4 *>(a.ws + (size_t)tile * a.tile_bytes + a.off_ctl);
}
template <int T>
__device__ __forceinline__ int4 *tile_warm(const KArgs &a, int tile)
{
    return tile_ctl<T>(a, tile) + T + 1;
}
template <int T>
__device__ __forceinline__ double *tile_prevf(const KArgs &a, int tile)
{
    return reinterpret_cast<double *>(tile_ctl<T>(a, tile) + 2 * T + 1);
}

// Boundary rows [B][n][2] <-> tile layout [n][T], through LDS: each round moves kMBlock / T
// buses of the tile's T instances, reading (or writing) every instance's row segment
// contiguously and the tile layout contiguously.  Slot b's row is its instance's.  The
// grid's y dimension splits a tile's buses into ranges of kStageRounds rounds, one
// workgroup each (one workgroup per tile left most CUs idle and ran its rounds one after
// another: 9000-bus grid, 2,000 instances, 0.53 ms for the layout in).
constexpr int kStageRounds = 8;
template <int T>
struct RowStage {
    static constexpr int CH = kMBlock / T;
    double v[2][2 * CH][T + 1];
};
template <int T>
static int stage_splits(int n)
{
    constexpr int per = kStageRounds * RowStage<T>::CH;
    return (n + per - 1) / per;
}
// the buses [*i_lo, *i_hi) of workgroup blockIdx.y
template <int T>
__device__ __forceinline__ void stage_range(int n, int *i_lo, int *i_hi)
{
    constexpr int per = kStageRounds * RowStage<T>::CH;
    *i_lo = blockIdx.y * per;
    *i_hi = min(n, *i_lo + per);
}

// layout in: |V| and angle from vsrc (the start v0, or the rows parked after the first
// update), the P and Q set points from sbus; instance states either initialised or, with
// csrc, taken from the parked control words (see split_park_kernel)
template <int T>
__global__ __launch_bounds__(kMBlock) void split_in_kernel(KArgs a, const double *vsrc, const int4 *csrc)
{
    constexpr int CH = RowStage<T>::CH;
    __shared__ RowStage<T> st;
    __shared__ int s_row[T];
    const int tile = blockIdx.x, tid = threadIdx.x;
    const int n = a.p.n;
    if (tid < T) {
        const int b = tile * T + tid;
        s_row[tid] = b < a.batch ? inst_of(a, b) : -1;
    }
    __syncthreads();
    double *vec = reinterpret_cast<double *>(a.ws + (size_t)tile * a.tile_bytes + a.off_vec);
    const size_t nT = (size_t)n * T;
    int i_lo, i_hi;
    stage_range<T>(n, &i_lo, &i_hi);
    for (int i0 = i_lo; i0 < i_hi; i0 += CH) {
        const int nb = min(CH, i_hi - i0);
        for (int e = tid; e < T * 2 * CH; e += kMBlock) {
            const int t = e / (2 * CH), w = e - t * (2 * CH);      // w = 2 * bus + (0 |V| or P, 1 angle or Q)
            const int row = s_row[t];
            double v = (w & 1) ? 0.0 : 1.0, sp = 0.0;
            if (row >= 0 && w < 2 * nb) {
                const size_t o = ((size_t)row * n + i0) * 2 + w;
                v = vsrc[o];
                sp = a.sbus[o];
            }
            st.v[0][w][t] = v;
            st.v[1][w][t] = sp;
        }
        __syncthreads();
        for (int e = tid; e < nb * T; e += kMBlock) {
            const int il = e / T, t = e - il * T;
            const size_t o = (size_t)(i0 + il) * T + t;
            vec[o] = st.v[0][2 * il][t];
            vec[nT + o] = st.v[0][2 * il + 1][t];
            vec[2 * nT + o] = st.v[1][2 * il][t];
            vec[3 * nT + o] = st.v[1][2 * il + 1][t];
        }
        __syncthreads();
    }
    if (blockIdx.y != 0) return;
    int4 *ctl = tile_ctl<T>(a, tile);
    __shared__ int s_act[T], s_err[T];
    if (tid < T) {
        const int row = s_row[tid];
        int4 c = make_int4(PF_ST_MAXITER, 0, 0, row >= 0 ? 1 : 0), w = make_int4(0, 0, 0, 0);
        double pfv = INFINITY;
        int er = 0;
        if (csrc && row >= 0) {
            c = csrc[(size_t)row * 3];
            w = csrc[(size_t)row * 3 + 1];
            const int4 x = csrc[(size_t)row * 3 + 2];
            pfv = __hiloint2double(x.y, x.x);
            er = x.z;
        } else if (csrc) {
            c.w = 0;
        }
        ctl[tid] = c;
        tile_warm<T>(a, tile)[tid] = w;
        tile_prevf<T>(a, tile)[tid] = pfv;
        s_act[tid] = c.w;
        s_err[tid] = er;
    }
    __syncthreads();
    if (tid == 0) {
        int any = 0, err = 0;
        for (int q = 0; q < T; q++) { any |= s_act[q]; err |= s_err[q]; }
        int *tf = reinterpret_cast<int *>(ctl + T);
        tf[0] = any;
        tf[1] = err;
    }
}

// After the first update of a batch that is then reordered: every slot's |V| and angle go
// to row inst_of(slot) of park ([B][n][2]) and its control words (state, fallback state,
// last max |F| and the tile's internal-error flag) to ctl_park[3 row ...].
template <int T>
__global__ __launch_bounds__(kMBlock) void split_park_kernel(KArgs a, double *park, int4 *ctl_park)
{
    constexpr int CH = RowStage<T>::CH;
    __shared__ RowStage<T> st;
    __shared__ int s_row[T];
    const int tile = blockIdx.x, tid = threadIdx.x;
    const int n = a.p.n;
    if (tid < T) {
        const int b = tile * T + tid;
        s_row[tid] = b < a.batch ? inst_of(a, b) : -1;
    }
    __syncthreads();
    const double *vec = reinterpret_cast<const double *>(a.ws + (size_t)tile * a.tile_bytes + a.off_vec);
    const size_t nT = (size_t)n * T;
    int i_lo, i_hi;
    stage_range<T>(n, &i_lo, &i_hi);
    for (int i0 = i_lo; i0 < i_hi; i0 += CH) {
        const int nb = min(CH, i_hi - i0);
        for (int e = tid; e < nb * T; e += kMBlock) {
            const int il = e / T, t = e - il * T;
            const size_t o = (size_t)(i0 + il) * T + t;
            st.v[0][2 * il][t] = vec[o];
            st.v[0][2 * il + 1][t] = vec[nT + o];
        }
        __syncthreads();
        for (int e = tid; e < T * 2 * CH; e += kMBlock) {
            const int t = e / (2 * CH), w = e - t * (2 * CH);
            const int row = s_row[t];
            if (row >= 0 && w < 2 * nb) park[((size_t)row * n + i0) * 2 + w] = st.v[0][w][t];
        }
        __syncthreads();
    }
    if (blockIdx.y == 0 && tid < T && s_row[tid] >= 0) {
        const int4 *ctl = tile_ctl<T>(a, tile);
        const size_t r = (size_t)s_row[tid] * 3;
        ctl_park[r] = ctl[tid];
        ctl_park[r + 1] = tile_warm<T>(a, tile)[tid];
        const double pfv = tile_prevf<T>(a, tile)[tid];
        ctl_park[r + 2] = make_int4(__double2loint(pfv), __double2hiint(pfv), reinterpret_cast<const int *>(ctl + T)[1], 0);
    }
}

// rectangular V = |V| e^{j angle} of every bus of the active tiles (one sine/cosine per
// bus, as in nr_tile_body)
template <int T>
__global__ __launch_bounds__(kMBlock) void split_v_kernel(KArgs a, int ntiles)
{
    const int tid = threadIdx.x, t = tid % T;
    const int n = a.p.n, nbb = a.nbb;
    const size_t nT = (size_t)n * T;
    const int nitems = ntiles * nbb;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int tile = item / nbb, blk = item - tile * nbb;
        char *base = a.ws + (size_t)tile * a.tile_bytes;
        const int4 *ctl = reinterpret_cast<const int4 *>(base + a.off_ctl);
        if (!reinterpret_cast<const int *>(ctl + T)[0]) continue;
        const int i = blk * (kMBlock / T) + tid / T;
        if (i >= n) continue;
        double *vec = reinterpret_cast<double *>(base + a.off_vec);
        double2 *Vc = reinterpret_cast<double2 *>(vec + 4 * nT);
        // an instance whose first attempt failed restarts from the fallback point
        const int b = tile * T + t;
        if (a.v_fb && b < a.batch && tile_warm<T>(a, tile)[t].y) {
            const size_t o = ((size_t)inst_of(a, b) * n + i) * 2;
            vec[i * T + t] = a.v_fb[o];
            vec[nT + i * T + t] = a.v_fb[o + 1];
        }
        double sn, cs;
        const double vm = vec[i * T + t];
        sincos_angle(vec[nT + i * T + t], &sn, &cs);
        Vc[i * T + t] = make_double2(vm * cs, vm * sn);
    }
}

// mismatch (Eq. 1) and, with build, the Jacobian written into the LU positions (Sec. 3.1.2)
// for kMBlock / T buses of one tile per work item; each work item leaves the largest |F|
// (and a non-finite flag) of its buses per instance for the convergence decision
template <typename R, int T>
__global__ __launch_bounds__(kMBlock) void split_m_kernel(KArgs a, int ntiles, int build)
{
    constexpr int BUSB = kMBlock / T;
    __shared__ double s_mx[kMBlock];
    __shared__ int s_bd[kMBlock];
    const DevPlan &P = a.p;
    const int tid = threadIdx.x, t = tid % T, ib = tid / T;
    const int n = P.n, nbb = a.nbb;
    const size_t nT = (size_t)n * T;
    const int nitems = ntiles * nbb;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int tile = item / nbb, blk = item - tile * nbb;
        char *base = a.ws + (size_t)tile * a.tile_bytes;
        const int4 *ctl = reinterpret_cast<const int4 *>(base + a.off_ctl);
        if (!reinterpret_cast<const int *>(ctl + T)[0]) continue;      // no instance active
        R *LU = reinterpret_cast<R *>(base);
        R *Yv = reinterpret_cast<R *>(base + a.off_y);
        const double *vec = reinterpret_cast<const double *>(base + a.off_vec);
        const double *Vm = vec, *Ps = vec + 2 * nT, *Qs = vec + 3 * nT;
        const double2 *Vc = reinterpret_cast<const double2 *>(vec + 4 * nT);
        const int b = tile * T + t;
        const bool valid = b < a.batch;
        const double2 *yrow = reinterpret_cast<const double2 *>(
            a.ybus + (valid && a.ybus_stride ? (size_t)inst_of(a, b) * a.ybus_stride : 0));
        const int i = blk * BUSB + ib;
        double mx = 0.0;
        int bad = 0;
        if (i < n) {
            const double2 vv = Vc[i * T + t];
            double ir, ii;
            double2 ydg;
            int qdg;
            bus_row<R, T, kMRow>(P, yrow, Vc, Vm, LU, i, t, vv, build, ir, ii, ydg, qdg);
            const double sr = vv.x * ir + vv.y * ii, si = vv.y * ir - vv.x * ii;       // S_i
            if (build && qdg >= 0) {
                const JPos jp = P.jpos[qdg];
                const double vmi = Vm[i * T + t];
                const double m2 = vmi * vmi;
                if (jp.pt >= 0) LU[(size_t)jp.pt * T + t] = (R)(-si - m2 * ydg.y);
                if (jp.pv >= 0) LU[(size_t)jp.pv * T + t] = (R)(sr / vmi + vmi * ydg.x);
                if (jp.qt >= 0) LU[(size_t)jp.qt * T + t] = (R)(sr - m2 * ydg.x);
                if (jp.qv >= 0) LU[(size_t)jp.qv * T + t] = (R)(si / vmi - vmi * ydg.y);
            }
            const int pe = P.bus_peq[i], qe = P.bus_qeq[i];
            if (pe >= 0) {
                const double f = sr - Ps[i * T + t];
                Yv[pe * T + t] = (R)f;
                if (!isfinite(f)) bad = 1; else mx = fmax(mx, fabs(f));
            }
            if (qe >= 0) {
                const double f = si - Qs[i * T + t];
                Yv[qe * T + t] = (R)f;
                if (!isfinite(f)) bad = 1; else mx = fmax(mx, fabs(f));
            }
        }
        s_mx[tid] = mx;
        s_bd[tid] = bad;
        __syncthreads();
        if (tid < T) {
            double m = 0.0;
            int bd = 0;
            for (int x = 0; x < BUSB; x++) { m = fmax(m, s_mx[x * T + t]); bd |= s_bd[x * T + t]; }
            double *pm = reinterpret_cast<double *>(base + a.off_part);
            int *pb = reinterpret_cast<int *>(pm + (size_t)nbb * T);
            pm[blk * T + t] = m;
            pb[blk * T + t] = bd;
        }
        __syncthreads();
    }
}

// The convergence decision of instance t of a tile from the mismatch kernel's maxima, the
// rule of nr_tile_body: non-finite, below tol, or max_iter updates done in the current
// attempt; with a fallback start, a first attempt also ends when an update did not reduce
// max |F|, and a failed first attempt restarts from the fallback point (the V kernel of the
// next iteration reloads it) instead of ending.  Called by the tile's first T threads;
// returns whether the instance stays active and in *reset whether it restarts.
template <int T>
__device__ __forceinline__ int split_decide(const KArgs &a, int tile, int t, int *reset)
{
    int4 *ctl = tile_ctl<T>(a, tile);
    int4 c = ctl[t];
    int4 w = tile_warm<T>(a, tile)[t];
    w.y = 0;                                        // a pending restart has been reloaded
    if (c.w) {
        const double *pm = reinterpret_cast<const double *>(a.ws + (size_t)tile * a.tile_bytes + a.off_part);
        const int *pb = reinterpret_cast<const int *>(pm + (size_t)a.nbb * T);
        double nf = 0.0;
        int nb = 0;
        for (int k = 0; k < a.nbb; k++) { nf = fmax(nf, pm[k * T + t]); nb |= pb[k * T + t]; }
        double *pfp = tile_prevf<T>(a, tile) + t;
        int fail = 0;
        if (nb) fail = PF_ST_NONFINITE;
        else if (nf < a.tol) { c.x = PF_ST_CONVERGED; c.w = 0; c.y = c.z; }
        else if (c.z - w.z >= a.max_iter) fail = PF_ST_MAXITER;
        else if (a.v_fb && !w.x && !(nf < *pfp)) fail = PF_ST_MAXITER;
        *pfp = nf;
        if (fail) {
            if (a.v_fb && !w.x) { w.x = 1; w.y = 1; w.z = c.z; }
            else { c.x = fail; c.w = 0; c.y = c.z; }
        }
        ctl[t] = c;
    }
    tile_warm<T>(a, tile)[t] = w;
    *reset = w.y;
    return c.w;
}

// The tile's LDS view of nr_tile_body for the refactorization (same layout)
template <typename R, int T, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void split_lu_kernel(KArgs a)
{
    extern __shared__ char smem_raw[];
    __shared__ int s_active[T], s_piv[T], s_reset[T];
    __shared__ int s_any, s_err;
    __shared__ int s_prog[NW];
    const DevPlan &P = a.p;
    const int tile = blockIdx.x, tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, t = lane % T, s = lane / T;
    const bool valid = tile * T + t < a.batch;
    int4 *ctl = tile_ctl<T>(a, tile);
    int *tf = reinterpret_cast<int *>(ctl + T);
    if (!__builtin_amdgcn_readfirstlane(tf[0])) return;
    if (tid < T) {
        int rs = 0;
        s_active[t] = split_decide<T>(a, tile, t, &rs);
        s_piv[t] = 0;
        s_reset[t] = rs;
    }
    if (tid == 0) s_err = 0;
    if (tid < NW) s_prog[tid] = 0;
    __syncthreads();
    if (tid == 0) {
        int any = 0;
        for (int q = 0; q < T; q++) any |= s_active[q];
        s_any = any;
        tf[0] = any;
    }
    __syncthreads();
    if (!s_any) return;
    char *base = a.ws + (size_t)tile * a.tile_bytes;
    double *vec = reinterpret_cast<double *>(base + a.off_vec);
    const size_t nT = (size_t)P.n * T;
    R *const short_base = reinterpret_cast<R *>(smem_raw);
    R *const long_base = short_base + (size_t)NW * 2 * P.slot_rows * T;
    R *ysl = long_base + (size_t)a.n_long * 2 * P.max_col * T + (size_t)wave * 2 * T;
    R *cmx = long_base + (size_t)a.n_long * 2 * P.max_col * T + (size_t)NW * 2 * T + (size_t)wave * 2 * T;
    unsigned char *done = reinterpret_cast<unsigned char *>(
        long_base + (size_t)a.n_long * 2 * P.max_col * T + (size_t)NW * 4 * T);
    int nprog = 0;
    TileCtx<R> cx{a, tid, wave, lane, t, s, valid, reinterpret_cast<R *>(base), reinterpret_cast<R *>(base + a.off_y),
                  vec, vec + nT, short_base, long_base, ysl, ysl + T, cmx, cmx + T, done, done + P.N, &s_err,
                  s_prog, s_piv, s_active, s_reset, nprog, nullptr, P.N};
    lu_phase<R, T, NW, kWideLu<R>>(cx);
    __syncthreads();
    if (tid < T && s_piv[t] && s_active[t] && !s_reset[t]) {
        int4 c = ctl[t];
        int4 w = tile_warm<T>(a, tile)[t];
        if (a.v_fb && !w.x) {
            w.x = 1; w.y = 1; w.z = c.z;
            tile_warm<T>(a, tile)[t] = w;
        } else {
            c.x = PF_ST_PIVOT; c.w = 0; c.y = c.z;
            ctl[t] = c;
        }
    }
    if (tid == 0 && s_err) tf[1] = 1;
}

// back substitution and voltage update; LDS holds only the row publication bytes
template <typename R, int T, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void split_bs_kernel(KArgs a)
{
    extern __shared__ char smem_raw[];
    __shared__ int s_active[T], s_reset[T];
    __shared__ int s_any, s_err;
    __shared__ int s_prog[NW];
    const DevPlan &P = a.p;
    const int tile = blockIdx.x, tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, t = lane % T, s = lane / T;
    const bool valid = tile * T + t < a.batch;
    int4 *ctl = tile_ctl<T>(a, tile);
    int *tf = reinterpret_cast<int *>(ctl + T);
    if (!__builtin_amdgcn_readfirstlane(tf[0])) return;
    unsigned char *done = reinterpret_cast<unsigned char *>(smem_raw);
    if (tid < T) { s_active[t] = ctl[t].w; s_reset[t] = tile_warm<T>(a, tile)[t].y; }
    if (tid == 0) s_err = 0;
    if (tid < NW) s_prog[tid] = 0;
    for (int w = tid; w < P.N; w += NW * 64)
        __hip_atomic_store(&done[w], (unsigned char)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    if (tid == 0) {
        int any = 0;
        for (int q = 0; q < T; q++) any |= s_active[q];
        s_any = any;
    }
    __syncthreads();
    if (!s_any) return;
    char *base = a.ws + (size_t)tile * a.tile_bytes;
    double *vec = reinterpret_cast<double *>(base + a.off_vec);
    const size_t nT = (size_t)P.n * T;
    int nprog = 0;
    // z of the highest positions (the dense tail, solved first) in LDS after the flags
    R *zlds = reinterpret_cast<R *>(smem_raw + ((P.N + 255) & ~255));
    const int zb = max(0, P.N - (int)((size_t)a.bs_zbytes / (sizeof(R) * T)));
    TileCtx<R> cx{a, tid, wave, lane, t, s, valid, reinterpret_cast<R *>(base), reinterpret_cast<R *>(base + a.off_y),
                  vec, vec + nT, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, done, nullptr, &s_err, s_prog,
                  nullptr, s_active, s_reset, nprog, zlds, zb};
    bs_phase<R, T, NW, kWideBs<R>>(cx, true);
    __syncthreads();
    if (tid < T && s_active[t] && !s_reset[t]) ctl[t].z += 1;
    if (tid == 0 && s_err) tf[1] = 1;
}

// the final convergence decision and the tile layout -> boundary layout
template <int T>
__global__ __launch_bounds__(kMBlock) void split_out_kernel(KArgs a)
{
    const int tile = blockIdx.x, tid = threadIdx.x, t = tid % T;
    const int b = tile * T + t;
    const bool valid = b < a.batch;
    int4 *ctl = tile_ctl<T>(a, tile);
    const int *tf = reinterpret_cast<const int *>(ctl + T);
    const bool first = blockIdx.y == 0;     // the workgroup that decides and writes the states
    if (first && tid < T && tf[0]) {
        int rs = 0;
        if (split_decide<T>(a, tile, t, &rs) && rs) {
            // a restart requested at the last decision has no iteration left
            int4 *c = tile_ctl<T>(a, tile) + t;
            c->x = PF_ST_MAXITER; c->w = 0; c->y = c->z;
        }
    }
    __syncthreads();
    constexpr int CH = RowStage<T>::CH;
    __shared__ RowStage<T> st;
    __shared__ int s_row[T];
    if (tid < T) s_row[tid] = valid ? inst_of(a, b) : -1;
    __syncthreads();
    const int n = a.p.n;
    const double *vec = reinterpret_cast<const double *>(a.ws + (size_t)tile * a.tile_bytes + a.off_vec);
    const size_t nT = (size_t)n * T;
    int i_lo, i_hi;
    stage_range<T>(n, &i_lo, &i_hi);
    for (int i0 = i_lo; i0 < i_hi; i0 += CH) {
        const int nb = min(CH, i_hi - i0);
        for (int e = tid; e < nb * T; e += kMBlock) {
            const int il = e / T, tt = e - il * T;
            const size_t o = (size_t)(i0 + il) * T + tt;
            st.v[0][2 * il][tt] = vec[o];
            st.v[0][2 * il + 1][tt] = vec[nT + o];
        }
        __syncthreads();
        for (int e = tid; e < T * 2 * CH; e += kMBlock) {
            const int tt = e / (2 * CH), w = e - tt * (2 * CH);
            const int row = s_row[tt];
            if (row >= 0 && w < 2 * nb) a.v_out[((size_t)row * n + i0) * 2 + w] = st.v[0][w][tt];
        }
        __syncthreads();
    }
    if (first && tid < T && valid) {
        const int bi = s_row[t];
        const int4 c = ctl[t];
        const int st_ = tf[1] ? PF_ST_INTERNAL : c.x;
        a.iters_out[bi] = c.y;
        a.conv_out[bi] = st_ == PF_ST_CONVERGED ? 1 : 0;
        if (a.status_out) a.status_out[bi] = (int8_t)st_;
    }
}

// ---- hardest-first reordering of a batch after its first update (per-phase launches)
// The instances that need the most Newton iterations are those whose first step was the
// largest.  Placing them in the first tiles gives the later iterations dense tiles (a tile
// runs until its slowest instance stops) and starts their long iteration chains first, so
// those overlap the rest of the batch instead of extending its end.

// Sort key of each slot after the first update: 16 bits of max |dx| (the float's sign,
// exponent and leading mantissa bits, monotone for non-negative values), stored inverted
// so that an ascending sort puts the largest steps first.  A slot whose instance has
// stopped gets the smallest key, one that restarts from its fallback point the largest
// (a fresh solve lies ahead of it).  ids[b] = b.
template <typename R, int T>
__global__ __launch_bounds__(kMBlock) void split_key_kernel(KArgs a, uint32_t *keys, int32_t *ids)
{
    __shared__ float s_mx[kMBlock];
    const int tile = blockIdx.x, tid = threadIdx.x, t = tid % T;
    const int b = tile * T + t;
    const int4 *ctl = tile_ctl<T>(a, tile);
    const R *Yv = reinterpret_cast<const R *>(a.ws + (size_t)tile * a.tile_bytes + a.off_y);
    float mx = 0.f;
    for (int j = tid / T; j < a.p.N; j += kMBlock / T) {
        const float z = fabsf((float)Yv[j * T + t]);
        mx = (z > mx || z != z) ? z : mx;                 // NaN wins
    }
    s_mx[tid] = mx;
    __syncthreads();
    if (tid < T && b < a.batch) {
        float m = 0.f;
        for (int x = 0; x < kMBlock / T; x++) {
            const float z = s_mx[x * T + t];
            m = (z > m || z != z) ? z : m;
        }
        uint32_t bits;
        if (!ctl[t].w) bits = 0;
        else if (tile_warm<T>(a, tile)[t].y || m != m) bits = 0xFFFFu;
        else bits = __float_as_uint(m) >> 16;             // m >= 0: at most 0x7F80 (inf)
        keys[b] = 0xFFFFu - bits;
        ids[b] = b;
    }
}

// One pass of a stable least-significant-digit radix sort over 8 bits of 16-bit keys:
// per block of kSortSeg items a digit histogram, an exclusive scan over (digit, block),
// then a stable scatter.
constexpr int kSortSeg = 1024;

__global__ __launch_bounds__(256) void sort_hist_kernel(const uint32_t *keys, int n, int shift, int32_t *hist)
{
    __shared__ int cnt[256];
    const int tid = threadIdx.x, blk = blockIdx.x, nblk = gridDim.x;
    cnt[tid] = 0;
    __syncthreads();
    for (int r = 0; r < kSortSeg / 256; r++) {
        const int p = blk * kSortSeg + r * 256 + tid;
        if (p < n) atomicAdd(&cnt[(keys[p] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[(size_t)tid * nblk + blk] = cnt[tid];
}

// exclusive scan of m counts in place by one workgroup
__global__ __launch_bounds__(1024) void sort_scan_kernel(int32_t *hist, int m)
{
    __shared__ int part[1024];
    const int tid = threadIdx.x;
    const int per = (m + 1023) / 1024;
    const int lo = min(m, tid * per), hi = min(m, lo + per);
    int s = 0;
    for (int i = lo; i < hi; i++) s += hist[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int i = lo; i < hi; i++) {
        const int c = hist[i];
        hist[i] = run;
        run += c;
    }
}

__global__ __launch_bounds__(256) void sort_scatter_kernel(const uint32_t *kin, const int32_t *iin, uint32_t *kout,
                                                           int32_t *iout, int n, int shift, const int32_t *hist)
{
    __shared__ int dig[256];
    __shared__ int base[256];
    const int tid = threadIdx.x, blk = blockIdx.x, nblk = gridDim.x;
    base[tid] = 0;
    __syncthreads();
    for (int r = 0; r < kSortSeg / 256; r++) {
        const int p = blk * kSortSeg + r * 256 + tid;
        const bool ok = p < n;
        const uint32_t k = ok ? kin[p] : 0u;
        const int d = ok ? (int)((k >> shift) & 255) : 256;
        dig[tid] = d;
        __syncthreads();
        if (ok) {
            int rank = 0;
            for (int j = 0; j < tid; j++) rank += dig[j] == d;
            const int pos = hist[(size_t)d * nblk + blk] + base[d] + rank;
            kout[pos] = k;
            iout[pos] = iin[p];
        }
        __syncthreads();
        int c = 0;
        for (int j = 0; j < 256; j++) c += dig[j] == tid;
        base[tid] += c;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launch configuration
struct Config {
    int precision, tile, waves, schedule, n_long, launch, reorder;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct TileLayout {
    size_t off_y, off_vec, off_ctl, off_part, bytes;
    int nbb;
};

// One tile's block of the workspace: LU values, right-hand sides / steps, the per-bus
// vectors (|V|, angle, P and Q set points, rectangular V), then for the per-phase launches
// the instances' states (status, iterations, updates, active) with two tile flags (any
// instance active, internal error), and the mismatch kernel's per-bus-block maxima.
static TileLayout tile_layout(const HostPlan &h, const Config &c)
{
    const size_t rs = c.precision == PF_FP32_LU ? 4 : 8;
    TileLayout L;
    L.off_y = align256((size_t)(h.col_ptr.empty() ? 0 : h.col_ptr[h.N]) * c.tile * rs);
    L.off_vec = L.off_y + align256((size_t)h.N * c.tile * rs);
    L.off_ctl = L.off_vec + align256((size_t)6 * h.n * c.tile * 8);
    L.off_part = L.off_ctl + align256((size_t)40 * c.tile + 16);
    L.nbb = (h.n + kMBlock / c.tile - 1) / (kMBlock / c.tile);
    L.bytes = L.off_part + align256((size_t)L.nbb * c.tile * 12);
    return L;
}

static size_t lds_bytes(const HostPlan &h, const Config &c)
{
    const size_t rs = c.precision == PF_FP32_LU ? 4 : 8;
    return ((size_t)c.waves * 2 * ((size_t)h.slot_rows * c.tile + 2 * c.tile) + (size_t)c.n_long * 2 * h.max_col * c.tile) * rs +
           (size_t)h.N + (size_t)h.n_longp;
}

static size_t lds_bytes(const HostPlan &h, const Config &c);
static constexpr size_t kLdsLimit = 160 * 1024 - 8192;

// Explicit tile/waves are validated.  A zero picks the value that minimises a latency
// model of the solve: a tile's time grows with the panels each wavefront handles in turn
// (n_panels / waves), mildly with the rows per lane (1 + T/32), and falls with the long
// working-column slots L as 0.76 + 0.48 / L (fitted to the 1350-bus grid: 32.2 / 29.1 /
// 27.6 ms with 2 / 3 / 4 slots): the long panels form the serial tail of the elimination,
// and a long panel can only start once the panel that held its slot before has
// published, so more slots let more of the tail overlap.  Tiles run in
// max(1, tiles / resident workgroups) generations, where the resident workgroups per CU are
// limited by LDS and by the 16 wavefronts per CU that four waves per SIMD allow.  Within 3%
// of the lowest cost, 8-wave workgroups are preferred, then more resident workgroups.  An
// automatic L is, for each candidate, the most slots (up to kMaxLong) that keep the resident
// workgroups per CU the batch can use.  batch <= 0 assumes a batch much larger than the GPU.
static bool resolve_config(const HostPlan &h, const pf_solve_opts *o, Config &c, std::string &err,
                           int64_t batch = 0, bool solve = true)
{
    c.precision = o ? o->precision : PF_FP64;
    c.schedule = o ? o->schedule : 0;
    c.launch = o ? o->launch : PF_LAUNCH_AUTO;
    if (c.launch < PF_LAUNCH_AUTO || c.launch > PF_LAUNCH_PHASES) { err = "launch must be 0, 1 or 2"; return false; }
    c.reorder = o ? o->reorder : PF_REORDER_AUTO;
    if (c.reorder != PF_REORDER_AUTO && c.reorder != PF_REORDER_OFF) { err = "reorder must be 0 or 1"; return false; }
    if (c.schedule != 0 && c.schedule != 1) { err = "schedule must be 0 or 1"; return false; }
    const int long_slots = o ? o->long_slots : 0;
    if (long_slots < 0 || long_slots > kMaxLong) {
        err = "long_slots must be 0.." + std::to_string(kMaxLong);
        return false;
    }
    const int nl_max = std::min(kMaxLong, h.n_longp);
    const int tile = o ? o->tile : 0, waves = o ? o->waves : 0;
    if (c.precision != PF_FP64 && c.precision != PF_FP32_LU) { err = "unknown precision"; return false; }
    const bool fp64 = c.precision == PF_FP64;
    if (tile != 0 && !(fp64 ? (tile == 4 || tile == 8 || tile == 16) : (tile == 8 || tile == 16 || tile == 32))) {
        err = "unsupported tile size for this precision"; return false;
    }
    if (waves != 0 && waves != 2 && waves != 4 && waves != 8 && waves != 16) {
        err = "waves must be 2, 4, 8 or 16"; return false;
    }
    static const int tiles64[] = {4, 8, 16}, tiles32[] = {8, 16, 32}, wv[] = {2, 4, 8, 16};
    const double b = batch > 0 ? (double)batch : 1e9;
    auto resident = [&](const Config &k) {
        const size_t lds = lds_bytes(h, k);
        return lds > kLdsLimit ? 0 : (int)std::min<size_t>(kLdsLimit / lds, 16 / k.waves);
    };
    struct Cand { int tile, waves, n_long, wg; double cost; };
    std::vector<Cand> cands;
    for (const int tc : (fp64 ? tiles64 : tiles32))
        for (const int wc : wv) {
            if ((tile && tc != tile) || (waves && wc != waves)) continue;
            Config k = c;
            k.tile = tc;
            k.waves = wc;
            k.n_long = long_slots ? std::min(long_slots, nl_max) : std::min(2, nl_max);
            const int wg0 = resident(k);
            if (wg0 == 0) continue;
            if (!long_slots && k.n_long > 0) {
                const int usable = (int)std::max(1.0, std::ceil(std::ceil(b / tc) / 256.0));
                const int keep = std::min(wg0, usable);
                Config m = k;
                for (int nl = k.n_long + 1; nl <= nl_max; nl++) {
                    m.n_long = nl;
                    if (resident(m) >= keep) k.n_long = nl;
                }
            }
            const int wg = std::max(1, resident(k));
            const double gens = std::max(1.0, std::ceil(b / tc) / (256.0 * wg));
            const double slots = k.n_long > 0 ? 0.76 + 0.48 / k.n_long : 1.0;
            cands.push_back(Cand{tc, wc, k.n_long, wg, gens / wc * (1.0 + tc / 32.0) * slots});
        }
    if (!cands.empty()) {
        double lo = cands[0].cost;
        for (const Cand &k : cands) lo = std::min(lo, k.cost);
        const Cand *pick = nullptr;
        for (const Cand &k : cands) {
            if (k.cost > lo * 1.03) continue;
            if (!pick) { pick = &k; continue; }
            const bool k8 = k.waves == 8, p8 = pick->waves == 8;
            if (k8 != p8) { if (k8) pick = &k; continue; }
            if (k.wg != pick->wg) { if (k.wg > pick->wg) pick = &k; continue; }
            if (k.cost < pick->cost) pick = &k;
        }
        c.tile = pick->tile;
        c.waves = pick->waves;
        c.n_long = pick->n_long;
        // per-phase launches for grids whose iterations are long against a launch (at least
        // 10,000 LU entries): each phase runs without the fused kernel's spills, and a
        // batch of several generations of tiles is cut into one-generation chunks on
        // concurrent streams.  Small grids keep the single fused launch, where three
        // launches per iteration would cost more than the phases gain.
        if (c.launch == PF_LAUNCH_AUTO)
            c.launch = h.col_ptr[h.N] >= kPhasesMinLu ? PF_LAUNCH_PHASES : PF_LAUNCH_FUSED;
        // The model above was fitted to the fused kernel.  The per-phase refactorisation
        // fits a 16-instance tile of eight wavefronts in one CU's registers; in FP64, when
        // four long slots still fit and the batch spans two generations of such tiles, one
        // 16-instance tile per CU out-runs one 8-instance tile of sixteen wavefronts
        // (1350-bus grid, 10,000 instances: 23.9 -> 23.0 ms per solve; with a single long
        // slot, the 9000-bus grid's would be 2.4x slower, so that case keeps the model's).
        if (solve && c.launch == PF_LAUNCH_PHASES && fp64 && !tile && !waves && !long_slots && b >= 2 * 256.0 * 16) {
            Config k = c;
            k.tile = 16;
            k.waves = 8;
            for (k.n_long = std::min(kMaxLong, h.n_longp); k.n_long >= 4 && lds_bytes(h, k) > kLdsLimit; k.n_long--) {}
            if (k.n_long >= 4 && lds_bytes(h, k) <= kLdsLimit) c = k;
        }
        return true;
    }
    err = "the longest LU column (" + std::to_string(h.max_col) + " entries) does not fit in LDS for any "
          "supported tile/wave configuration";
    return false;
}

template <typename F>
static hipError_t allow_lds(F fn, size_t lds)
{
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(160 * 1024 - 8192));
}

template <typename R, int T, int NW>
static hipError_t launch_t(const KArgs &a, int grid, size_t lds, hipStream_t st)
{
    auto fn = nr_tile_kernel<R, T, NW>;
    const hipError_t e = allow_lds(fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NW * 64), lds, st, a);
    return hipGetLastError();
}

#define PF_DISPATCH_NW(R, T)                                                   \
    switch (c.waves) {                                                         \
    case 2: return launch_t<R, T, 2>(a, grid, lds, st);                        \
    case 4: return launch_t<R, T, 4>(a, grid, lds, st);                        \
    case 16: return launch_t<R, T, 16>(a, grid, lds, st);                      \
    default: return launch_t<R, T, 8>(a, grid, lds, st);                       \
    }

// The persistent queue kernel for a launch configuration.
template <typename R, int T>
static const void *queue_kernel_nw(int waves)
{
    if (waves == 2) return reinterpret_cast<const void *>(nr_queue_kernel<R, T, 2>);
    if (waves == 4) return reinterpret_cast<const void *>(nr_queue_kernel<R, T, 4>);
    if (waves == 16) return reinterpret_cast<const void *>(nr_queue_kernel<R, T, 16>);
    return reinterpret_cast<const void *>(nr_queue_kernel<R, T, 8>);
}

static const void *queue_kernel(const Config &c)
{
    if (c.precision == PF_FP64) {
        if (c.tile == 4) return queue_kernel_nw<double, 4>(c.waves);
        if (c.tile == 8) return queue_kernel_nw<double, 8>(c.waves);
        return queue_kernel_nw<double, 16>(c.waves);
    }
    if (c.tile == 8) return queue_kernel_nw<float, 8>(c.waves);
    if (c.tile == 16) return queue_kernel_nw<float, 16>(c.waves);
    return queue_kernel_nw<float, 32>(c.waves);
}

static hipError_t launch(const Config &c, const KArgs &a, int grid, size_t lds, hipStream_t st)
{
    if (c.precision == PF_FP64) {
        if (c.tile == 4) { PF_DISPATCH_NW(double, 4) }
        if (c.tile == 8) { PF_DISPATCH_NW(double, 8) }
        PF_DISPATCH_NW(double, 16)
    } else {
        if (c.tile == 8) { PF_DISPATCH_NW(float, 8) }
        if (c.tile == 16) { PF_DISPATCH_NW(float, 16) }
        PF_DISPATCH_NW(float, 32)
    }
}

// The per-phase launches of one solve: layout in, then per iteration the mismatch and
// Jacobian, the refactorization (with the convergence decision first) and the back
// substitution, then the final mismatch, decision and layout out.  A part of the sequence:
// with head the layout in, iterations [it0, it1), with tail the final pass and layout out.
// With a fallback start, the attempts' updates and the restart's decision take at most
// 2 max_iter + 1 iterations.
static int phase_iterations(const KArgs &a) { return a.v_fb ? 2 * a.max_iter + 1 : a.max_iter; }

template <typename R, int T, int NW>
static hipError_t launch_phases_t(const KArgs &a, int ntiles, size_t lds, hipStream_t st, bool head, int it0, int it1,
                                  bool tail, const double *vsrc, const int4 *csrc)
{
    auto lu = split_lu_kernel<R, T, NW>;
    auto bs = split_bs_kernel<R, T, NW>;
    hipError_t e = allow_lds(lu, lds);
    if (e != hipSuccess) return e;
    // The substitution's dynamic LDS: its rows' publication bytes and, in the wide form only,
    // z of the dense tail (kBsZBytes).  Without that cache a substitution workgroup fits
    // beside a refactorization workgroup on a CU whenever the wavefronts allow, so one
    // chunk's substitution runs beside another chunk's refactorization instead of waiting
    // for its CU (1350-bus grid, 10,000 instances, FP64 16 x 8 tiles: 22.9 -> 21.7 ms per
    // solve with the 48 KB that used to be reserved whatever the form).
    KArgs ab = a;
    ab.bs_zbytes = kWideBs<R> ? (int)kBsZBytes : 0;
    const size_t bs_lds = (((size_t)a.p.N + 255) & ~(size_t)255) + (size_t)ab.bs_zbytes;
    if ((e = allow_lds(bs, bs_lds)) != hipSuccess) return e;
    const int mgrid = std::max(1, std::min(ntiles * a.nbb, 4096));
    const dim3 sgrid(ntiles, stage_splits<T>(a.p.n));
    if (head) hipLaunchKernelGGL(split_in_kernel<T>, sgrid, dim3(kMBlock), 0, st, a, vsrc ? vsrc : a.v0, csrc);
    for (int k = it0; k < it1; k++) {
        hipLaunchKernelGGL(split_v_kernel<T>, dim3(mgrid), dim3(kMBlock), 0, st, a, ntiles);
        hipLaunchKernelGGL((split_m_kernel<R, T>), dim3(mgrid), dim3(kMBlock), 0, st, a, ntiles, 1);
        hipLaunchKernelGGL(lu, dim3(ntiles), dim3(NW * 64), lds, st, a);
        hipLaunchKernelGGL(bs, dim3(ntiles), dim3(NW * 64), bs_lds, st, ab);
    }
    if (tail) {
        hipLaunchKernelGGL(split_v_kernel<T>, dim3(mgrid), dim3(kMBlock), 0, st, a, ntiles);
        hipLaunchKernelGGL((split_m_kernel<R, T>), dim3(mgrid), dim3(kMBlock), 0, st, a, ntiles, 0);
        hipLaunchKernelGGL(split_out_kernel<T>, sgrid, dim3(kMBlock), 0, st, a);
    }
    return hipGetLastError();
}

// Reorders a batch hardest first after its first update (see split_key_kernel): the sort
// key per slot and two radix passes (ids0 receives the sorted slots, which are the
// instances), and every instance's |V|, angle and control words parked in instance order.
template <typename R, int T>
static hipError_t launch_reorder_t(const KArgs &a, int ntiles, hipStream_t st, uint32_t *keys0, int32_t *ids0,
                                   uint32_t *keys1, int32_t *ids1, int32_t *hist, double *park, int4 *ctl_park)
{
    const int n = a.batch, nblk = (n + kSortSeg - 1) / kSortSeg;
    hipLaunchKernelGGL((split_key_kernel<R, T>), dim3(ntiles), dim3(kMBlock), 0, st, a, keys0, ids0);
    for (int pass = 0; pass < 2; pass++) {
        const uint32_t *ki = pass ? keys1 : keys0;
        const int32_t *ii = pass ? ids1 : ids0;
        uint32_t *ko = pass ? keys0 : keys1;
        int32_t *io = pass ? ids0 : ids1;
        hipLaunchKernelGGL(sort_hist_kernel, dim3(nblk), dim3(256), 0, st, ki, n, 8 * pass, hist);
        hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(1024), 0, st, hist, 256 * nblk);
        hipLaunchKernelGGL(sort_scatter_kernel, dim3(nblk), dim3(256), 0, st, ki, ii, ko, io, n, 8 * pass, hist);
    }
    hipLaunchKernelGGL(split_park_kernel<T>, dim3(ntiles, stage_splits<T>(a.p.n)), dim3(kMBlock), 0, st, a, park,
                       ctl_park);
    return hipGetLastError();
}

// workgroups of the refactorization kernel that fit on one CU (registers, LDS, waves)
template <typename R, int T, int NW>
static hipError_t lu_residency_t(size_t lds, int *nb)
{
    auto lu = split_lu_kernel<R, T, NW>;
    hipError_t e = allow_lds(lu, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, lu, NW * 64, lds);
}

#define PF_DISPATCH_PHASES_NW(R, T)                                                                     \
    switch (c.waves) {                                                                                  \
    case 2: return launch_phases_t<R, T, 2>(a, grid, lds, st, head, it0, it1, tail, vsrc, csrc);        \
    case 4: return launch_phases_t<R, T, 4>(a, grid, lds, st, head, it0, it1, tail, vsrc, csrc);        \
    case 16: return launch_phases_t<R, T, 16>(a, grid, lds, st, head, it0, it1, tail, vsrc, csrc);      \
    default: return launch_phases_t<R, T, 8>(a, grid, lds, st, head, it0, it1, tail, vsrc, csrc);       \
    }

static hipError_t launch_phases(const Config &c, const KArgs &a, int grid, size_t lds, hipStream_t st,
                                bool head = true, int it0 = 0, int it1 = -1, bool tail = true,
                                const double *vsrc = nullptr, const int4 *csrc = nullptr)
{
    if (it1 < 0) it1 = phase_iterations(a);
    if (c.precision == PF_FP64) {
        if (c.tile == 4) { PF_DISPATCH_PHASES_NW(double, 4) }
        if (c.tile == 8) { PF_DISPATCH_PHASES_NW(double, 8) }
        PF_DISPATCH_PHASES_NW(double, 16)
    } else {
        if (c.tile == 8) { PF_DISPATCH_PHASES_NW(float, 8) }
        if (c.tile == 16) { PF_DISPATCH_PHASES_NW(float, 16) }
        PF_DISPATCH_PHASES_NW(float, 32)
    }
}

#define PF_DISPATCH_RESIDENCY_NW(R, T)                                         \
    switch (c.waves) {                                                         \
    case 2: return lu_residency_t<R, T, 2>(lds, nb);                           \
    case 4: return lu_residency_t<R, T, 4>(lds, nb);                           \
    case 16: return lu_residency_t<R, T, 16>(lds, nb);                         \
    default: return lu_residency_t<R, T, 8>(lds, nb);                          \
    }

static hipError_t lu_residency(const Config &c, size_t lds, int *nb)
{
    if (c.precision == PF_FP64) {
        if (c.tile == 4) { PF_DISPATCH_RESIDENCY_NW(double, 4) }
        if (c.tile == 8) { PF_DISPATCH_RESIDENCY_NW(double, 8) }
        PF_DISPATCH_RESIDENCY_NW(double, 16)
    } else {
        if (c.tile == 8) { PF_DISPATCH_RESIDENCY_NW(float, 8) }
        if (c.tile == 16) { PF_DISPATCH_RESIDENCY_NW(float, 16) }
        PF_DISPATCH_RESIDENCY_NW(float, 32)
    }
}

static hipError_t launch_reorder(const Config &c, const KArgs &a, int ntiles, hipStream_t st, uint32_t *k0,
                                 int32_t *i0, uint32_t *k1, int32_t *i1, int32_t *hist, double *park, int4 *cp)
{
    if (c.precision == PF_FP64) {
        if (c.tile == 4) return launch_reorder_t<double, 4>(a, ntiles, st, k0, i0, k1, i1, hist, park, cp);
        if (c.tile == 8) return launch_reorder_t<double, 8>(a, ntiles, st, k0, i0, k1, i1, hist, park, cp);
        return launch_reorder_t<double, 16>(a, ntiles, st, k0, i0, k1, i1, hist, park, cp);
    }
    if (c.tile == 8) return launch_reorder_t<float, 8>(a, ntiles, st, k0, i0, k1, i1, hist, park, cp);
    if (c.tile == 16) return launch_reorder_t<float, 16>(a, ntiles, st, k0, i0, k1, i1, hist, park, cp);
    return launch_reorder_t<float, 32>(a, ntiles, st, k0, i0, k1, i1, hist, park, cp);
}

static int upload(Plan *pl);

// Validates a solve's arguments and fills its kernel arguments (shared by pf_solve_batch,
// the single-step entry points and the queue).
static int make_args(Plan *pl, const Config &c, int32_t batch, const double *ybus, const double *sbus,
                     const double *v0, double tol, int32_t max_iter, void *workspace, size_t workspace_bytes,
                     int mode, double *v_out, int32_t *iters_out, uint8_t *conv_out, int8_t *status_out,
                     double *aux, double *aux2, KArgs &a, int &ntiles, size_t &lds)
{
    const HostPlan &h = pl->h;
    if (!ybus || !sbus || !v0) { set_error("null input pointer"); return PF_EINVAL; }
    if (mode == MODE_SOLVE && (!v_out || !iters_out || !conv_out)) { set_error("null output pointer"); return PF_EINVAL; }
    if (mode != MODE_SOLVE && !aux) { set_error("null output pointer"); return PF_EINVAL; }
    if (mode == MODE_MISMATCH && !aux2) { set_error("null output pointer"); return PF_EINVAL; }
    if (mode == MODE_SOLVE && (max_iter < 0 || !(tol >= 0.0))) { set_error("invalid tol or max_iter"); return PF_EINVAL; }
    const TileLayout L = tile_layout(h, c);
    ntiles = (batch + c.tile - 1) / c.tile;
    const size_t need = L.bytes * (size_t)ntiles;
    if (!workspace || workspace_bytes < need) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return PF_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) { set_error("workspace must be 256-byte aligned"); return PF_EINVAL; }
    lds = lds_bytes(h, c);
    if (lds > kLdsLimit) {
        set_error("longest LU column needs " + std::to_string(lds) + " B of LDS; use a smaller tile or fewer waves");
        return PF_EINVAL;
    }
    if (!pl->dev_mem) {
        const int rcu = upload(pl);
        if (rcu != PF_OK) return rcu;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != pl->device) {
        set_error("the current device differs from the plan's device");
        return PF_EDEVICE;
    }
    std::memset(&a, 0, sizeof(a));
    a.p = pl->d;
    a.perm = pl->perm_dev;
    a.ybus = ybus; a.sbus = sbus; a.v0 = v0;
    a.tol = tol; a.max_iter = max_iter; a.batch = batch; a.mode = mode;
    a.ws = reinterpret_cast<char *>(workspace);
    a.tile_bytes = L.bytes; a.off_y = L.off_y; a.off_vec = L.off_vec;
    a.off_ctl = L.off_ctl; a.off_part = L.off_part; a.nbb = L.nbb;
    a.sched = c.schedule;
    // the kernel derives a long panel's slot from its rank with this reciprocal; a count
    // outside 1..kMaxLong (0 only without long panels) would index past the slot counters
    if (c.n_long < (h.n_longp > 0 ? 1 : 0) || c.n_long > kMaxLong) {
        set_error("internal: long-slot count out of range");
        return PF_EINVAL;
    }
    a.n_long = c.n_long;
    a.v_out = v_out; a.iters_out = iters_out; a.conv_out = conv_out; a.status_out = status_out;
    a.aux_out = aux; a.aux2_out = aux2;
    return PF_OK;
}

// Per-phase launches over a batch of several generations of tiles: the batch is cut into
// chunks of one generation each (the tiles whose refactorization workgroups fit on the
// device at once), and the chunks' launch sequences go to four workers: the caller's
// stream and three pool streams (default priority) that start after it and that it waits
// for.  A chunk whose instances need many iterations then overlaps the other chunks' work
// instead of running alone after them.  When the workspace holds the reorder area, the
// first update runs over the whole batch on the caller's stream, the batch is reordered
// hardest first, and the first chunk (the hardest instances) gets the caller's stream to
// itself.  The pool and its events are created once per device and kept; `pooled` = false
// (the allocation-free entry point) keeps everything on the caller's stream.
constexpr int kPhaseStreams = 3;
constexpr int kHeadTiles = 32;
// without a head, the first chunk: the hardest instances in this many of the batch's own
// tiles (9000-bus grid, 2,000 FP32-LU instances in tiles of eight: 40.2 ms per solve with 8
// tiles, 40.6 with 16, 41.0 with 32)
constexpr int kLeadTiles = 8;
struct PhasePool {
    hipStream_t st[kPhaseStreams] = {};
    hipEvent_t start = nullptr, fin[kPhaseStreams] = {};
    int cus = 0;
    bool ready = false;
};
static std::mutex g_pool_mu;
static PhasePool g_pool[64];

// The head of a reordered batch runs in a low-latency form: tiles of four instances (sixteen
// sub-lanes each), sixteen wavefronts, and as many long slots as fit (measured per iteration
// of one tile on the 1350-bus grid: FP64 0.56 ms against 0.62 ms with eight instances; four
// instances also beat two over whole solves), in the fused kernel or, for FP64 from the
// given start, as per-phase launches.
static bool head_config(const HostPlan &h, const Config &c, Config &ch)
{
    ch = c;
    ch.tile = 4;
    ch.waves = 16;
    ch.launch = PF_LAUNCH_FUSED;
    const int lo = h.n_longp > 0 ? 1 : 0;
    for (ch.n_long = std::min(kMaxLong, h.n_longp); ch.n_long >= lo; ch.n_long--)
        if (lds_bytes(h, ch) <= kLdsLimit) return true;
    return false;
}

// bytes after the tiles' blocks that the reorder needs: two key and two slot arrays of batch
// words, the radix sort's (digit, block) counts, the parked |V| and angle rows
// ([batch][n][2]) and control words (three int4 per instance), and the head's tiles
static size_t order_bytes(const HostPlan &h, const Config &c, int64_t batch)
{
    const size_t nblk = (size_t)((batch + kSortSeg - 1) / kSortSeg);
    size_t bytes = 4 * align256((size_t)batch * 4) + align256(nblk * 256 * 4) + align256((size_t)batch * h.n * 16) +
                   align256((size_t)batch * 48);
    Config ch;
    if (head_config(h, c, ch)) bytes += (size_t)kHeadTiles * tile_layout(h, ch).bytes;
    return bytes;
}

#define PF_HEAD_LAUNCH(R, TH, PAIR)                                                           \
    {                                                                                         \
        auto fn = nr_head_kernel<R, TH, 16, PAIR>;                                            \
        hipError_t e = allow_lds(fn, lds);                                                    \
        if (e != hipSuccess) return e;                                                        \
        hipLaunchKernelGGL(fn, dim3(grid), dim3(16 * 64), lds, st, ah);                       \
        return hipGetLastError();                                                             \
    }

// pair: a warm-started batch, two slots per instance (see nr_tile_body)
static hipError_t launch_head(const Config &ch, const KArgs &ah, int grid, size_t lds, hipStream_t st, bool pair)
{
    if (ch.precision == PF_FP64) {
        if (pair) PF_HEAD_LAUNCH(double, 4, true)
        PF_HEAD_LAUNCH(double, 4, false)
    }
    if (pair) PF_HEAD_LAUNCH(float, 4, true)
    PF_HEAD_LAUNCH(float, 4, false)
}

static hipError_t launch_phases_chunked(const HostPlan &h, const Config &c, const KArgs &a, int ntiles, size_t lds,
                                        hipStream_t user, bool pooled, bool reorder)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (!pooled || dev < 0 || dev >= 64) return launch_phases(c, a, ntiles, lds, user);
    std::lock_guard<std::mutex> lk(g_pool_mu);
    PhasePool &pp = g_pool[dev];
    if (!pp.ready) {
        if ((e = hipDeviceGetAttribute(&pp.cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        for (int i = 0; i < kPhaseStreams; i++) {
            if ((e = hipStreamCreateWithFlags(&pp.st[i], hipStreamNonBlocking)) != hipSuccess) return e;
            if ((e = hipEventCreateWithFlags(&pp.fin[i], hipEventDisableTiming)) != hipSuccess) return e;
        }
        if ((e = hipEventCreateWithFlags(&pp.start, hipEventDisableTiming)) != hipSuccess) return e;
        pp.ready = true;
    }
    int per_cu = 0;
    if ((e = lu_residency(c, lds, &per_cu)) != hipSuccess) return e;
    const int gen = std::max(1, pp.cus * std::max(1, per_cu));
    const int nchunk = (ntiles + gen - 1) / gen;
    const int iters = phase_iterations(a);
    // a batch of at least half a generation is still worth reordering: its few long chains
    // would otherwise keep every tile's launches going until they end
    if (nchunk <= 1 && !(reorder && iters > 1 && 2 * ntiles >= gen)) return launch_phases(c, a, ntiles, lds, user);
    const int32_t *order = nullptr;
    double *park = nullptr;
    int4 *ctl_park = nullptr;
    Config ch;
    // The hardest instances run as the head (below), except in an FP32-LU flat-start batch
    // of at most one generation: there they are the first chunk of the batch's own tiles
    // (9000-bus grid, 2,000 instances: 43.3 -> 40.3 ms per solve against the fused FP32 head,
    // which spills; in FP64 the head's four-instance tiles are the faster, 53.1 against
    // 58.5 ms with the batch's eight; with more generations the fused FP32 head stays ahead,
    // 1350-bus 14.9 against 15.1-15.5 ms)
    const bool head = reorder && head_config(h, c, ch) && !(c.precision == PF_FP32_LU && nchunk <= 1 && !a.v_fb);
    char *head_ws = nullptr;
    if (reorder && iters > 1) {
        char *ob = a.ws + (size_t)ntiles * a.tile_bytes;
        const size_t w = align256((size_t)a.batch * 4);
        uint32_t *k0 = reinterpret_cast<uint32_t *>(ob);
        int32_t *i0 = reinterpret_cast<int32_t *>(ob + w);
        uint32_t *k1 = reinterpret_cast<uint32_t *>(ob + 2 * w);
        int32_t *i1 = reinterpret_cast<int32_t *>(ob + 3 * w);
        int32_t *hist = reinterpret_cast<int32_t *>(ob + 4 * w);
        const size_t nblk = (size_t)((a.batch + kSortSeg - 1) / kSortSeg);
        park = reinterpret_cast<double *>(ob + 4 * w + align256(nblk * 256 * 4));
        ctl_park = reinterpret_cast<int4 *>(reinterpret_cast<char *>(park) + align256((size_t)a.batch * a.p.n * 16));
        head_ws = reinterpret_cast<char *>(ctl_park) + align256((size_t)a.batch * 48);
        if ((e = launch_phases(c, a, ntiles, lds, user, true, 0, 1, false)) != hipSuccess) return e;
        if ((e = launch_reorder(c, a, ntiles, user, k0, i0, k1, i1, hist, park, ctl_park)) != hipSuccess) return e;
        order = i0;
    }
    // With the reorder, the head (the hardest instances: kHeadTiles tiles of the head
    // configuration) runs alone on the caller's stream (one fused launch, or its per-phase
    // launches): its workgroups run their long iteration chains at one tile's latency per
    // iteration.
    // The other instances follow in one-generation chunks of per-phase launches on the pool's
    // streams (on every worker without the reorder).
    // the pool's streams start after the reorder, not after the head
    if ((e = hipEventRecord(pp.start, user)) != hipSuccess) return e;
    int hcount = 0, hgrid = 0;
    if (order && head) {
        // with a fallback start each head instance takes two slots: its attempt from the
        // given start and, at the same time, its flat-start restart, so that the longest
        // chains (an attempt that fails, then a full restart) take the longer of the two
        // instead of their sum
        const bool pair = a.v_fb != nullptr;
        const TileLayout Lh = tile_layout(h, ch);
        // pairs for the first half of the head's tiles, single slots for the rest
        const int pslots = pair ? std::min(kHeadTiles / 2 * ch.tile, 2 * a.batch) & ~(2 * ch.tile - 1) : 0;
        hcount = std::min(a.batch, pslots / 2 + kHeadTiles * ch.tile - pslots);
        const int hslots = hcount + pslots / 2;
        KArgs ah = a;
        ah.ws = head_ws;
        ah.tile_bytes = Lh.bytes; ah.off_y = Lh.off_y; ah.off_vec = Lh.off_vec;
        ah.off_ctl = Lh.off_ctl; ah.off_part = Lh.off_part; ah.nbb = Lh.nbb;
        ah.n_long = ch.n_long;
        ah.batch = hslots;
        ah.inst = order;
        ah.vpark = park;
        ah.cpark = ctl_park;
        ah.pair_slots = pslots;
        hgrid = (hslots + ch.tile - 1) / ch.tile;
        if (!pair && ch.precision == PF_FP64) {
            // FP64 from the given start: the head's tiles as per-phase launches, whose
            // refactorization keeps its wider loads without spilling (9000-bus grid, 2,000
            // instances: 53.1 -> 51.8 ms per solve; the 1350-bus grid unchanged); a
            // warm-started head needs the fused kernel's paired slots
            Config cp = ch;
            cp.launch = PF_LAUNCH_PHASES;
            if ((e = launch_phases(cp, ah, hgrid, lds_bytes(h, cp), user, true, 1, iters, true, park, ctl_park)) !=
                hipSuccess)
                return e;
        } else if ((e = launch_head(ch, ah, hgrid, lds_bytes(h, ch), user, pair)) != hipSuccess)
            return e;
    }
    const int btiles = (a.batch - hcount + c.tile - 1) / c.tile;
    // the head's workgroups hold their CUs (fused) or keep returning to them (per-phase): a
    // generation of the others fits the rest (sized for every CU instead, the 9000-bus bulk
    // slows the head: 51.8 -> 57.3 ms)
    const int bgen = hcount > 0 ? std::max(1, (pp.cus - std::min(hgrid, pp.cus / 2)) * std::max(1, per_cu)) : gen;
    std::vector<int> cut{0};
    if (order && !head) cut.push_back(std::min(btiles, kLeadTiles));
    while (cut.back() < btiles) cut.push_back(std::min(btiles, cut.back() + bgen));
    const int nparts = (int)cut.size() - 1;
    // workers: 0 = the caller's stream, then the pool's streams; with a head the caller's
    // stream holds only the head
    hipStream_t wk[kPhaseStreams + 1] = {user, pp.st[0], pp.st[1], pp.st[2]};
    const int w0 = hcount > 0 ? 1 : 0;
    const int nw = std::min(nparts + w0, kPhaseStreams + 1);
    for (int i = 1; i < nw; i++)
        if ((e = hipStreamWaitEvent(wk[i], pp.start, 0)) != hipSuccess) return e;
    const size_t n2 = (size_t)2 * a.p.n;
    for (int ci = 0; ci < nparts; ci++) {
        const int t0 = cut[ci], nt = cut[ci + 1] - cut[ci];
        const size_t b0 = (size_t)t0 * c.tile;
        KArgs ac = a;
        ac.batch = (int)std::min<size_t>((size_t)(a.batch - hcount) - b0, (size_t)nt * c.tile);
        ac.ws = a.ws + (size_t)t0 * a.tile_bytes;
        int w;
        if (order) {
            // slots now name instances through the order; the boundary arrays stay whole
            ac.inst = order + hcount + b0;
            if (hcount > 0) w = 1 + ci % (nw - 1);
            else w = (nw == 1 || ci == 0) ? 0 : 1 + (ci - 1) % (nw - 1);
        } else {
            w = ci % nw;
            ac.sbus = a.sbus + b0 * n2;
            ac.v0 = a.v0 + b0 * n2;
            if (a.v_fb) ac.v_fb = a.v_fb + b0 * n2;
            ac.ybus = a.ybus + b0 * a.ybus_stride;
            ac.v_out = a.v_out + b0 * n2;
            ac.iters_out = a.iters_out + b0;
            ac.conv_out = a.conv_out + b0;
            if (a.status_out) ac.status_out = a.status_out + b0;
        }
        if ((e = launch_phases(c, ac, nt, lds, wk[w], true, order ? 1 : 0, iters, true, park, ctl_park)) != hipSuccess)
            return e;
    }
    for (int i = 1; i < nw; i++) {
        if ((e = hipEventRecord(pp.fin[i - 1], wk[i])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(user, pp.fin[i - 1], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

static int run(pf_plan plan_h, int32_t batch, const double *ybus, const double *sbus, const double *v0,
               double tol, int32_t max_iter, const pf_solve_opts *opts, void *workspace,
               size_t workspace_bytes, int mode, double *v_out, int32_t *iters_out, uint8_t *conv_out,
               int8_t *status_out, double *aux, double *aux2, void *stream, const double *v_fb = nullptr,
               int ybus_batched = 0, bool pooled = true)
{
    Plan *pl = reinterpret_cast<Plan *>(plan_h);
    if (!pl) { set_error("null plan"); return PF_EINVAL; }
    if (batch < 0) { set_error("negative batch"); return PF_EINVAL; }
    if (batch == 0) return PF_OK;
    Config c;
    std::string err;
    // the single-step entry points run the fused kernel: they take its configuration
    if (!resolve_config(pl->h, opts, c, err, batch, mode == MODE_SOLVE)) { set_error(err); return PF_EINVAL; }
    KArgs a;
    int ntiles = 0;
    size_t lds = 0;
    const int rc = make_args(pl, c, batch, ybus, sbus, v0, tol, max_iter, workspace, workspace_bytes, mode, v_out,
                             iters_out, conv_out, status_out, aux, aux2, a, ntiles, lds);
    if (rc != PF_OK) return rc;
    a.v_fb = v_fb;
    a.ybus_stride = ybus_batched ? (size_t)2 * pl->h.nnzy : 0;
    const bool phases = mode == MODE_SOLVE && c.launch == PF_LAUNCH_PHASES;
    const TileLayout L = tile_layout(pl->h, c);
    const bool reorder = phases && c.reorder == PF_REORDER_AUTO &&
                         workspace_bytes >= L.bytes * (size_t)ntiles + order_bytes(pl->h, c, batch);
    hipError_t e = phases ? launch_phases_chunked(pl->h, c, a, ntiles, lds, reinterpret_cast<hipStream_t>(stream),
                                                  pooled, reorder)
                          : launch(c, a, ntiles, lds, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) { set_error(std::string("kernel launch failed: ") + hipGetErrorString(e)); return PF_EDEVICE; }
    return PF_OK;
}

// ------------------------------------------------------------------ fixed scratch
// The workspace of pf_solve_batch_noalloc: a file-scope device array, so that a caller that
// cannot allocate (graph capture, serving loops) still gets a solve.  Each device holds its
// own copy at its own address, looked up once per device with hipGetSymbolAddress; host
// code passes that address, never the array's name.  No part of it needs clearing: the
// kernel writes every word of a tile's block before reading it.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static int scratch_address(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("no usable HIP device for the fixed scratch");
        return PF_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("hipGetSymbolAddress of the fixed scratch failed: ") + hipGetErrorString(e));
            return PF_EDEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PF_OK;
}

// ------------------------------------------------------------------ plan upload
// Zero padding after the tables the kernels read in whole chunks, so that those loads
// need no bounds guard (a guarded load becomes a masked load plus a register copy, and the
// copy makes the compiler wait for the load at once): update records are read 16 at a
// time from a panel's first record, back-substitution entries SL at a time (SL <= 16)
// from a row's first entry, and panel descriptors 8 per wavefront, two chunks ahead, so
// up to 23 * NW (NW <= 16) beyond the last panel.
constexpr size_t PAD_UPD = 16 * sizeof(Update);
// the per-phase refactorization reads four rows per sub-lane (SL <= 16) past a column's end
constexpr size_t PAD_ROWS = 4 * 16;
constexpr size_t PAD_BS = 64 * sizeof(int32_t);
constexpr size_t PAD_DESC = 24 * 16 * sizeof(LuPanel);
static_assert(sizeof(LuPanel) == sizeof(BsPanel), "descriptor tables share one padding");

struct DevOffsets {
    size_t bytes = 0;
    template <typename V>
    size_t add(const V &v, size_t pad = 0)
    {
        size_t o = bytes;
        bytes = align256(bytes + v.size() * sizeof(typename V::value_type) + pad + 1);
        return o;
    }
};

static int upload(Plan *pl)
{
    const HostPlan &h = pl->h;
    if (hipGetDevice(&pl->device) != hipSuccess) { set_error("no HIP device"); return PF_EDEVICE; }
    DevOffsets off;
    const size_t o_yrp = off.add(h.yrp), o_yci = off.add(h.yci);
    const size_t o_jpos = off.add(h.jpos), o_isj = off.add(h.isj, PAD_ROWS), o_rel = off.add(h.rel, 4 * PAD_ROWS);
    const size_t o_upd = off.add(h.upd, PAD_UPD);
    const size_t o_bpos = off.add(h.bs_pos, PAD_BS), o_bcol = off.add(h.bs_col, PAD_BS);
    const size_t o_pe = off.add(h.bus_peq), o_qe = off.add(h.bus_qeq);
    const size_t o_perm = off.add(h.perm);
    const size_t o_lud = off.add(h.lu_desc, PAD_DESC), o_bsd = off.add(h.bs_desc, PAD_DESC);
    const size_t o_ring = off.add(h.ring);
    std::vector<char> host(off.bytes, 0);
    auto put = [&](size_t o, const auto &v) {
        if (!v.empty()) std::memcpy(host.data() + o, v.data(), v.size() * sizeof(v[0]));
    };
    put(o_yrp, h.yrp); put(o_yci, h.yci); put(o_jpos, h.jpos); put(o_isj, h.isj); put(o_rel, h.rel);
    put(o_upd, h.upd); put(o_bpos, h.bs_pos); put(o_bcol, h.bs_col); put(o_pe, h.bus_peq);
    put(o_qe, h.bus_qeq); put(o_perm, h.perm); put(o_lud, h.lu_desc); put(o_bsd, h.bs_desc);
    put(o_ring, h.ring);
    void *dm = nullptr;
    if (hipMalloc(&dm, off.bytes) != hipSuccess) { set_error("hipMalloc of the plan failed"); return PF_ENOMEM; }
    if (hipMemcpy(dm, host.data(), off.bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dm);
        set_error("plan upload failed");
        return PF_EDEVICE;
    }
    pl->dev_mem = dm;
    pl->dev_bytes = off.bytes;
    const char *D = reinterpret_cast<const char *>(dm);
    DevPlan &d = pl->d;
    d.n = h.n; d.nnzy = h.nnzy; d.N = h.N; d.nnzlu = h.col_ptr[h.N]; d.max_col = h.max_col;
    d.yrp = (const int32_t *)(D + o_yrp); d.yci = (const int32_t *)(D + o_yci);
    d.jpos = (const JPos *)(D + o_jpos); d.isj = (const uint8_t *)(D + o_isj);
    d.rel = (const int32_t *)(D + o_rel); d.upd = (const Update *)(D + o_upd);
    d.bs_pos = (const int32_t *)(D + o_bpos); d.bs_col = (const int32_t *)(D + o_bcol);
    d.bus_peq = (const int32_t *)(D + o_pe); d.bus_qeq = (const int32_t *)(D + o_qe);
    pl->perm_dev = (const int32_t *)(D + o_perm);
    d.lu_desc = (const LuPanel *)(D + o_lud);
    d.bs_desc = (const BsPanel *)(D + o_bsd);
    d.ring = (const RingSlot *)(D + o_ring);
    d.n_panels = (int)h.panel_ptr.size() - 1;
    d.slot_rows = h.slot_rows;
    d.n_longp = h.n_longp;
    return PF_OK;
}


// ------------------------------------------------------------------ pattern hash
// FNV-1a over the sizes, bus types, Ybus pattern and elimination order: two plans with
// the same hash run the same schedule, so a tuned configuration can be reused.
static uint64_t pattern_hash(const HostPlan &h)
{
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t bytes) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < bytes; i++) { x ^= c[i]; x *= 1099511628211ull; }
    };
    mix(&h.n, sizeof(h.n));
    mix(&h.N, sizeof(h.N));
    mix(h.bus_type.data(), h.bus_type.size());
    mix(h.yrp.data(), h.yrp.size() * sizeof(int32_t));
    mix(h.yci.data(), h.yci.size() * sizeof(int32_t));
    mix(h.perm.data(), h.perm.size() * sizeof(int32_t));
    return x;
}

// ------------------------------------------------------------------ multi-pattern queue
// Work items (a plan, its instances, inputs, outputs and launch configuration) are grouped
// by precision and workgroup size; each group becomes one persistent kernel whose
// workgroups pop tiles from the group's counter.  Inside a group the items are ordered by
// decreasing cost per tile, so the largest tiles start first and the small ones fill the
// tail.  The reset kernel and the group kernels form one graph, built on the first run and
// replayed afterwards.
struct QueueItem {
    Plan *plan;
    Config c;
    int32_t batch;
    const double *ybus, *sbus, *v0;
    double tol;
    int32_t max_iter;
    double *v_out;
    int32_t *iters_out;
    uint8_t *conv_out;
    int8_t *status_out;
    unsigned long long *ticks_out;
};

struct Queue {
    int device = -1;
    std::vector<QueueItem> items;
    bool built = false;
    void *dev_mem = nullptr;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t n_tiles = 0, n_instances = 0;
    std::vector<int> grid;
    double clock_hz = 0.0;
};

static void queue_release(Queue *q)
{
    if (q->exec) (void)hipGraphExecDestroy(q->exec);
    if (q->graph) (void)hipGraphDestroy(q->graph);
    if (q->dev_mem) {
        (void)hipDeviceSynchronize();
        (void)hipFree(q->dev_mem);
    }
    q->exec = nullptr; q->graph = nullptr; q->dev_mem = nullptr;
    q->built = false;
    q->grid.clear();
}

static double tile_cost(const QueueItem &it)
{
    const HostPlan &h = it.plan->h;
    const double rs = it.c.precision == PF_FP32_LU ? 4.0 : 8.0;
    return (4.0 * rs * h.col_ptr[h.N] + 80.0 * h.n + 32.0 * h.N) * it.c.tile;
}

static int queue_build(Queue *q)
{
    queue_release(q);
    // groups keyed by (precision, tile, waves), items ordered by cost per tile
    std::map<std::tuple<int, int, int>, std::vector<int>> groups;
    for (int i = 0; i < (int)q->items.size(); i++)
        if (q->items[i].batch > 0) {
            const Config &c = q->items[i].c;
            groups[std::make_tuple(c.precision, c.tile, c.waves)].push_back(i);
        }
    for (auto &g : groups)
        std::stable_sort(g.second.begin(), g.second.end(),
                         [&](int x, int y) { return tile_cost(q->items[x]) > tile_cost(q->items[y]); });
    const int ng = (int)groups.size();
    int nitems = 0;
    for (auto &g : groups) nitems += (int)g.second.size();

    // device block: KArgs[nitems] | prefix[nitems + ng] | counters[ng] | t0 | workspaces
    const size_t off_prefix = align256(sizeof(KArgs) * (size_t)std::max(nitems, 1));
    const size_t off_counter = off_prefix + align256(sizeof(int) * (size_t)(nitems + ng + 1));
    const size_t off_t0 = off_counter + align256(sizeof(int) * (size_t)std::max(ng, 1));
    size_t off_ws = off_t0 + 256;
    std::vector<size_t> ws_off(q->items.size(), 0);
    std::vector<int> ntiles(q->items.size(), 0);
    for (auto &g : groups)
        for (int i : g.second) {
            const QueueItem &it = q->items[i];
            const TileLayout L = tile_layout(it.plan->h, it.c);
            ntiles[i] = (it.batch + it.c.tile - 1) / it.c.tile;
            ws_off[i] = off_ws;
            off_ws += align256(L.bytes * (size_t)ntiles[i]);
        }
    const size_t total = off_ws;
    if (hipMalloc(&q->dev_mem, total) != hipSuccess) {
        (void)hipGetLastError();
        q->dev_mem = nullptr;
        set_error("out of device memory for the queue (" + std::to_string(total) + " bytes)");
        return PF_ENOMEM;
    }
    char *base = static_cast<char *>(q->dev_mem);
    q->ws_bytes = total - (off_t0 + 256);
    auto *d_t0 = reinterpret_cast<unsigned long long *>(base + off_t0);
    int *d_counter = reinterpret_cast<int *>(base + off_counter);
    int *d_prefix = reinterpret_cast<int *>(base + off_prefix);
    auto *d_items = reinterpret_cast<KArgs *>(base);

    std::vector<KArgs> h_items(std::max(nitems, 1));
    std::vector<int> h_prefix(nitems + ng + 1, 0);
    struct GroupLaunch { const void *fn; int first, count, prefix_at, waves; size_t lds; };
    std::vector<GroupLaunch> gl;
    int pos = 0, pre = 0;
    q->n_tiles = 0; q->n_instances = 0;
    for (auto &g : groups) {
        const Config &gc = q->items[g.second[0]].c;
        GroupLaunch L{queue_kernel(gc), pos, (int)g.second.size(), pre, gc.waves, 0};
        int acc = 0;
        for (int i : g.second) {
            const QueueItem &it = q->items[i];
            int nt = 0;
            size_t lds = 0;
            KArgs &a = h_items[pos];
            const int rc = make_args(it.plan, it.c, it.batch, it.ybus, it.sbus, it.v0, it.tol, it.max_iter,
                                     base + ws_off[i], (size_t)ntiles[i] * tile_layout(it.plan->h, it.c).bytes,
                                     MODE_SOLVE, it.v_out, it.iters_out, it.conv_out, it.status_out, nullptr,
                                     nullptr, a, nt, lds);
            if (rc != PF_OK) { queue_release(q); return rc; }
            a.done_ticks = it.ticks_out;
            a.t0 = d_t0;
            L.lds = std::max(L.lds, lds);
            h_prefix[pre++] = acc;
            acc += nt;
            pos++;
            q->n_instances += it.batch;
        }
        h_prefix[pre++] = acc;
        q->n_tiles += acc;
        gl.push_back(L);
    }
    hipError_t e = hipMemcpy(base, h_items.data(), sizeof(KArgs) * (size_t)nitems, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(d_prefix, h_prefix.data(), sizeof(int) * h_prefix.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_error(std::string("queue upload failed: ") + hipGetErrorString(e));
        queue_release(q);
        return PF_EDEVICE;
    }

    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, q->device);
    auto fail = [&](const std::string &what, hipError_t err) {
        set_error(what + ": " + hipGetErrorString(err));
        queue_release(q);
        return PF_EDEVICE;
    };
    if ((e = hipGraphCreate(&q->graph, 0)) != hipSuccess) return fail("graph creation failed", e);
    hipGraphNode_t reset;
    {
        int ngv = ng;
        void *args[] = {&d_counter, &ngv, &d_t0};
        hipKernelNodeParams kp{};
        kp.func = reinterpret_cast<void *>(queue_reset_kernel);
        kp.gridDim = dim3(1);
        kp.blockDim = dim3(64);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        if ((e = hipGraphAddKernelNode(&reset, q->graph, nullptr, 0, &kp)) != hipSuccess)
            return fail("graph reset node failed", e);
    }
    for (int gi = 0; gi < ng; gi++) {
        const GroupLaunch &L = gl[gi];
        hipFuncAttributes fa{};
        if ((e = hipFuncGetAttributes(&fa, L.fn)) != hipSuccess) return fail("kernel attributes", e);
        if (fa.sharedSizeBytes + L.lds > 160 * 1024) {
            set_error("queue group needs " + std::to_string(fa.sharedSizeBytes + L.lds) + " B of LDS");
            queue_release(q);
            return PF_EINVAL;
        }
        if (L.lds > 64 * 1024 &&
            (e = hipFuncSetAttribute(L.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(160 * 1024 - fa.sharedSizeBytes))) != hipSuccess)
            return fail("LDS attribute", e);
        int per_cu = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, L.fn, L.waves * 64, L.lds)) != hipSuccess)
            return fail("occupancy query", e);
        if (per_cu < 1) {
            set_error("queue kernel cannot be resident with its LDS");
            queue_release(q);
            return PF_EINVAL;
        }
        const int tiles = h_prefix[L.prefix_at + L.count];
        const int grid = std::max(1, std::min(tiles, per_cu * std::max(cus, 1)));
        q->grid.push_back(grid);
        const KArgs *items_p = d_items + L.first;
        const int *prefix_p = d_prefix + L.prefix_at;
        int cnt = L.count;
        int *counter_p = d_counter + gi;
        void *args[] = {&items_p, &prefix_p, &cnt, &counter_p};
        hipKernelNodeParams kp{};
        kp.func = const_cast<void *>(L.fn);
        kp.gridDim = dim3(grid);
        kp.blockDim = dim3(L.waves * 64);
        kp.sharedMemBytes = (unsigned)L.lds;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t node;
        if ((e = hipGraphAddKernelNode(&node, q->graph, &reset, 1, &kp)) != hipSuccess)
            return fail("graph kernel node failed", e);
    }
    if ((e = hipGraphInstantiate(&q->exec, q->graph, nullptr, nullptr, 0)) != hipSuccess)
        return fail("graph instantiation failed", e);
    q->built = true;
    return PF_OK;
}

// ------------------------------------------------------------------ autotuner
// A tuned configuration belongs to a pattern (its hash), a device model (FNV-1a of the
// architecture name and the CU count, so that a saved cache applies to any device of the
// same kind), the precision, the waves asked for, the batch, max_iter and tol.
struct TuneKey {
    uint64_t hash, device;
    int precision, waves, batch, max_iter;
    double tol;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(hash, device, precision, waves, batch, max_iter, tol) <
               std::tie(o.hash, o.device, o.precision, o.waves, o.batch, o.max_iter, o.tol);
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, std::pair<pf_solve_opts, double>> g_tune_cache;

static int device_model_hash(int dev, uint64_t *out)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) { set_error("hipGetDeviceProperties failed"); return PF_EDEVICE; }
    uint64_t x = 1469598103934665603ull;
    for (const char *c = prop.gcnArchName; *c; c++) { x ^= (unsigned char)*c; x *= 1099511628211ull; }
    const int cus = prop.multiProcessorCount;
    for (int i = 0; i < 4; i++) { x ^= (unsigned char)(cus >> (8 * i)); x *= 1099511628211ull; }
    *out = x;
    return PF_OK;
}

}  // namespace pf

// ====================================================================== C ABI
using namespace pf;

extern "C" {

const char *pf_last_error(void) { return g_err.c_str(); }

int pf_analyze(int32_t n_bus, int32_t nnz_y, const int32_t *row_ptr, const int32_t *col_idx,
               const int8_t *bus_type, int32_t ordering, const int32_t *user_perm, pf_plan *out)
{
    if (!out) { set_error("null output plan pointer"); return PF_EINVAL; }
    *out = nullptr;
    Plan *pl = new (std::nothrow) Plan();
    if (!pl) { set_error("out of host memory"); return PF_ENOMEM; }
    std::string err;
    int rc;
    try {
        rc = analyze(n_bus, nnz_y, row_ptr, col_idx, bus_type, ordering, user_perm, pl->h, err);
    } catch (const std::bad_alloc &) {
        rc = PF_ENOMEM; err = "out of host memory during analysis";
    }
    if (rc != PF_OK) { set_error(err); delete pl; return rc; }
    // Upload to the current device when there is one; otherwise the plan stays host-only
    // (its host queries work) and the first solve uploads it.
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
        rc = upload(pl);
        if (rc != PF_OK) { delete pl; return rc; }
    } else {
        (void)hipGetLastError();
    }
    *out = reinterpret_cast<pf_plan>(pl);
    return PF_OK;
}

int pf_plan_info(pf_plan plan, pf_plan_info_t *o)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl || !o) { set_error("null argument"); return PF_EINVAL; }
    const HostPlan &h = pl->h;
    std::memset(o, 0, sizeof(*o));
    o->n_bus = h.n; o->n_pv = h.npv; o->n_pq = h.npq; o->n_unknowns = h.N; o->nnz_y = h.nnzy;
    int64_t nnzj = 0;
    for (int i = 0; i < h.n; i++)
        for (int p = h.yrp[i]; p < h.yrp[i + 1]; p++) {
            int k = h.yci[p];
            if (h.bus_type[i] == PF_BUS_REF || h.bus_type[k] == PF_BUS_REF) continue;
            nnzj += (1 + (h.bus_type[i] == PF_BUS_PQ)) * (1 + (h.bus_type[k] == PF_BUS_PQ));
        }
    o->nnz_j = (int32_t)nnzj;
    o->nnz_lu = h.col_ptr[h.N];
    o->n_levels = (int32_t)h.lev_ptr.size() - 1;
    o->n_bs_levels = (int32_t)h.bs_lev_ptr.size() - 1;
    o->n_panels = (int32_t)h.panel_ptr.size() - 1;
    o->slot_rows = h.slot_rows;
    o->max_col = h.max_col;
    o->n_updates = (int64_t)h.upd.size();
    o->flops_refactor = h.flops;
    // compulsory bytes per instance-iteration: mismatch 32n+8N, Jacobian 16n+b nnz_lu,
    // refactor 2b nnz_lu, substitutions b nnz_lu + 16N, update 8N+32n
    o->bytes_iter_fp64 = 4 * 8 * (int64_t)o->nnz_lu + 80 * (int64_t)h.n + 32 * (int64_t)h.N;
    o->bytes_iter_fp32 = 4 * 4 * (int64_t)o->nnz_lu + 80 * (int64_t)h.n + 32 * (int64_t)h.N;
    o->pattern_hash = pattern_hash(h);
    return PF_OK;
}

int pf_plan_levels(pf_plan plan, int32_t *cols_per_level, int64_t *madds_per_level)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl || !cols_per_level) { set_error("null argument"); return PF_EINVAL; }
    const HostPlan &h = pl->h;
    const int nlev = (int)h.lev_ptr.size() - 1;
    for (int l = 0; l < nlev; l++) cols_per_level[l] = h.lev_ptr[l + 1] - h.lev_ptr[l];
    if (madds_per_level) {
        for (int l = 0; l < nlev; l++) madds_per_level[l] = 0;
        for (int j = 0; j < h.N; j++) {
            int64_t w = 0;
            for (int u = h.upd_ptr[j]; u < h.upd_ptr[j + 1]; u++) w += h.upd[u].krel_lcnt >> 16;
            madds_per_level[h.level[j]] += w;
        }
    }
    return PF_OK;
}

int pf_plan_order(pf_plan plan, int32_t *perm)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl || !perm) { set_error("null argument"); return PF_EINVAL; }
    std::memcpy(perm, pl->h.perm.data(), sizeof(int32_t) * pl->h.perm.size());
    return PF_OK;
}

int pf_plan_lu_pattern(pf_plan plan, int32_t *col_ptr, int32_t *row_idx, int32_t *level)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl || !col_ptr || !row_idx) { set_error("null argument"); return PF_EINVAL; }
    const HostPlan &h = pl->h;
    std::memcpy(col_ptr, h.col_ptr.data(), sizeof(int32_t) * h.col_ptr.size());
    std::memcpy(row_idx, h.row_idx.data(), sizeof(int32_t) * h.row_idx.size());
    if (level) std::memcpy(level, h.level.data(), sizeof(int32_t) * h.level.size());
    return PF_OK;
}

int pf_plan_schedule(pf_plan plan, int32_t order, int32_t *first, int32_t *width, int32_t *long_rank,
                     int32_t *prev_long)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl || !first || !width || !long_rank || !prev_long) { set_error("null argument"); return PF_EINVAL; }
    if (order != 0 && order != 1) { set_error("order must be 0 or 1"); return PF_EINVAL; }
    const HostPlan &h = pl->h;
    const int np = (int)h.panel_ptr.size() - 1;
    for (int q = 0; q < np; q++) {
        const LuPanel &d = h.lu_desc[(size_t)order * np + q];
        first[q] = d.j2 & ((1 << 30) - 1);
        width[q] = 1 + ((d.j2 >> 30) & 1);
        long_rank[q] = d.lrank;
        prev_long[q] = d.lrank > 0 ? h.long_first[(size_t)order * h.n_longp + d.lrank - 1] : -1;
    }
    return PF_OK;
}

int pf_plan_ring(pf_plan plan, int32_t order, int32_t n_long, int32_t *offset, int32_t *rows, int32_t *wait_lo,
                 int32_t *wait_hi)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl || !offset || !rows || !wait_lo || !wait_hi) { set_error("null argument"); return PF_EINVAL; }
    if (order != 0 && order != 1) { set_error("order must be 0 or 1"); return PF_EINVAL; }
    if (n_long < 1 || n_long > kMaxLong) { set_error("n_long must be 1.." + std::to_string(kMaxLong)); return PF_EINVAL; }
    const HostPlan &h = pl->h;
    for (int r = 0; r < h.n_longp; r++) {
        const RingSlot &e = h.ring[(((size_t)n_long - 1) * 2 + order) * h.n_longp + r];
        const int j = h.long_first[(size_t)order * h.n_longp + r];
        const int w = *std::upper_bound(h.panel_ptr.begin(), h.panel_ptr.end(), j) - j;
        offset[r] = e.off;
        rows[r] = w * (h.col_ptr[j + 1] - h.col_ptr[j]);
        wait_lo[r] = e.blk & 0xffff;
        wait_hi[r] = e.blk >> 16;
    }
    return PF_OK;
}

size_t pf_workspace_bytes(pf_plan plan, int32_t batch, const pf_solve_opts *opts)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl || batch <= 0) return 0;
    Config c;
    std::string err;
    if (!resolve_config(pl->h, opts, c, err, batch)) { set_error(err); return 0; }
    const TileLayout L = tile_layout(pl->h, c);
    return L.bytes * (size_t)((batch + c.tile - 1) / c.tile) + order_bytes(pl->h, c, batch);
}

int pf_resolve_opts(pf_plan plan, int32_t batch, const pf_solve_opts *opts, pf_solve_opts *out)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl || !out) { set_error("null argument"); return PF_EINVAL; }
    Config c;
    std::string err;
    if (!resolve_config(pl->h, opts, c, err, batch)) { set_error(err); return PF_EINVAL; }
    std::memset(out, 0, sizeof(*out));
    out->precision = c.precision;
    out->tile = c.tile;
    out->waves = c.waves;
    out->schedule = c.schedule;
    out->long_slots = c.n_long;
    out->launch = c.launch;
    out->reorder = c.reorder;
    return PF_OK;
}

int pf_solve_batch(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched,
                   const double *sbus, const double *v0, double tol, int32_t max_iter,
                   const pf_solve_opts *opts, void *workspace, size_t workspace_bytes,
                   double *v_out, int32_t *iters_out, uint8_t *converged_out,
                   int8_t *status_out, void *stream)
{
    if (ybus_batched != 0 && ybus_batched != 1) { set_error("ybus_batched must be 0 or 1"); return PF_EINVAL; }
    return run(plan, batch, ybus, sbus, v0, tol, max_iter, opts, workspace, workspace_bytes, MODE_SOLVE,
               v_out, iters_out, converged_out, status_out, nullptr, nullptr, stream, nullptr, ybus_batched);
}

int pf_solve_batch_noalloc(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched,
                           const double *sbus, const double *v0, double tol, int32_t max_iter,
                           const pf_solve_opts *opts, double *v_out, int32_t *iters_out, uint8_t *converged_out,
                           int8_t *status_out, void *stream)
{
    if (ybus_batched != 0 && ybus_batched != 1) { set_error("ybus_batched must be 0 or 1"); return PF_EINVAL; }
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl) { set_error("null plan"); return PF_EINVAL; }
    if (batch < 0) { set_error("negative batch"); return PF_EINVAL; }
    if (batch == 0) return PF_OK;
    // the plan must already be resident: uploading it here would allocate
    if (!pl->dev_mem) { set_error("the plan is not resident on a device (pf_analyze found none)"); return PF_EINVAL; }
    // the tiles' blocks only: without the stream pool the batch is never reordered
    Config c;
    std::string err;
    if (!resolve_config(pl->h, opts, c, err, batch)) { set_error(err); return PF_EINVAL; }
    const size_t need = tile_layout(pl->h, c).bytes * (size_t)((batch + c.tile - 1) / c.tile);
    if (need > kScratchBytes) {
        set_error("pf_solve_batch_noalloc: " + std::to_string(batch) + " instances need " + std::to_string(need) +
                  " bytes of scratch, more than its fixed " + std::to_string(kScratchBytes) +
                  " bytes; use fewer instances per call or pf_solve_batch with a workspace");
        return PF_EINVAL;
    }
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != PF_OK) return rc;
    return run(plan, batch, ybus, sbus, v0, tol, max_iter, opts, ws, kScratchBytes, MODE_SOLVE, v_out, iters_out,
               converged_out, status_out, nullptr, nullptr, stream, nullptr, ybus_batched, false);
}

int pf_solve_batch_warm(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched,
                        const double *sbus, const double *v0, const double *v_fallback, double tol,
                        int32_t max_iter, const pf_solve_opts *opts, void *workspace,
                        size_t workspace_bytes, double *v_out, int32_t *iters_out, uint8_t *converged_out,
                        int8_t *status_out, void *stream)
{
    if (ybus_batched != 0 && ybus_batched != 1) { set_error("ybus_batched must be 0 or 1"); return PF_EINVAL; }
    if (!v_fallback) { set_error("null fallback start"); return PF_EINVAL; }
    return run(plan, batch, ybus, sbus, v0, tol, max_iter, opts, workspace, workspace_bytes, MODE_SOLVE,
               v_out, iters_out, converged_out, status_out, nullptr, nullptr, stream, v_fallback, ybus_batched);
}

int pf_eval_mismatch(pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                     const double *v, const pf_solve_opts *opts, void *workspace,
                     size_t workspace_bytes, double *f_out, double *normf_out, void *stream)
{
    return run(plan, batch, ybus, sbus, v, 0.0, 0, opts, workspace, workspace_bytes, MODE_MISMATCH,
               nullptr, nullptr, nullptr, nullptr, f_out, normf_out, stream);
}

int pf_eval_factor(pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                   const double *v, const pf_solve_opts *opts, void *workspace,
                   size_t workspace_bytes, double *lu_out, void *stream)
{
    return run(plan, batch, ybus, sbus, v, 0.0, 0, opts, workspace, workspace_bytes, MODE_FACTOR,
               nullptr, nullptr, nullptr, nullptr, lu_out, nullptr, stream);
}

int pf_eval_step(pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                 const double *v, const pf_solve_opts *opts, void *workspace,
                 size_t workspace_bytes, double *dx_out, void *stream)
{
    return run(plan, batch, ybus, sbus, v, 0.0, 0, opts, workspace, workspace_bytes, MODE_STEP,
               nullptr, nullptr, nullptr, nullptr, dx_out, nullptr, stream);
}

int pf_queue_create(pf_queue *out)
{
    if (!out) { set_error("null output queue pointer"); return PF_EINVAL; }
    *out = nullptr;
    Queue *q = new (std::nothrow) Queue();
    if (!q) { set_error("out of host memory"); return PF_ENOMEM; }
    if (hipGetDevice(&q->device) != hipSuccess) {
        (void)hipGetLastError();
        delete q;
        set_error("no current device");
        return PF_EDEVICE;
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, q->device) != hipSuccess) {
        (void)hipGetLastError();
        khz = 0;
    }
    q->clock_hz = 1e3 * khz;
    *out = reinterpret_cast<pf_queue>(q);
    return PF_OK;
}

int pf_queue_add(pf_queue queue, pf_plan plan, int32_t batch, const double *ybus, const double *sbus,
                 const double *v0, double tol, int32_t max_iter, const pf_solve_opts *opts, double *v_out,
                 int32_t *iters_out, uint8_t *converged_out, int8_t *status_out, uint64_t *done_ticks_out)
{
    Queue *q = reinterpret_cast<Queue *>(queue);
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!q || !pl) { set_error("null queue or plan"); return PF_EINVAL; }
    if (batch < 0) { set_error("negative batch"); return PF_EINVAL; }
    if (max_iter < 0 || !(tol >= 0.0)) { set_error("invalid tol or max_iter"); return PF_EINVAL; }
    if (batch == 0) return PF_OK;     // nothing to solve: the item is not kept
    if (!ybus || !sbus || !v0 || !v_out || !iters_out || !converged_out) { set_error("null pointer"); return PF_EINVAL; }
    if (pl->dev_mem && pl->device != q->device) { set_error("plan and queue are on different devices"); return PF_EDEVICE; }
    Config c;
    std::string err;
    if (!resolve_config(pl->h, opts, c, err, batch)) { set_error(err); return PF_EINVAL; }
    if (lds_bytes(pl->h, c) > kLdsLimit) { set_error("configuration does not fit in LDS"); return PF_EINVAL; }
    QueueItem it{pl, c, batch, ybus, sbus, v0, tol, max_iter, v_out, iters_out, converged_out, status_out,
                 reinterpret_cast<unsigned long long *>(done_ticks_out)};
    try {
        q->items.push_back(it);
    } catch (const std::bad_alloc &) {
        set_error("out of host memory");
        return PF_ENOMEM;
    }
    q->built = false;
    return PF_OK;
}

int pf_queue_run(pf_queue queue, void *stream)
{
    Queue *q = reinterpret_cast<Queue *>(queue);
    if (!q) { set_error("null queue"); return PF_EINVAL; }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != q->device) {
        set_error("the current device differs from the queue's device");
        return PF_EDEVICE;
    }
    if (q->items.empty()) return PF_OK;
    if (!q->built) {
        const int rc = queue_build(q);
        if (rc != PF_OK) return rc;
    }
    if (q->n_tiles == 0) return PF_OK;
    const hipError_t e = hipGraphLaunch(q->exec, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) { set_error(std::string("graph launch failed: ") + hipGetErrorString(e)); return PF_EDEVICE; }
    return PF_OK;
}

int pf_queue_info(pf_queue queue, pf_queue_info_t *o)
{
    Queue *q = reinterpret_cast<Queue *>(queue);
    if (!q || !o) { set_error("null argument"); return PF_EINVAL; }
    std::memset(o, 0, sizeof(*o));
    o->n_items = (int32_t)q->items.size();
    o->built = q->built ? 1 : 0;
    o->n_groups = (int32_t)q->grid.size();
    for (int i = 0; i < (int)q->grid.size() && i < 18; i++) o->grid[i] = q->grid[i];
    o->n_tiles = q->n_tiles;
    o->n_instances = q->n_instances;
    o->workspace_bytes = q->ws_bytes;
    o->wall_clock_hz = q->clock_hz;
    return PF_OK;
}

void pf_queue_destroy(pf_queue queue)
{
    Queue *q = reinterpret_cast<Queue *>(queue);
    if (!q) return;
    queue_release(q);
    delete q;
}

int pf_tune(pf_plan plan, int32_t batch, const double *ybus, const double *sbus, const double *v0, double tol,
            int32_t max_iter, int32_t precision, int32_t waves, int32_t reps, int32_t flags,
            pf_solve_opts *best_out, double *best_ms_out, void *stream)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl || !best_out) { set_error("null plan or output"); return PF_EINVAL; }
    if (batch <= 0 || reps <= 0) { set_error("batch and reps must be positive"); return PF_EINVAL; }
    if (!ybus || !sbus || !v0) { set_error("null input pointer"); return PF_EINVAL; }
    if (precision != PF_FP64 && precision != PF_FP32_LU) { set_error("unknown precision"); return PF_EINVAL; }
    if (waves != 0 && waves != 2 && waves != 4 && waves != 8 && waves != 16) {
        set_error("waves must be 0, 2, 4, 8 or 16");
        return PF_EINVAL;
    }
    if (max_iter < 0 || !(tol >= 0.0)) { set_error("invalid tol or max_iter"); return PF_EINVAL; }
    if (!pl->dev_mem) {
        const int rcu = upload(pl);
        if (rcu != PF_OK) return rcu;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != pl->device) {
        set_error("the current device differs from the plan's device");
        return PF_EDEVICE;
    }
    uint64_t model = 0;
    const int rcm = device_model_hash(dev, &model);
    if (rcm != PF_OK) return rcm;
    const TuneKey key{pattern_hash(pl->h), model, precision, waves, batch, max_iter, tol};
    if (!(flags & PF_TUNE_FORCE)) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto f = g_tune_cache.find(key);
        if (f != g_tune_cache.end()) {
            *best_out = f->second.first;
            if (best_ms_out) *best_ms_out = f->second.second;
            return PF_OK;
        }
    }
    // candidate configurations that fit in LDS
    std::vector<pf_solve_opts> cand;
    const int tiles64[] = {4, 8, 16}, tiles32[] = {8, 16, 32}, wv[] = {2, 4, 8, 16};
    for (int ti = 0; ti < 3; ti++)
        for (int w : wv) {
            if (waves && w != waves) continue;
            for (int sc = 0; sc < 2; sc++) {
                // long-slot counts: the automatic choice for this batch, and 2, 4, 8 (each
                // resolved count once)
                std::vector<int> seen;
                for (const int ls : {0, 2, 4, 8}) {
                    pf_solve_opts o{};
                    o.precision = precision;
                    o.tile = precision == PF_FP64 ? tiles64[ti] : tiles32[ti];
                    o.waves = w;
                    o.schedule = sc;
                    o.long_slots = ls;
                    o.launch = PF_LAUNCH_FUSED;      // the form the queue runs
                    Config c;
                    std::string err;
                    if (!resolve_config(pl->h, &o, c, err, batch) || lds_bytes(pl->h, c) > kLdsLimit) continue;
                    if (std::find(seen.begin(), seen.end(), c.n_long) != seen.end()) continue;
                    seen.push_back(c.n_long);
                    o.long_slots = c.n_long;
                    cand.push_back(o);
                }
            }
        }
    if (cand.empty()) { set_error("no configuration fits in LDS"); return PF_EINVAL; }
    size_t ws = 0;
    for (auto &o : cand) ws = std::max(ws, pf_workspace_bytes(plan, batch, &o));
    const size_t n = (size_t)pl->h.n;
    const size_t out_bytes = align256(sizeof(double) * 2 * n * batch) + align256(sizeof(int32_t) * batch) +
                             align256((size_t)batch) + align256((size_t)batch);
    void *mem = nullptr;
    if (hipMalloc(&mem, ws + out_bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("out of device memory for tuning");
        return PF_ENOMEM;
    }
    char *m = static_cast<char *>(mem);
    double *v_out = reinterpret_cast<double *>(m + ws);
    int32_t *it_out = reinterpret_cast<int32_t *>(m + ws + align256(sizeof(double) * 2 * n * batch));
    uint8_t *cv_out = reinterpret_cast<uint8_t *>(it_out) + align256(sizeof(int32_t) * batch);
    int8_t *st_out = reinterpret_cast<int8_t *>(cv_out + align256((size_t)batch));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PF_OK;
    // candidates are scored by converged flows per millisecond; one that converges fewer
    // instances than the default configuration, or reports an internal error, is rejected
    std::vector<int8_t> h_st((size_t)batch);
    auto outcome = [&](int &nconv, int &nint) -> int {
        if (hipMemcpyAsync(h_st.data(), st_out, (size_t)batch, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error("tuning run failed");
            return PF_EDEVICE;
        }
        nconv = 0; nint = 0;
        for (const int8_t x : h_st) { nconv += x == PF_ST_CONVERGED; nint += x == PF_ST_INTERNAL; }
        return PF_OK;
    };
    int ref_conv = -1;
    {
        pf_solve_opts d{};
        d.precision = precision;
        d.waves = waves;
        rc = pf_solve_batch(plan, batch, ybus, 0, sbus, v0, tol, max_iter, &d, m, ws, v_out, it_out, cv_out, st_out,
                            stream);
        int ni = 0;
        if (rc == PF_OK) rc = outcome(ref_conv, ni);
    }
    double best = -1.0, best_ms = 0.0;
    pf_solve_opts best_o = cand[0];
    if (rc == PF_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
        set_error("event creation failed");
        rc = PF_EDEVICE;
    }
    for (size_t ci = 0; rc == PF_OK && ci < cand.size(); ci++) {
        const pf_solve_opts &o = cand[ci];
        rc = pf_solve_batch(plan, batch, ybus, 0, sbus, v0, tol, max_iter, &o, m, ws, v_out, it_out, cv_out, st_out,
                            stream);
        if (rc != PF_OK) break;
        int nconv = 0, nint = 0;
        if ((rc = outcome(nconv, nint)) != PF_OK) break;
        if (nint > 0 || nconv < ref_conv) continue;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && rc == PF_OK; r++)
            rc = pf_solve_batch(plan, batch, ybus, 0, sbus, v0, tol, max_iter, &o, m, ws, v_out, it_out, cv_out,
                                st_out, stream);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) { set_error("tuning run failed"); rc = PF_EDEVICE; break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double per = ms / reps;
        const double score = per > 0.0 ? nconv / per : 0.0;
        if (score > best) { best = score; best_ms = per; best_o = o; }
    }
    if (rc == PF_OK && best < 0.0) {
        set_error("no candidate configuration matched the default configuration's converged count");
        rc = PF_EINVAL;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(mem);
    if (rc != PF_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = {best_o, best_ms};
    }
    *best_out = best_o;
    if (best_ms_out) *best_ms_out = best_ms;
    return PF_OK;
}

// One line per entry after a header line: the key (pattern hash and device model in hex,
// precision, waves, batch, max_iter, tol as a C99 hex float), then the configuration
// (precision, tile, waves, schedule, long_slots, launch, reorder) and the tuned ms per solve.
static const char *kTuneHeader = "pf_tune_cache 1";

int pf_tune_cache_save(const char *path)
{
    if (!path) { set_error("null path"); return PF_EINVAL; }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) { set_error(std::string("cannot open ") + path + " for writing"); return PF_EINVAL; }
    bool ok = std::fprintf(f, "%s\n", kTuneHeader) > 0;
    for (const auto &kv : g_tune_cache) {
        const TuneKey &k = kv.first;
        const pf_solve_opts &o = kv.second.first;
        ok = ok && std::fprintf(f, "%016llx %016llx %d %d %d %d %a %d %d %d %d %d %d %d %a\n", (unsigned long long)k.hash,
                                (unsigned long long)k.device, k.precision, k.waves, k.batch, k.max_iter, k.tol,
                                o.precision, o.tile, o.waves, o.schedule, o.long_slots, o.launch, o.reorder,
                                kv.second.second) > 0;
    }
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) { set_error(std::string("writing ") + path + " failed"); return PF_EINVAL; }
    return PF_OK;
}

int pf_tune_cache_load(const char *path)
{
    if (!path) { set_error("null path"); return PF_EINVAL; }
    FILE *f = std::fopen(path, "r");
    if (!f) { set_error(std::string("cannot open ") + path); return PF_EINVAL; }
    char line[512];
    std::vector<std::pair<TuneKey, std::pair<pf_solve_opts, double>>> got;
    bool ok = std::fgets(line, sizeof line, f) && std::strncmp(line, kTuneHeader, std::strlen(kTuneHeader)) == 0;
    int lineno = 1;
    while (ok && std::fgets(line, sizeof line, f)) {
        lineno++;
        if (line[0] == '\n' || line[0] == 0) continue;
        unsigned long long h = 0, d = 0;
        TuneKey k{};
        pf_solve_opts o{};
        double ms = 0.0;
        const int n = std::sscanf(line, "%llx %llx %d %d %d %d %la %d %d %d %d %d %d %d %la", &h, &d, &k.precision,
                                  &k.waves, &k.batch, &k.max_iter, &k.tol, &o.precision, &o.tile, &o.waves,
                                  &o.schedule, &o.long_slots, &o.launch, &o.reorder, &ms);
        k.hash = h;
        k.device = d;
        ok = n == 15;
        if (ok) got.push_back({k, {o, ms}});
    }
    std::fclose(f);
    if (!ok) {
        set_error(std::string(path) + ": not a pf_tune cache (line " + std::to_string(lineno) + ")");
        return PF_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : got) g_tune_cache[kv.first] = kv.second;
    return PF_OK;
}

int pf_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
    return PF_OK;
}

int32_t pf_tune_cache_size(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return (int32_t)g_tune_cache.size();
}

int pf_cpu_solve_batch(pf_plan plan, int32_t batch, const double *ybus, const double *sbus, const double *v0,
                       double tol, int32_t max_iter, int32_t threads, double *v_out, int32_t *iters_out,
                       uint8_t *converged_out, int8_t *status_out)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl) { set_error("null plan"); return PF_EINVAL; }
    if (batch < 0 || threads < 0) { set_error("negative batch or thread count"); return PF_EINVAL; }
    if (batch == 0) return PF_OK;
    if (!ybus || !sbus || !v0 || !v_out || !iters_out || !converged_out) { set_error("null pointer"); return PF_EINVAL; }
    if (max_iter < 0 || !(tol >= 0.0)) { set_error("invalid tol or max_iter"); return PF_EINVAL; }
    std::string err;
    const int rc = cpu_solve(pl->h, batch, ybus, sbus, v0, tol, max_iter, threads, v_out, iters_out, converged_out,
                             status_out, err);
    if (rc != PF_OK) set_error(err);
    return rc;
}

void pf_plan_destroy(pf_plan plan)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl) return;
    if (pl->dev_mem) (void)hipFree(pl->dev_mem);
    delete pl;
}

}  // extern "C"
