// Batched Newton-Raphson power flow on gfx950: one fused, persistent-per-tile kernel.
//
// A workgroup owns a tile of T instances and runs their whole Newton loop (Sec. 3 of
// the paper) without leaving the kernel:
//   M   mismatch S = V o conj(Y V) (Eq. 1), F = calculated - specified (Alg. 1), the
//       per-instance infinity norm by wavefront shuffles and an LDS reduction, and the
//       convergence / divergence decision;
//   LU  a sync-free dataflow form of the left-looking refactorization (Sec. 4.2-4.3):
//       each wavefront takes the next column j of A = P J P^T from a counter, builds its
//       Jacobian entries straight from V and Ybus into an LDS working column (Sec. 3.1.2,
//       "direct into permuted form A"), applies the update of every column k with
//       U(k,j) != 0 in ascending k (the sparse VMAD with direct indexing of Alg. 3) as
//       soon as k is published, carries the forward substitution of the right-hand side
//       along (row j of L is read in the same pass), normalises the L part, writes the
//       column back and publishes it.  This generalises the paper's stage 2 (partial
//       updates of unfinished columns) to every column: no level barriers remain, and
//       the serial tail of the factorization pipelines across wavefronts;
//   BS  backward substitution in the same dataflow style (row j waits for the rows
//       i > j it reads), one wavefront per row, and the voltage update V <- V - dx for
//       instances still iterating.
// Each entry of every per-instance array is stored tile-interleaved: element e of
// instance t of a tile lives at [e][t], so a wavefront reading entry e for the tile's
// instances issues one contiguous T * sizeof(real) access (the paper's batched layout,
// Sec. 3.1, Fig. "CRS sparse matrix ... batched data" d).  Inside a wavefront the
// 64 lanes are T instances x (64 / T) sub-lanes that split the rows of a column
// update (the paper's extra VMAD parallelism).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "pf_internal.h"

namespace pf {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

enum Mode { MODE_SOLVE = 0, MODE_MISMATCH = 1, MODE_FACTOR = 2, MODE_STEP = 3 };

struct KArgs {
    DevPlan p;
    const int32_t *perm;        // position -> unknown (device)
    const double *ybus;         // [nnzy][2]
    const double *sbus;         // [B][n][2]
    const double *v0;           // [B][n][2]
    double tol;
    int max_iter, batch, mode;
    char *ws;
    size_t tile_bytes, off_y, off_vec;   // byte offsets inside one tile's block
    double *v_out;
    int32_t *iters_out;
    uint8_t *conv_out;
    int8_t *status_out;
    double *aux_out;            // F, LU or dx for the single-step modes
    double *aux2_out;           // max |F| for MODE_MISMATCH
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One Jacobian entry dF_e/dx_u from its descriptor (Sec. 3.1.2).  With w = V_i conj(Y_ik V_k):
//   off-diagonal  dS_i/dangle_k = -j w,          dS_i/d|V_k| = w / |V_k|
//   diagonal      dS_i/dangle_i = j (S_i - |V_i|^2 conj Y_ii),
//                 dS_i/d|V_i|   = S_i / |V_i| + |V_i| conj Y_ii
// P equations take the real part, Q equations the imaginary part.
// The column's own bus k supplies V_k, |V_k| and I_k (loaded once per panel); each
// off-diagonal entry loads only V_i and Y_ik.  The angle and |V| columns of a PQ bus share
// the entry's Ybus element and row, so one call yields both derivatives:
//   angle:  off-diagonal -j w, diagonal j (S_k - |V_k|^2 conj Y_kk)
//   |V|:    off-diagonal w / |V_k|, diagonal S_k / |V_k| + |V_k| conj Y_kk
// with w = V_i conj(Y_ik V_k); P rows take the real part, Q rows the imaginary part.
struct JacPair {
    double th, vm;
};

__device__ __forceinline__ JacPair jac_entry(const JacDesc d, const double *ybus, const double2 *Vc_t,
                                             double2 vk, double vmk, double2 ik)
{
    if (d.p < 0) return JacPair{0.0, 0.0};
    const double2 y = reinterpret_cast<const double2 *>(ybus)[d.p];
    double tr, ti, vr, vi;     // d/d angle and d/d|V| of S_i, complex
    if (d.i != d.k) {
        const double2 v = Vc_t[0];
        const double cr = y.x * vk.x - y.y * vk.y, ci = y.x * vk.y + y.y * vk.x;     // Y_ik V_k
        const double wr = v.x * cr + v.y * ci, wi = v.y * cr - v.x * ci;              // V_i conj(.)
        tr = wi; ti = -wr;
        const double inv = 1.0 / vmk;
        vr = wr * inv; vi = wi * inv;
    } else {
        const double sr = vk.x * ik.x + vk.y * ik.y, si = vk.y * ik.x - vk.x * ik.y;  // S_k
        const double m2 = vmk * vmk;
        tr = -si - m2 * y.y; ti = sr - m2 * y.x;
        vr = sr / vmk + vmk * y.x; vi = si / vmk - vmk * y.y;
    }
    const bool q = d.kind & 2;
    return JacPair{q ? ti : tr, q ? vi : vr};
}

// Publication flags of the dataflow phases: one LDS byte per column (row).  A producer
// makes its global writes visible to the workgroup (release fence) and then every lane of
// the wavefront stores the same flag byte (plain stores, no atomics, so the loops stay free
// of lane-divergent regions).  A consumer polls the byte uniformly across the wavefront
// and acquires.  Every wait is bounded: a wait that exceeds the limit raises the tile's
// error flag and stops waiting, so a wrong schedule can only produce wrong numbers and an
// error status, never a hang.
__device__ __forceinline__ void wait_published(unsigned char *flags, int j, int *err)
{
    for (unsigned spins = 0;; ++spins) {
        const int f = __builtin_amdgcn_readfirstlane(
            (int)__hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (f) break;
        const int e = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (e) break;
        if (spins >= (1u << 22)) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <typename R, int T, int NW>
__global__ __launch_bounds__(NW * 64) void nr_tile_kernel(KArgs a)
{
    constexpr int SL = 64 / T;          // sub-lanes per instance inside a wavefront
    constexpr int NT = NW * 64;
    constexpr int SLOTS = NT / T;       // bus slots per workgroup

    extern __shared__ char smem_raw[];
    __shared__ double s_red[NW][T];
    __shared__ int s_bad[NW][T];
    __shared__ int s_active[T], s_status[T], s_iters[T], s_piv[T];
    __shared__ double s_normf[T];
    __shared__ int s_any, s_err;

    const DevPlan &P = a.p;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int t = lane % T;
    const int s = lane / T;
    const int slot = tid / T;
    const int tile = blockIdx.x;
    const int b = tile * T + t;
    const bool valid = b < a.batch;
    const int n = P.n;
    const int N = P.N;

    char *base = a.ws + (size_t)tile * a.tile_bytes;
    R *LU = reinterpret_cast<R *>(base);
    R *Yv = reinterpret_cast<R *>(base + a.off_y);
    double *vec = reinterpret_cast<double *>(base + a.off_vec);
    const size_t nT = (size_t)n * T;
    double *Vm = vec, *Va = vec + nT, *Ps = vec + 2 * nT, *Qs = vec + 3 * nT;
    double2 *Vc = reinterpret_cast<double2 *>(vec + 4 * nT);     // V = |V| e^{j angle}
    double2 *Ic = reinterpret_cast<double2 *>(vec + 6 * nT);     // I = Y V

    // per wavefront: two working columns (a panel) and two right-hand-side slots
    R *xw = reinterpret_cast<R *>(smem_raw) + (size_t)wave * 2 * (P.max_col * T + T);
    R *xw1 = xw + (size_t)P.max_col * T;
    R *ysl = xw1 + (size_t)P.max_col * T;
    R *ysl1 = ysl + T;
    unsigned char *done = reinterpret_cast<unsigned char *>(
        reinterpret_cast<R *>(smem_raw) + (size_t)NW * 2 * (P.max_col * T + T));
    int *err = &s_err;

    // ---- boundary layout [B][n][2] -> tile layout [n][T]
    for (int i = slot; i < n; i += SLOTS) {
        double vm = 1.0, va = 0.0, ps = 0.0, qs = 0.0;
        if (valid) {
            const size_t o = ((size_t)b * n + i) * 2;
            vm = a.v0[o]; va = a.v0[o + 1];
            ps = a.sbus[o]; qs = a.sbus[o + 1];
        }
        Vm[i * T + t] = vm; Va[i * T + t] = va;
        Ps[i * T + t] = ps; Qs[i * T + t] = qs;
    }
    if (tid < T) {
        s_active[t] = valid ? 1 : 0;
        s_status[t] = PF_ST_MAXITER;
        s_iters[t] = 0;
    }
    if (tid == 0) s_err = 0;
    __syncthreads();

    for (int it = 0;; ++it) {
        // ============================ M: mismatch and convergence test
        for (int i = slot; i < n; i += SLOTS) {
            double sn, cs;
            const double vm = Vm[i * T + t];
            sincos(Va[i * T + t], &sn, &cs);
            Vc[i * T + t] = make_double2(vm * cs, vm * sn);
        }
        __syncthreads();
        double mx = 0.0;
        int bad = 0;
        for (int i = slot; i < n; i += SLOTS) {
            double ir = 0.0, ii = 0.0;
            for (int q = P.yrp[i]; q < P.yrp[i + 1]; q++) {
                const double2 y = reinterpret_cast<const double2 *>(a.ybus)[q];
                const double2 v = Vc[P.yci[q] * T + t];
                ir += y.x * v.x - y.y * v.y;
                ii += y.x * v.y + y.y * v.x;
            }
            Ic[i * T + t] = make_double2(ir, ii);
            const double2 vv = Vc[i * T + t];
            const double vr = vv.x, vi = vv.y;
            const int pe = P.bus_peq[i], qe = P.bus_qeq[i];
            if (pe >= 0) {
                const double f = (vr * ir + vi * ii) - Ps[i * T + t];
                Yv[pe * T + t] = (R)f;
                if (!isfinite(f)) bad = 1; else mx = fmax(mx, fabs(f));
                if (a.mode == MODE_MISMATCH && valid) a.aux_out[(size_t)b * N + a.perm[pe]] = f;
            }
            if (qe >= 0) {
                const double f = (vi * ir - vr * ii) - Qs[i * T + t];
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
                if (nb) { s_status[t] = PF_ST_NONFINITE; s_active[t] = 0; s_iters[t] = it; }
                else if (nf < a.tol) { s_status[t] = PF_ST_CONVERGED; s_active[t] = 0; s_iters[t] = it; }
                else if (it >= a.max_iter) { s_status[t] = PF_ST_MAXITER; s_active[t] = 0; s_iters[t] = it; }
            }
        }
        __syncthreads();
        if (tid == 0) {
            int any = 0;
            for (int q = 0; q < T; q++) any |= s_active[q];
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

        // ============================ LU: Jacobian -> refactorization -> forward substitution
        for (int w = tid; w < N; w += NT)
            __hip_atomic_store(&done[w], (unsigned char)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
        // Panels (one column, or the angle/|V| pair of a PQ bus sharing one row list) in
        // elimination order, round-robin over the wavefronts: the smallest unfinished panel
        // always has every source published, so some wavefront always makes progress.
        for (int pi = wave; pi < P.n_panels; pi += NW) {
            const int j = P.panel_ptr[pi];
            const bool two = P.panel_ptr[pi + 1] - j == 2;
            const int cs = P.col_ptr[j];
            const int cnt = P.col_ptr[j + 1] - cs;
            const int dr = P.col_diag[j];
            {
                const int kb = P.pos_upd[j] >> 1;      // bus of the panel's unknowns
                const double2 vk = Vc[kb * T + t], ik = Ic[kb * T + t];
                const double vmk = Vm[kb * T + t];
                for (int e = s; e < cnt; e += SL) {
                    const JacDesc d0 = P.desc[cs + e];
                    const JacPair jp = jac_entry(d0, a.ybus, Vc + d0.i * T + t, vk, vmk, ik);
                    xw[e * T + t] = (R)((d0.kind & 1) ? jp.vm : jp.th);
                    if (two) xw1[e * T + t] = (R)jp.vm;
                }
            }
            if (s == 0) {
                ysl[t] = Yv[j * T + t];
                if (two) ysl1[t] = Yv[(j + 1) * T + t];
            }
            const int u0 = P.upd_ptr[j], u1 = P.upd_ptr[j + 1];
            Update upn{};
            if (u0 < u1) upn = P.upd[u0];
            for (int u = u0; u < u1; u++) {
                const Update up = upn;
                if (u + 1 < u1) upn = P.upd[u + 1];     // next descriptor in flight meanwhile
                const int krel = up.krel_lcnt & 0xffff, lcnt = up.krel_lcnt >> 16;
                wait_published(done, up.k, err);
                wave_sync();
                const R m0 = xw[krel * T + t];
                const R m1 = two ? xw1[krel * T + t] : (R)0;
                for (int r = s; r < lcnt; r += SL) {
                    const R l = LU[(size_t)(up.lbeg + r) * T + t];
                    const int tr = P.rel[up.roff + r];
                    xw[tr * T + t] = fma(-m0, l, xw[tr * T + t]);
                    if (two) xw1[tr * T + t] = fma(-m1, l, xw1[tr * T + t]);
                    if (tr == dr) ysl[t] = fma(-l, Yv[up.k * T + t], ysl[t]);
                    else if (two && tr == dr + 1) ysl1[t] = fma(-l, Yv[up.k * T + t], ysl1[t]);
                }
            }
            wave_sync();
            const R d = xw[dr * T + t];
            if (s == 0 && valid && !(fabs((double)d) > 1e-300 && isfinite((double)d))) s_piv[t] = 1;
            for (int e = dr + 1 + s; e < cnt; e += SL) xw[e * T + t] = xw[e * T + t] / d;
            wave_sync();
            if (two) {
                // the pair's second column receives the update of the first (its last source)
                const R m = xw1[dr * T + t];
                for (int e = dr + 1 + s; e < cnt; e += SL) xw1[e * T + t] = fma(-m, xw[e * T + t], xw1[e * T + t]);
                wave_sync();
                if (s == 0) ysl1[t] = fma(-xw[(dr + 1) * T + t], ysl[t], ysl1[t]);
                const R d1 = xw1[(dr + 1) * T + t];
                if (s == 0 && valid && !(fabs((double)d1) > 1e-300 && isfinite((double)d1))) s_piv[t] = 1;
                for (int e = dr + 2 + s; e < cnt; e += SL) xw1[e * T + t] = xw1[e * T + t] / d1;
                wave_sync();
            }
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
        }
        __syncthreads();
        if (tid < T && s_piv[t] && s_active[t] && a.mode == MODE_SOLVE) {
            s_status[t] = PF_ST_PIVOT; s_active[t] = 0; s_iters[t] = it;
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
        // Panels in reverse elimination order.  For a pair (j, j+1) the rows share their
        // column set i > j+1, and U(j, i), U(j+1, i) sit next to each other in column i.
        const bool upd_v = (a.mode == MODE_SOLVE);
        for (int pi = P.n_panels - 1 - wave; pi >= 0; pi -= NW) {
            const int j = P.panel_ptr[pi];
            const bool two = P.panel_ptr[pi + 1] - j == 2;
            const int jl = two ? j + 1 : j;            // the panel's last row
            R acc0 = 0, acc1 = 0;
            const int q0 = P.bs_ptr[jl], q1 = P.bs_ptr[jl + 1];
            for (int q = q0; q < q1; q++) wait_published(done, P.bs_col[q], err);
            for (int q = q0 + s; q < q1; q += SL) {
                const R z = Yv[P.bs_col[q] * T + t];
                const size_t pq = (size_t)P.bs_pos[q];
                if (two) {
                    acc1 = fma(LU[pq * T + t], z, acc1);
                    acc0 = fma(LU[(pq - 1) * T + t], z, acc0);
                } else {
                    acc0 = fma(LU[pq * T + t], z, acc0);
                }
            }
#pragma unroll
            for (int off = T; off < 64; off <<= 1) {
                acc0 += __shfl_xor(acc0, off);
                acc1 += __shfl_xor(acc1, off);
            }
            if (s == 0) {
                const int cs = P.col_ptr[j], dr = P.col_diag[j];
                R zl = 0;
                if (two) {
                    const int cs1 = P.col_ptr[j + 1];
                    zl = (Yv[(j + 1) * T + t] - acc1) / LU[(size_t)(cs1 + dr + 1) * T + t];
                    Yv[(j + 1) * T + t] = zl;
                    acc0 = fma(LU[(size_t)(cs1 + dr) * T + t], zl, acc0);
                }
                const R z0 = (Yv[j * T + t] - acc0) / LU[(size_t)(cs + dr) * T + t];
                Yv[j * T + t] = z0;
                if (upd_v && s_active[t]) {
                    const int pu = P.pos_upd[j];
                    const int bus = pu >> 1;
                    if (pu & 1) Vm[bus * T + t] -= (double)z0;
                    else Va[bus * T + t] -= (double)z0;
                    if (two) Vm[bus * T + t] -= (double)zl;
                }
            }
            wave_sync();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __hip_atomic_store(&done[j], (unsigned char)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (two) __hip_atomic_store(&done[j + 1], (unsigned char)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        if (a.mode == MODE_STEP) {
            if (valid)
                for (int j = slot; j < N; j += SLOTS) a.aux_out[(size_t)b * N + a.perm[j]] = (double)Yv[j * T + t];
            return;
        }
    }

    // ---- tile layout -> boundary layout
    if (valid) {
        for (int i = slot; i < n; i += SLOTS) {
            const size_t o = ((size_t)b * n + i) * 2;
            a.v_out[o] = Vm[i * T + t];
            a.v_out[o + 1] = Va[i * T + t];
        }
        if (s == 0 && wave == 0) {
            const int st = s_err ? PF_ST_INTERNAL : s_status[t];
            a.iters_out[b] = s_iters[t];
            a.conv_out[b] = st == PF_ST_CONVERGED ? 1 : 0;
            if (a.status_out) a.status_out[b] = (int8_t)st;
        }
    }
}

// ------------------------------------------------------------------ launch configuration
struct Config {
    int precision, tile, waves;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct TileLayout {
    size_t off_y, off_vec, bytes;
};

static TileLayout tile_layout(const HostPlan &h, const Config &c)
{
    const size_t rs = c.precision == PF_FP32_LU ? 4 : 8;
    TileLayout L;
    L.off_y = align256((size_t)(h.col_ptr.empty() ? 0 : h.col_ptr[h.N]) * c.tile * rs);
    L.off_vec = L.off_y + align256((size_t)h.N * c.tile * rs);
    L.bytes = L.off_vec + align256((size_t)8 * h.n * c.tile * 8);
    return L;
}

static size_t lds_bytes(const HostPlan &h, const Config &c)
{
    const size_t rs = c.precision == PF_FP32_LU ? 4 : 8;
    return (size_t)c.waves * 2 * ((size_t)h.max_col * c.tile + c.tile) * rs + (size_t)h.N;
}

static size_t lds_bytes(const HostPlan &h, const Config &c);
static constexpr size_t kLdsLimit = 160 * 1024 - 8192;

// Explicit tile/waves are validated; zeros pick the first candidate whose working columns
// fit in LDS (larger tiles first: wider coalesced rows and fewer workgroups).
static bool resolve_config(const HostPlan &h, const pf_solve_opts *o, Config &c, std::string &err)
{
    c.precision = o ? o->precision : PF_FP64;
    const int tile = o ? o->tile : 0, waves = o ? o->waves : 0;
    if (c.precision != PF_FP64 && c.precision != PF_FP32_LU) { err = "unknown precision"; return false; }
    const bool fp64 = c.precision == PF_FP64;
    if (tile != 0 && !(fp64 ? (tile == 4 || tile == 8 || tile == 16) : (tile == 8 || tile == 16 || tile == 32))) {
        err = "unsupported tile size for this precision"; return false;
    }
    if (waves != 0 && waves != 2 && waves != 4 && waves != 8 && waves != 16) {
        err = "waves must be 2, 4, 8 or 16"; return false;
    }
    static const int cand64[][2] = {{8, 4}, {4, 8}, {8, 2}, {4, 4}, {4, 2}};
    static const int cand32[][2] = {{16, 4}, {8, 8}, {16, 2}, {8, 4}, {8, 2}};
    for (const auto &cw : (fp64 ? cand64 : cand32)) {
        c.tile = tile ? tile : cw[0];
        c.waves = waves ? waves : cw[1];
        if (lds_bytes(h, c) <= kLdsLimit) return true;
    }
    err = "the longest LU column (" + std::to_string(h.max_col) + " entries) does not fit in LDS for any "
          "supported tile/wave configuration";
    return false;
}

template <typename R, int T, int NW>
static hipError_t launch_t(const KArgs &a, int grid, size_t lds, hipStream_t st)
{
    auto fn = nr_tile_kernel<R, T, NW>;
    if (lds > 64 * 1024) {
        static std::once_flag once;
        static hipError_t attr_err = hipSuccess;
        std::call_once(once, [&] {
            attr_err = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 8192);
        });
        if (attr_err != hipSuccess) return attr_err;
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NW * 64), lds, st, a);
    return hipGetLastError();
}

#define PF_DISPATCH_NW(R, T)                                                   \
    switch (c.waves) {                                                         \
    case 2: return launch_t<R, T, 2>(a, grid, lds, st);                        \
    case 4: return launch_t<R, T, 4>(a, grid, lds, st);                        \
    case 8: return launch_t<R, T, 8>(a, grid, lds, st);                        \
    default: return launch_t<R, T, 16>(a, grid, lds, st);                      \
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

static int upload(Plan *pl);

static int run(pf_plan plan_h, int32_t batch, const double *ybus, const double *sbus, const double *v0,
               double tol, int32_t max_iter, const pf_solve_opts *opts, void *workspace,
               size_t workspace_bytes, int mode, double *v_out, int32_t *iters_out, uint8_t *conv_out,
               int8_t *status_out, double *aux, double *aux2, void *stream)
{
    Plan *pl = reinterpret_cast<Plan *>(plan_h);
    if (!pl) { set_error("null plan"); return PF_EINVAL; }
    if (batch < 0) { set_error("negative batch"); return PF_EINVAL; }
    if (batch == 0) return PF_OK;
    const HostPlan &h = pl->h;
    Config c;
    std::string err;
    if (!resolve_config(h, opts, c, err)) { set_error(err); return PF_EINVAL; }
    if (!ybus || !sbus || !v0) { set_error("null input pointer"); return PF_EINVAL; }
    if (mode == MODE_SOLVE && (!v_out || !iters_out || !conv_out)) { set_error("null output pointer"); return PF_EINVAL; }
    if (mode != MODE_SOLVE && !aux) { set_error("null output pointer"); return PF_EINVAL; }
    if (mode == MODE_MISMATCH && !aux2) { set_error("null output pointer"); return PF_EINVAL; }
    if (mode == MODE_SOLVE && (max_iter < 0 || !(tol >= 0.0))) { set_error("invalid tol or max_iter"); return PF_EINVAL; }
    const TileLayout L = tile_layout(h, c);
    const int ntiles = (batch + c.tile - 1) / c.tile;
    const size_t need = L.bytes * (size_t)ntiles;
    if (!workspace || workspace_bytes < need) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return PF_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) { set_error("workspace must be 256-byte aligned"); return PF_EINVAL; }
    const size_t lds = lds_bytes(h, c);
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
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.p = pl->d;
    a.perm = pl->perm_dev;
    a.ybus = ybus; a.sbus = sbus; a.v0 = v0;
    a.tol = tol; a.max_iter = max_iter; a.batch = batch; a.mode = mode;
    a.ws = reinterpret_cast<char *>(workspace);
    a.tile_bytes = L.bytes; a.off_y = L.off_y; a.off_vec = L.off_vec;
    a.v_out = v_out; a.iters_out = iters_out; a.conv_out = conv_out; a.status_out = status_out;
    a.aux_out = aux; a.aux2_out = aux2;
    hipError_t e = launch(c, a, ntiles, lds, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) { set_error(std::string("kernel launch failed: ") + hipGetErrorString(e)); return PF_EDEVICE; }
    return PF_OK;
}

// ------------------------------------------------------------------ plan upload
struct DevOffsets {
    size_t bytes = 0;
    template <typename V>
    size_t add(const V &v)
    {
        size_t o = bytes;
        bytes = align256(bytes + v.size() * sizeof(typename V::value_type) + 1);
        return o;
    }
};

static int upload(Plan *pl)
{
    const HostPlan &h = pl->h;
    if (hipGetDevice(&pl->device) != hipSuccess) { set_error("no HIP device"); return PF_EDEVICE; }
    DevOffsets off;
    const size_t o_yrp = off.add(h.yrp), o_yci = off.add(h.yci), o_yrow = off.add(h.yrow);
    const size_t o_bt = off.add(h.bus_type), o_cp = off.add(h.col_ptr), o_cd = off.add(h.col_diag);
    const size_t o_desc = off.add(h.desc), o_up = off.add(h.upd_ptr), o_rel = off.add(h.rel);
    const size_t o_upd = off.add(h.upd), o_lp = off.add(h.lev_ptr);
    const size_t o_lc = off.add(h.lev_cols), o_blp = off.add(h.bs_lev_ptr), o_blr = off.add(h.bs_lev_rows);
    const size_t o_bp = off.add(h.bs_ptr), o_bpos = off.add(h.bs_pos), o_bcol = off.add(h.bs_col);
    const size_t o_pe = off.add(h.bus_peq), o_qe = off.add(h.bus_qeq), o_pu = off.add(h.pos_upd);
    const size_t o_perm = off.add(h.perm), o_pp = off.add(h.panel_ptr);
    std::vector<char> host(off.bytes, 0);
    auto put = [&](size_t o, const auto &v) {
        if (!v.empty()) std::memcpy(host.data() + o, v.data(), v.size() * sizeof(v[0]));
    };
    put(o_yrp, h.yrp); put(o_yci, h.yci); put(o_yrow, h.yrow); put(o_bt, h.bus_type);
    put(o_cp, h.col_ptr); put(o_cd, h.col_diag); put(o_desc, h.desc); put(o_up, h.upd_ptr);
    put(o_rel, h.rel); put(o_upd, h.upd); put(o_lp, h.lev_ptr);
    put(o_lc, h.lev_cols); put(o_blp, h.bs_lev_ptr); put(o_blr, h.bs_lev_rows); put(o_bp, h.bs_ptr);
    put(o_bpos, h.bs_pos); put(o_bcol, h.bs_col); put(o_pe, h.bus_peq); put(o_qe, h.bus_qeq);
    put(o_pu, h.pos_upd); put(o_perm, h.perm); put(o_pp, h.panel_ptr);
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
    d.n = h.n; d.nnzy = h.nnzy; d.N = h.N; d.nnzlu = h.col_ptr[h.N];
    d.n_levels = (int)h.lev_ptr.size() - 1; d.n_bs_levels = (int)h.bs_lev_ptr.size() - 1;
    d.max_col = h.max_col; d.npvpq = h.npvpq;
    d.yrp = (const int32_t *)(D + o_yrp); d.yci = (const int32_t *)(D + o_yci); d.yrow = (const int32_t *)(D + o_yrow);
    d.bus_type = (const int8_t *)(D + o_bt);
    d.col_ptr = (const int32_t *)(D + o_cp); d.col_diag = (const int32_t *)(D + o_cd); d.desc = (const JacDesc *)(D + o_desc);
    d.upd_ptr = (const int32_t *)(D + o_up); d.rel = (const int32_t *)(D + o_rel);
    d.upd = (const Update *)(D + o_upd);
    d.lev_ptr = (const int32_t *)(D + o_lp); d.lev_cols = (const int32_t *)(D + o_lc);
    d.bs_lev_ptr = (const int32_t *)(D + o_blp); d.bs_lev_rows = (const int32_t *)(D + o_blr);
    d.bs_ptr = (const int32_t *)(D + o_bp); d.bs_pos = (const int32_t *)(D + o_bpos); d.bs_col = (const int32_t *)(D + o_bcol);
    d.bus_peq = (const int32_t *)(D + o_pe); d.bus_qeq = (const int32_t *)(D + o_qe); d.pos_upd = (const int32_t *)(D + o_pu);
    pl->perm_dev = (const int32_t *)(D + o_perm);
    d.panel_ptr = (const int32_t *)(D + o_pp);
    d.n_panels = (int)h.panel_ptr.size() - 1;
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
    o->max_col = h.max_col;
    o->n_updates = (int64_t)h.upd.size();
    o->flops_refactor = h.flops;
    // compulsory bytes per instance-iteration: mismatch 32n+8N, Jacobian 16n+b nnz_lu,
    // refactor 2b nnz_lu, substitutions b nnz_lu + 16N, update 8N+32n
    o->bytes_iter_fp64 = 4 * 8 * (int64_t)o->nnz_lu + 80 * (int64_t)h.n + 32 * (int64_t)h.N;
    o->bytes_iter_fp32 = 4 * 4 * (int64_t)o->nnz_lu + 80 * (int64_t)h.n + 32 * (int64_t)h.N;
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

size_t pf_workspace_bytes(pf_plan plan, int32_t batch, const pf_solve_opts *opts)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl || batch <= 0) return 0;
    Config c;
    std::string err;
    if (!resolve_config(pl->h, opts, c, err)) { set_error(err); return 0; }
    const TileLayout L = tile_layout(pl->h, c);
    return L.bytes * (size_t)((batch + c.tile - 1) / c.tile);
}

int pf_solve_batch(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched,
                   const double *sbus, const double *v0, double tol, int32_t max_iter,
                   const pf_solve_opts *opts, void *workspace, size_t workspace_bytes,
                   double *v_out, int32_t *iters_out, uint8_t *converged_out,
                   int8_t *status_out, void *stream)
{
    if (ybus_batched != 0) { set_error("per-instance Ybus values are not supported"); return PF_EINVAL; }
    return run(plan, batch, ybus, sbus, v0, tol, max_iter, opts, workspace, workspace_bytes, MODE_SOLVE,
               v_out, iters_out, converged_out, status_out, nullptr, nullptr, stream);
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

void pf_plan_destroy(pf_plan plan)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl) return;
    if (pl->dev_mem) (void)hipFree(pl->dev_mem);
    delete pl;
}

}  // extern "C"
