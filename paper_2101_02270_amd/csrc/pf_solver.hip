// Batched Newton-Raphson power flow on gfx950: one fused, persistent-per-tile kernel.
//
// A workgroup owns a tile of T instances and runs their whole Newton loop (Sec. 3 of
// the paper) without leaving the kernel:
//   M   mismatch S = V o conj(Y V) (Eq. 1), F = calculated - specified (Alg. 1), the
//       per-instance infinity norm by wavefront shuffles and an LDS reduction, and the
//       convergence / divergence decision;
//   LU  level by level (Sec. 4.3.1), each wavefront takes a column j of A = P J P^T:
//       it builds the Jacobian entries of the column straight from V and Ybus into an
//       LDS working column (Sec. 3.1.2 "direct into permuted form A"), applies the
//       left-looking updates from every finished column k with U(k,j) != 0 in ascending
//       k (Alg. 2, the sparse VMAD with direct indexing of Alg. 3), carries the forward
//       substitution of the right-hand side along (row j of L is read in the same
//       pass), normalises the L part and writes the column back;
//   BS  backward substitution by row levels, one wavefront per row, and the voltage
//       update V <- V - dx for instances still iterating.
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
template <int T>
__device__ __forceinline__ double jac_entry(int desc, int t, const int32_t *yrow, const int32_t *yci,
                                            const double *ybus, const double *Vm, const double *Vr,
                                            const double *Vi, const double *Ir, const double *Ii)
{
    if (desc < 0) return 0.0;
    const int p = desc >> 2, kind = desc & 3;
    const int i = yrow[p], k = yci[p];
    const double g = ybus[2 * p], bsus = ybus[2 * p + 1];
    const double vri = Vr[i * T + t], vii = Vi[i * T + t];
    double re, im;
    if (i != k) {
        const double vrk = Vr[k * T + t], vik = Vi[k * T + t];
        const double cr = g * vrk - bsus * vik, ci = g * vik + bsus * vrk;      // Y_ik V_k
        const double wr = vri * cr + vii * ci, wi = vii * cr - vri * ci;          // V_i conj(.)
        if (kind & 1) {
            const double inv = 1.0 / Vm[k * T + t];
            re = wr * inv; im = wi * inv;
        } else {
            re = wi; im = -wr;
        }
    } else {
        const double ir = Ir[i * T + t], ii = Ii[i * T + t];
        const double sr = vri * ir + vii * ii, si = vii * ir - vri * ii;          // S_i
        const double vmi = Vm[i * T + t];
        if (kind & 1) {
            re = sr / vmi + vmi * g;
            im = si / vmi - vmi * bsus;
        } else {
            const double m2 = vmi * vmi;
            re = -si - m2 * bsus;
            im = sr - m2 * g;
        }
    }
    return (kind & 2) ? im : re;
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
    __shared__ int s_any;

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
    double *Vm = vec, *Va = vec + nT, *Vr = vec + 2 * nT, *Vi = vec + 3 * nT;
    double *Ir = vec + 4 * nT, *Ii = vec + 5 * nT, *Ps = vec + 6 * nT, *Qs = vec + 7 * nT;

    R *xw = reinterpret_cast<R *>(smem_raw) + (size_t)wave * (P.max_col * T + T);
    R *ysl = xw + (size_t)P.max_col * T;

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
    __syncthreads();

    for (int it = 0;; ++it) {
        // ============================ M: mismatch and convergence test
        for (int i = slot; i < n; i += SLOTS) {
            double sn, cs;
            const double vm = Vm[i * T + t];
            sincos(Va[i * T + t], &sn, &cs);
            Vr[i * T + t] = vm * cs;
            Vi[i * T + t] = vm * sn;
        }
        __syncthreads();
        double mx = 0.0;
        int bad = 0;
        for (int i = slot; i < n; i += SLOTS) {
            double ir = 0.0, ii = 0.0;
            for (int q = P.yrp[i]; q < P.yrp[i + 1]; q++) {
                const int k = P.yci[q];
                const double g = a.ybus[2 * q], bs = a.ybus[2 * q + 1];
                const double vr = Vr[k * T + t], vi = Vi[k * T + t];
                ir += g * vr - bs * vi;
                ii += g * vi + bs * vr;
            }
            Ir[i * T + t] = ir;
            Ii[i * T + t] = ii;
            const double vr = Vr[i * T + t], vi = Vi[i * T + t];
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
        for (int lv = 0; lv < P.n_levels; lv++) {
            const int c1 = P.lev_ptr[lv + 1];
            for (int c = P.lev_ptr[lv] + wave; c < c1; c += NW) {
                const int j = P.lev_cols[c];
                const int cs = P.col_ptr[j];
                const int cnt = P.col_ptr[j + 1] - cs;
                const int dr = P.col_diag[j];
                for (int e = s; e < cnt; e += SL)
                    xw[e * T + t] = (R)jac_entry<T>(P.desc[cs + e], t, P.yrow, P.yci, a.ybus, Vm, Vr, Vi, Ir, Ii);
                if (s == 0) ysl[t] = Yv[j * T + t];
                wave_sync();
                const int u1 = P.upd_ptr[j + 1];
                for (int u = P.upd_ptr[j]; u < u1; u++) {
                    const Update up = P.upd[u];
                    const int k = P.upd_k[u];
                    const R m = xw[up.krel * T + t];
                    for (int r = s; r < up.lcnt; r += SL) {
                        const R l = LU[(size_t)(up.lbeg + r) * T + t];
                        const int tr = P.rel[up.roff + r];
                        xw[tr * T + t] = fma(-m, l, xw[tr * T + t]);
                        if (tr == dr) ysl[t] = fma(-l, Yv[k * T + t], ysl[t]);
                    }
                    wave_sync();
                }
                const R d = xw[dr * T + t];
                if (s == 0 && valid && !(fabs((double)d) > 1e-300 && isfinite((double)d))) s_piv[t] = 1;
                for (int e = dr + 1 + s; e < cnt; e += SL) xw[e * T + t] = xw[e * T + t] / d;
                wave_sync();
                for (int e = s; e < cnt; e += SL) LU[(size_t)(cs + e) * T + t] = xw[e * T + t];
                if (s == 0) Yv[j * T + t] = ysl[t];
                wave_sync();
            }
            __syncthreads();
        }
        if (tid < T && s_piv[t] && s_active[t] && a.mode == MODE_SOLVE) {
            s_status[t] = PF_ST_PIVOT; s_active[t] = 0; s_iters[t] = it;
        }
        if (a.mode == MODE_FACTOR) {
            const size_t nnz = (size_t)P.nnzlu;
            if (valid)
                for (size_t e = slot; e < nnz; e += SLOTS) a.aux_out[(size_t)b * nnz + e] = (double)LU[e * T + t];
            return;
        }
        __syncthreads();

        // ============================ BS: backward substitution and voltage update
        const bool upd_v = (a.mode == MODE_SOLVE);
        for (int lv = 0; lv < P.n_bs_levels; lv++) {
            const int r1 = P.bs_lev_ptr[lv + 1];
            for (int r = P.bs_lev_ptr[lv] + wave; r < r1; r += NW) {
                const int j = P.bs_lev_rows[r];
                R acc = 0;
                const int q1 = P.bs_ptr[j + 1];
                for (int q = P.bs_ptr[j] + s; q < q1; q += SL)
                    acc = fma(LU[(size_t)P.bs_pos[q] * T + t], Yv[P.bs_col[q] * T + t], acc);
#pragma unroll
                for (int off = T; off < 64; off <<= 1) acc += __shfl_xor(acc, off);
                if (s == 0) {
                    const R z = (Yv[j * T + t] - acc) / LU[(size_t)(P.col_ptr[j] + P.col_diag[j]) * T + t];
                    Yv[j * T + t] = z;
                    if (upd_v && s_active[t]) {
                        const int pu = P.pos_upd[j];
                        const int bus = pu >> 1;
                        if (pu & 1) Vm[bus * T + t] -= (double)z;
                        else Va[bus * T + t] -= (double)z;
                    }
                }
            }
            __syncthreads();
        }
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
            a.iters_out[b] = s_iters[t];
            a.conv_out[b] = s_status[t] == PF_ST_CONVERGED ? 1 : 0;
            if (a.status_out) a.status_out[b] = (int8_t)s_status[t];
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
    return (size_t)c.waves * ((size_t)h.max_col * c.tile + c.tile) * rs;
}

static bool resolve_config(const HostPlan &h, const pf_solve_opts *o, Config &c, std::string &err)
{
    c.precision = o ? o->precision : PF_FP64;
    c.tile = o ? o->tile : 0;
    c.waves = o ? o->waves : 0;
    if (c.precision != PF_FP64 && c.precision != PF_FP32_LU) { err = "unknown precision"; return false; }
    if (c.tile == 0) c.tile = c.precision == PF_FP64 ? 16 : 32;
    if (c.waves == 0) c.waves = 4;
    const bool ok_tile = c.precision == PF_FP64 ? (c.tile == 8 || c.tile == 16) : (c.tile == 16 || c.tile == 32);
    if (!ok_tile) { err = "unsupported tile size for this precision"; return false; }
    if (c.waves != 2 && c.waves != 4 && c.waves != 8) { err = "waves must be 2, 4 or 8"; return false; }
    (void)h;
    return true;
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
    default: return launch_t<R, T, 8>(a, grid, lds, st);                       \
    }

static hipError_t launch(const Config &c, const KArgs &a, int grid, size_t lds, hipStream_t st)
{
    if (c.precision == PF_FP64) {
        if (c.tile == 8) { PF_DISPATCH_NW(double, 8) }
        PF_DISPATCH_NW(double, 16)
    } else {
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
    if (lds > 160 * 1024 - 8192) {
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
    const size_t o_uk = off.add(h.upd_k), o_upd = off.add(h.upd), o_lp = off.add(h.lev_ptr);
    const size_t o_lc = off.add(h.lev_cols), o_blp = off.add(h.bs_lev_ptr), o_blr = off.add(h.bs_lev_rows);
    const size_t o_bp = off.add(h.bs_ptr), o_bpos = off.add(h.bs_pos), o_bcol = off.add(h.bs_col);
    const size_t o_pe = off.add(h.bus_peq), o_qe = off.add(h.bus_qeq), o_pu = off.add(h.pos_upd);
    const size_t o_perm = off.add(h.perm);
    std::vector<char> host(off.bytes, 0);
    auto put = [&](size_t o, const auto &v) {
        if (!v.empty()) std::memcpy(host.data() + o, v.data(), v.size() * sizeof(v[0]));
    };
    put(o_yrp, h.yrp); put(o_yci, h.yci); put(o_yrow, h.yrow); put(o_bt, h.bus_type);
    put(o_cp, h.col_ptr); put(o_cd, h.col_diag); put(o_desc, h.desc); put(o_up, h.upd_ptr);
    put(o_rel, h.rel); put(o_uk, h.upd_k); put(o_upd, h.upd); put(o_lp, h.lev_ptr);
    put(o_lc, h.lev_cols); put(o_blp, h.bs_lev_ptr); put(o_blr, h.bs_lev_rows); put(o_bp, h.bs_ptr);
    put(o_bpos, h.bs_pos); put(o_bcol, h.bs_col); put(o_pe, h.bus_peq); put(o_qe, h.bus_qeq);
    put(o_pu, h.pos_upd); put(o_perm, h.perm);
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
    d.col_ptr = (const int32_t *)(D + o_cp); d.col_diag = (const int32_t *)(D + o_cd); d.desc = (const int32_t *)(D + o_desc);
    d.upd_ptr = (const int32_t *)(D + o_up); d.rel = (const int32_t *)(D + o_rel); d.upd_k = (const int32_t *)(D + o_uk);
    d.upd = (const Update *)(D + o_upd);
    d.lev_ptr = (const int32_t *)(D + o_lp); d.lev_cols = (const int32_t *)(D + o_lc);
    d.bs_lev_ptr = (const int32_t *)(D + o_blp); d.bs_lev_rows = (const int32_t *)(D + o_blr);
    d.bs_ptr = (const int32_t *)(D + o_bp); d.bs_pos = (const int32_t *)(D + o_bpos); d.bs_col = (const int32_t *)(D + o_bcol);
    d.bus_peq = (const int32_t *)(D + o_pe); d.bus_qeq = (const int32_t *)(D + o_qe); d.pos_upd = (const int32_t *)(D + o_pu);
    pl->perm_dev = (const int32_t *)(D + o_perm);
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
