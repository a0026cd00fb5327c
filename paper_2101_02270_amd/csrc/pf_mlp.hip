// Learned warm start for the Newton iteration: a small fully connected network whose
// layers run on gfx950 matrix cores.  Every layer is a dense contraction, so the GEMMs use
// MFMA (v_mfma_f32_16x16x16_bf16): BF16 operands, FP32 accumulation.
//
//   forward   Z = op(X) W + b,  A = GELU(Z) (exact erf form) or A = Z on the output layer
//   backward  dZ = dA * GELU'(Z);  dW = X^T dZ;  db = sum_rows dZ;  dX = dZ W^T
//   Adam      m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;  w -= lr mhat / (sqrt(vhat) + eps)
//             on FP32 master weights, re-rounded to the BF16 copy the GEMMs read
//
// All matrices are row-major.  One GEMM kernel serves the three products through two
// transpose flags on how its operands are read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>

#include "pf_internal.h"

namespace pf {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

// round to nearest even; NaN stays NaN
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

constexpr int BM = 64, BN = 64, BK = 32;

// C[M][N] (+)= op(A)[M][K] * op(B)[K][N]
//   op(A) = A (A stored [M][K]) or A^T (A stored [K][M]) when ta
//   op(B) = B (B stored [K][N]) or B^T (B stored [N][K]) when tb
// Epilogue: z = acc + bias[n]; zout (FP32) <- z; aout <- GELU(z) or z, as BF16 or FP32.
struct GemmArgs {
    int M, N, K, ta, tb;
    const uint16_t *A, *B;
    const float *bias;
    float *zout;          // may be null
    uint16_t *aout_bf16;  // may be null
    float *aout_f32;      // may be null
    int gelu;
};

__device__ __forceinline__ float gelu_erf(float z)
{
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_erf_grad(float z)
{
    const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
    return cdf + z * pdf;
}

// 256 threads = 4 wavefronts; the workgroup computes a 64x64 tile of C, each wavefront a
// 32x32 quarter as 2x2 MFMA tiles of 16x16.  K advances in slices of 32 staged in LDS.
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g)
{
    __shared__ uint16_t sA[BM][BK + 4];   // row m, column k
    __shared__ uint16_t sB[BN][BK + 4];   // column n, row k (k contiguous per column)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += BK) {
        // stage A: 64 x 32 elements, 8 per thread
        for (int e = tid; e < BM * BK; e += 256) {
            const int mm = e / BK, kk = e % BK;
            const int m = m0 + mm, k = k0 + kk;
            uint16_t v = 0;
            if (m < g.M && k < g.K) v = g.ta ? g.A[(size_t)k * g.M + m] : g.A[(size_t)m * g.K + k];
            sA[mm][kk] = v;
        }
        for (int e = tid; e < BN * BK; e += 256) {
            const int nn = e / BK, kk = e % BK;
            const int n = n0 + nn, k = k0 + kk;
            uint16_t v = 0;
            if (n < g.N && k < g.K) v = g.tb ? g.B[(size_t)n * g.K + k] : g.B[(size_t)k * g.N + n];
            sB[nn][kk] = v;
        }
        __syncthreads();
        for (int ks = 0; ks < BK; ks += 16) {
            // A operand of a 16x16x16 MFMA: lane holds row (lane % 16), k = 4 (lane / 16) + 0..3
            // B operand: column (lane % 16), the same k
            bf16x4 av[2], bv[2];
            const int kq = ks + 4 * (lane >> 4);
            for (int a = 0; a < 2; a++) {
                const int r = wm + 16 * a + (lane & 15);
                av[a] = bf16x4{(short)sA[r][kq], (short)sA[r][kq + 1], (short)sA[r][kq + 2], (short)sA[r][kq + 3]};
            }
            for (int b = 0; b < 2; b++) {
                const int c = wn + 16 * b + (lane & 15);
                bv[b] = bf16x4{(short)sB[c][kq], (short)sB[c][kq + 1], (short)sB[c][kq + 2], (short)sB[c][kq + 3]};
            }
            for (int a = 0; a < 2; a++)
                for (int b = 0; b < 2; b++)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // D of a 16x16 MFMA: lane holds column (lane % 16), rows 4 (lane / 16) + 0..3
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int r = 0; r < 4; r++) {
                const int m = m0 + wm + 16 * a + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * b + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float z = acc[a][b][r] + (g.bias ? g.bias[n] : 0.f);
                const size_t o = (size_t)m * g.N + n;
                if (g.zout) g.zout[o] = z;
                const float act = g.gelu ? gelu_erf(z) : z;
                if (g.aout_bf16) g.aout_bf16[o] = f32_to_bf16(act);
                if (g.aout_f32) g.aout_f32[o] = act;
            }
}

// The same product on 128 x 128 tiles of C with gfx950's 16x16x32 BF16 MFMA: 256 threads
// = 4 wavefronts of 64 x 64 (4 x 4 MFMA tiles each).  K advances in slices of 32: every
// thread loads 4-byte pairs of both operands' slices (coalesced along each operand's
// contiguous dimension) for the next slice while the current one is multiplied from LDS,
// where both operands sit K-contiguous per row / column (an operand stored contiguous
// along M or N is transposed on the way in).  Needs the contiguous dimension of each
// stored operand to be even (4-byte pairs) and 4-byte aligned pointers.
constexpr int TBN = 128, TBK = 32, TLD = TBK + 8;    // LDS row: 80 B, 16-B aligned

// the NP pairs this thread loads of one operand's ROWS x 32 slice: operand row r (an M or
// N index, rows0 + r < rows) and depth k (k0 + k < K); stored contiguous along K (trans =
// false: element (r, k) at p[r * K + k]) or along r (trans: element (r, k) at p[k * rows + r])
template <int NP, int ROWS>
__device__ __forceinline__ void tile_fetch(uint32_t *dst, const uint16_t *p, int rows0, int rows, int k0, int K,
                                          bool trans, int tid)
{
#pragma unroll
    for (int j = 0; j < NP; j++) {
        const int e = tid + 256 * j;
        uint32_t v = 0;
        if (!trans) {
            const int r = e >> 4, k = k0 + 2 * (e & 15);             // 16 pairs per row
            if (rows0 + r < rows && k < K) v = *reinterpret_cast<const uint32_t *>(p + (size_t)(rows0 + r) * K + k);
        } else {
            const int k = e / (ROWS / 2), r = rows0 + 2 * (e % (ROWS / 2));    // ROWS / 2 pairs per depth
            if (k0 + k < K && r < rows) v = *reinterpret_cast<const uint32_t *>(p + (size_t)(k0 + k) * rows + r);
        }
        dst[j] = v;
    }
}

template <int NP, int ROWS>
__device__ __forceinline__ void tile_store(uint16_t (*sm)[TLD], const uint32_t *src, bool trans, int tid)
{
#pragma unroll
    for (int j = 0; j < NP; j++) {
        const int e = tid + 256 * j;
        if (!trans) {
            *reinterpret_cast<uint32_t *>(&sm[e >> 4][2 * (e & 15)]) = src[j];
        } else {
            const int k = e / (ROWS / 2), r = 2 * (e % (ROWS / 2));
            sm[r][k] = (uint16_t)(src[j] & 0xffffu);
            sm[r + 1][k] = (uint16_t)(src[j] >> 16);
        }
    }
}

// BM x 128 tiles of C (BM = 128 or 64): 4 wavefronts of BM/2 x 64, (BM/32) x 4 MFMA tiles each
template <int BM>
__global__ __launch_bounds__(256) void gemm_bf16_mfma32_kernel(GemmArgs g)
{
    constexpr int MI = BM / 32, NPA = BM * TBK / 2 / 256, NPB = TBN * TBK / 2 / 256;
    __shared__ __align__(16) uint16_t sA[BM][TLD];    // row m, k contiguous
    __shared__ __align__(16) uint16_t sB[TBN][TLD];   // column n, k contiguous
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * TBN;
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * 64;
    // A stored [M][K] (k contiguous) unless ta; B stored [N][K] (k contiguous) when tb
    const bool a_tr = g.ta != 0, b_tr = g.tb == 0;
    floatx4 acc[MI][4];
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    uint32_t la[NPA], lb[NPB];
    tile_fetch<NPA, BM>(la, g.A, m0, g.M, 0, g.K, a_tr, tid);
    tile_fetch<NPB, TBN>(lb, g.B, n0, g.N, 0, g.K, b_tr, tid);
    for (int k0 = 0; k0 < g.K; k0 += TBK) {
        tile_store<NPA, BM>(sA, la, a_tr, tid);
        tile_store<NPB, TBN>(sB, lb, b_tr, tid);
        __syncthreads();
        if (k0 + TBK < g.K) {
            tile_fetch<NPA, BM>(la, g.A, m0, g.M, k0 + TBK, g.K, a_tr, tid);
            tile_fetch<NPB, TBN>(lb, g.B, n0, g.N, k0 + TBK, g.K, b_tr, tid);
        }
        // operands of a 16x16x32 MFMA: lane holds row / column (lane % 16), k = 8 (lane / 16) + 0..7
        const int kq = 8 * (lane >> 4);
        bf16x8 av[MI], bv[4];
#pragma unroll
        for (int i = 0; i < MI; i++) av[i] = *reinterpret_cast<const bf16x8 *>(&sA[wm + 16 * i + (lane & 15)][kq]);
#pragma unroll
        for (int j = 0; j < 4; j++) bv[j] = *reinterpret_cast<const bf16x8 *>(&sB[wn + 16 * j + (lane & 15)][kq]);
#pragma unroll
        for (int i = 0; i < MI; i++)
#pragma unroll
            for (int j = 0; j < 4; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // D of a 16x16 MFMA: lane holds column (lane % 16), rows 4 (lane / 16) + 0..3
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int n = n0 + wn + 16 * j + (lane & 15);
            if (n >= g.N) continue;
            const float bias = g.bias ? g.bias[n] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                if (m >= g.M) continue;
                const float z = acc[i][j][r] + bias;
                const size_t o = (size_t)m * g.N + n;
                if (g.zout) g.zout[o] = z;
                const float act = g.gelu ? gelu_erf(z) : z;
                if (g.aout_bf16) g.aout_bf16[o] = f32_to_bf16(act);
                if (g.aout_f32) g.aout_f32[o] = act;
            }
        }
}

// rows of C per tile: 64 when 128-row tiles would leave CUs without a second workgroup
constexpr int kGemmSmallTileBelow = 512;

// dZ = dA * GELU'(Z) (or dA) rounded to BF16 for the backward GEMMs, and db = column sums of
// dZ (FP32, from the unrounded values).  One thread per column, looping over rows.
__global__ void act_backward_kernel(int M, int N, const float *dA, const float *Z, int gelu, uint16_t *dZ,
                                    float *db)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; m++) {
        const size_t o = (size_t)m * N + n;
        float d = dA[o];
        if (gelu) d *= gelu_erf_grad(Z[o]);
        dZ[o] = f32_to_bf16(d);
        s += d;
    }
    if (db) db[n] = s;
}

// Mean-squared error over all entries: loss = sum (p - y)^2 / count, grad = 2 (p - y) / count.
__global__ void mse_kernel(size_t count, const float *pred, const float *target, float *grad, float *loss_parts)
{
    __shared__ float red[256];
    float s = 0.f;
    const float inv = 1.0f / (float)count;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const float d = pred[i] - target[i];
        grad[i] = 2.0f * d * inv;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_parts[blockIdx.x] = red[0] * inv;
}

__global__ void adam_kernel(size_t n, float *w, uint16_t *w_bf16, const float *grad, float *m, float *v, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = grad[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        if (w_bf16) w_bf16[i] = f32_to_bf16(wi);
    }
}

__global__ void to_bf16_kernel(size_t n, const float *x, uint16_t *y)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = f32_to_bf16(x[i]);
}

// Network features from the specified injections: for every non-REF bus in bus order,
// (P, Q) at PQ buses and (P, |V| set-point) at PV buses, z-scored with (mu, sigma).
__global__ void features_kernel(int B, int n, const double *sbus, const double *v0, const int8_t *bus_type,
                                const int32_t *feat_bus, int nf_bus, const float *mu, const float *sigma,
                                uint16_t *x_bf16)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;   // feature pair index
    const int b = blockIdx.y;
    if (f >= nf_bus || b >= B) return;
    const int i = feat_bus[f];
    const size_t o = ((size_t)b * n + i) * 2;
    const double p = sbus[o];
    const double s2 = bus_type[i] == PF_BUS_PV ? v0[o] : sbus[o + 1];
    const size_t xo = (size_t)b * 2 * nf_bus + 2 * f;
    x_bf16[xo] = f32_to_bf16(((float)p - mu[2 * f]) / sigma[2 * f]);
    x_bf16[xo + 1] = f32_to_bf16(((float)s2 - mu[2 * f + 1]) / sigma[2 * f + 1]);
}

// Initial voltages from the network output (de-normalised with (mu, sigma)): angle and |V|
// for every non-REF bus; |V| of PV buses and the whole REF bus keep their set-points from
// v_set.  Non-finite predictions fall back to v_set (flat start) for that bus.
__global__ void warm_v0_kernel(int B, int n, const float *out, const int32_t *feat_bus, int nf_bus,
                               const float *mu, const float *sigma, const int8_t *bus_type, const double *v_set,
                               double *v0)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (b >= B) return;
    if (f < nf_bus) {
        const int i = feat_bus[f];
        const size_t oo = (size_t)b * 2 * nf_bus + 2 * f;
        double vm = (double)(out[oo] * sigma[2 * f] + mu[2 * f]);
        double va = (double)(out[oo + 1] * sigma[2 * f + 1] + mu[2 * f + 1]);
        const size_t o = ((size_t)b * n + i) * 2;
        if (bus_type[i] == PF_BUS_PV || !isfinite(vm) || vm <= 0.0) vm = v_set[o];
        if (!isfinite(va)) va = v_set[o + 1];
        v0[o] = vm;
        v0[o + 1] = va;
    }
    // the REF bus (the one bus without a feature slot) keeps its set-points
    if (f < n && bus_type[f] == PF_BUS_REF) {
        const size_t o = ((size_t)b * n + f) * 2;
        v0[o] = v_set[o];
        v0[o + 1] = v_set[o + 1];
    }
}

static int launch_status(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return PF_EDEVICE;
    }
    return PF_OK;
}

static int grid1(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 4096); }

}  // namespace pf

using namespace pf;

extern "C" {

int pf_mlp_gemm(int32_t M, int32_t N, int32_t K, int32_t trans_a, int32_t trans_b, const uint16_t *a,
                const uint16_t *b, const float *bias, int32_t gelu, float *z_out, uint16_t *act_bf16_out,
                float *act_f32_out, void *stream)
{
    if (M < 0 || N < 0 || K < 0 || !a || !b) { set_error("pf_mlp_gemm: bad arguments"); return PF_EINVAL; }
    if (M == 0 || N == 0) return PF_OK;
    GemmArgs g{M, N, K, trans_a ? 1 : 0, trans_b ? 1 : 0, a, b, bias, z_out, act_bf16_out, act_f32_out, gelu ? 1 : 0};
    // the 128 x 128 MFMA kernel loads 4-byte pairs along each stored operand's contiguous
    // dimension (K for A, or M when trans_a; N for B, or K when trans_b)
    const int a_contig = trans_a ? M : K, b_contig = trans_b ? K : N;
    const bool pairs = a_contig % 2 == 0 && b_contig % 2 == 0 && (reinterpret_cast<uintptr_t>(a) & 3) == 0 &&
                       (reinterpret_cast<uintptr_t>(b) & 3) == 0;
    if (pairs) {
        const int tiles128 = ((N + TBN - 1) / TBN) * ((M + 127) / 128);
        if (tiles128 < kGemmSmallTileBelow) {
            dim3 grid((N + TBN - 1) / TBN, (M + 63) / 64);
            hipLaunchKernelGGL(gemm_bf16_mfma32_kernel<64>, grid, dim3(256), 0, (hipStream_t)stream, g);
        } else {
            dim3 grid((N + TBN - 1) / TBN, (M + 127) / 128);
            hipLaunchKernelGGL(gemm_bf16_mfma32_kernel<128>, grid, dim3(256), 0, (hipStream_t)stream, g);
        }
    } else {
        dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
        hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, (hipStream_t)stream, g);
    }
    return launch_status("pf_mlp_gemm");
}

int pf_mlp_act_backward(int32_t M, int32_t N, const float *d_act, const float *z, int32_t gelu,
                        uint16_t *dz_bf16, float *db, void *stream)
{
    if (M < 0 || N < 0 || !d_act || !dz_bf16 || (gelu && !z)) { set_error("pf_mlp_act_backward: bad arguments"); return PF_EINVAL; }
    if (N == 0) return PF_OK;
    hipLaunchKernelGGL(act_backward_kernel, dim3((N + 255) / 256), dim3(256), 0, (hipStream_t)stream, M, N, d_act, z,
                       gelu ? 1 : 0, dz_bf16, db);
    return launch_status("pf_mlp_act_backward");
}

int pf_mlp_mse(int64_t count, const float *pred, const float *target, float *grad, float *loss_parts,
               int32_t n_parts, void *stream)
{
    if (count <= 0 || !pred || !target || !grad || !loss_parts || n_parts < 1) { set_error("pf_mlp_mse: bad arguments"); return PF_EINVAL; }
    hipLaunchKernelGGL(mse_kernel, dim3(n_parts), dim3(256), 0, (hipStream_t)stream, (size_t)count, pred, target, grad,
                       loss_parts);
    return launch_status("pf_mlp_mse");
}

int pf_mlp_adam(int64_t n, float *w, uint16_t *w_bf16, const float *grad, float *m, float *v, float lr,
                float beta1, float beta2, float eps, int32_t step, void *stream)
{
    if (n <= 0 || !w || !grad || !m || !v || step < 1) { set_error("pf_mlp_adam: bad arguments"); return PF_EINVAL; }
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(grid1((size_t)n)), dim3(256), 0, (hipStream_t)stream, (size_t)n, w, w_bf16, grad,
                       m, v, lr, beta1, beta2, eps, c1, c2);
    return launch_status("pf_mlp_adam");
}

int pf_mlp_to_bf16(int64_t n, const float *x, uint16_t *y, void *stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) { set_error("pf_mlp_to_bf16: bad arguments"); return PF_EINVAL; }
    if (n == 0) return PF_OK;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid1((size_t)n)), dim3(256), 0, (hipStream_t)stream, (size_t)n, x, y);
    return launch_status("pf_mlp_to_bf16");
}

int pf_mlp_features(int32_t batch, int32_t n_bus, const double *sbus, const double *v0, const int8_t *bus_type,
                    const int32_t *feat_bus, int32_t nf_bus, const float *mu, const float *sigma, uint16_t *x_bf16,
                    void *stream)
{
    if (batch < 0 || n_bus < 1 || nf_bus < 0 || !sbus || !v0 || !bus_type || !feat_bus || !mu || !sigma || !x_bf16) {
        set_error("pf_mlp_features: bad arguments");
        return PF_EINVAL;
    }
    if (batch == 0 || nf_bus == 0) return PF_OK;
    if (batch > 65535) { set_error("pf_mlp_features: batch above 65535"); return PF_EINVAL; }
    hipLaunchKernelGGL(features_kernel, dim3((nf_bus + 255) / 256, batch), dim3(256), 0, (hipStream_t)stream, batch,
                       n_bus, sbus, v0, bus_type, feat_bus, nf_bus, mu, sigma, x_bf16);
    return launch_status("pf_mlp_features");
}

int pf_mlp_warm_v0(int32_t batch, int32_t n_bus, const float *out, const int32_t *feat_bus, int32_t nf_bus,
                   const float *mu, const float *sigma, const int8_t *bus_type, const double *v_set, double *v0,
                   void *stream)
{
    if (batch < 0 || n_bus < 1 || nf_bus < 0 || !out || !feat_bus || !mu || !sigma || !bus_type || !v_set || !v0) {
        set_error("pf_mlp_warm_v0: bad arguments");
        return PF_EINVAL;
    }
    if (batch == 0) return PF_OK;
    if (batch > 65535) { set_error("pf_mlp_warm_v0: batch above 65535"); return PF_EINVAL; }
    hipLaunchKernelGGL(warm_v0_kernel, dim3((std::max(nf_bus, n_bus) + 255) / 256, batch), dim3(256), 0,
                       (hipStream_t)stream, batch,
                       n_bus, out, feat_bus, nf_bus, mu, sigma, bus_type, v_set, v0);
    return launch_status("pf_mlp_warm_v0");
}

}  // extern "C"
