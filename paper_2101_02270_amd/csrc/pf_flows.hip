// Branch power flows and losses at solved voltages: the post-processing step that follows
// the final convergence check, computed in parallel over instances (Sec. 3.2).  Pi-model
// branches with series admittance y = 1/(r + jx) and total charging b split b/2 per end:
//   I_from = y (V_from - V_to) + j b/2 V_from,   S_from = V_from conj(I_from)
//   I_to   = y (V_to - V_from) + j b/2 V_to,     S_to   = V_to conj(I_to)
// and the instance's losses are the sum over branches of S_from + S_to.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "pf_internal.h"
#include "pf_math.h"

namespace pf {

// One workgroup per instance; threads stride over the branches.  Bus indices outside
// [0, n) give NaN flows instead of a read outside the instance's voltages.
__global__ __launch_bounds__(256) void branch_flows_kernel(int n, int m, const int32_t *fb, const int32_t *tb,
                                                         const double *r, const double *x, const double *bt,
                                                         const double *v, double *sf, double *st, double *loss)
{
    const int b = blockIdx.x;
    const double *vb = v + (size_t)b * n * 2;
    double lr = 0.0, li = 0.0;
    for (int e = threadIdx.x; e < m; e += blockDim.x) {
        const int f = fb[e], t = tb[e];
        double sfr, sfi, str, sti;
        if (f < 0 || f >= n || t < 0 || t >= n) {
            sfr = sfi = str = sti = NAN;
        } else {
            double sn, cs;
            sincos_angle(vb[2 * f + 1], &sn, &cs);
            const double vfr = vb[2 * f] * cs, vfi = vb[2 * f] * sn;
            sincos_angle(vb[2 * t + 1], &sn, &cs);
            const double vtr = vb[2 * t] * cs, vti = vb[2 * t] * sn;
            const double d = r[e] * r[e] + x[e] * x[e];
            const double yr = r[e] / d, yi = -x[e] / d;
            const double hb = 0.5 * bt[e];
            const double dr = vfr - vtr, di = vfi - vti;
            const double cr = yr * dr - yi * di, ci = yr * di + yi * dr;     // y (V_f - V_t)
            const double ifr = cr - hb * vfi, ifi = ci + hb * vfr;
            const double itr = -cr - hb * vti, iti = -ci + hb * vtr;
            sfr = vfr * ifr + vfi * ifi; sfi = vfi * ifr - vfr * ifi;
            str = vtr * itr + vti * iti; sti = vti * itr - vtr * iti;
        }
        const size_t o = ((size_t)b * m + e) * 2;
        sf[o] = sfr; sf[o + 1] = sfi;
        st[o] = str; st[o + 1] = sti;
        lr += sfr + str;
        li += sfi + sti;
    }
    if (!loss) return;
    __shared__ double s_r[4], s_i[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lr += __shfl_xor(lr, off);
        li += __shfl_xor(li, off);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { s_r[wave] = lr; s_i[wave] = li; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tr = 0.0, ti = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) { tr += s_r[w]; ti += s_i[w]; }
        loss[2 * (size_t)b] = tr;
        loss[2 * (size_t)b + 1] = ti;
    }
}

}  // namespace pf

using namespace pf;

extern "C" int pf_branch_flows(int32_t n_bus, int32_t n_branch, const int32_t *from_bus, const int32_t *to_bus,
                               const double *r, const double *x, const double *b_total, int32_t batch,
                               const double *v, double *s_from, double *s_to, double *loss, void *stream)
{
    if (n_bus <= 0 || n_branch < 0 || batch < 0) { set_error("invalid sizes"); return PF_EINVAL; }
    if (batch == 0 || n_branch == 0) return PF_OK;
    if (!from_bus || !to_bus || !r || !x || !b_total || !v || !s_from || !s_to) {
        set_error("null pointer");
        return PF_EINVAL;
    }
    hipLaunchKernelGGL(branch_flows_kernel, dim3(batch), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), n_bus,
                       n_branch, from_bus, to_bus, r, x, b_total, v, s_from, s_to, loss);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_error(std::string("kernel launch failed: ") + hipGetErrorString(e)); return PF_EDEVICE; }
    return PF_OK;
}
