// Device math shared by the solver and the branch-flow kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace pf {

// sin and cos of a voltage angle.  Reduction x = k pi/2 + r with k = rint(2x/pi) and
// pi/2 split into three doubles (c1 = RN(pi/2), c2 = RN(pi/2 - c1), c3 = RN(pi/2 - c1 - c2)),
// each step one fused multiply-add; then the Taylor series of sin r (to r^17) and cos r (to
// r^18) on |r| <= pi/4, whose truncation error is below 1e-19, and the quadrant k mod 4.
// Absolute error a few ulp for |x| < 2^20 pi/2; larger angles (only seen in diverging
// solves) keep a finite but less accurate result, and NaN propagates.  A short path with
// few live registers: the general library routine carries a long-argument reduction.
__device__ __forceinline__ void sincos_angle(double x, double *sn, double *cs)
{
    constexpr double two_over_pi = 0x1.45f306dc9c883p-1;
    constexpr double c1 = 0x1.921fb54442d18p+0, c2 = 0x1.1a62633145c07p-54, c3 = -0x1.f1976b7ed8fbcp-110;
    const double k = rint(x * two_over_pi);
    double r = fma(-k, c1, x);
    r = fma(-k, c2, r);
    r = fma(-k, c3, r);
    const double r2 = r * r;
    // (-1)^m / (2m+1)!  and  (-1)^m / (2m)!
    double ps = 2.8114572543455206e-15;
    ps = fma(ps, r2, -7.647163731819816e-13);
    ps = fma(ps, r2, 1.6059043836821613e-10);
    ps = fma(ps, r2, -2.505210838544172e-08);
    ps = fma(ps, r2, 2.7557319223985893e-06);
    ps = fma(ps, r2, -0.0001984126984126984);
    ps = fma(ps, r2, 0.008333333333333333);
    ps = fma(ps, r2, -0.16666666666666666);
    const double s = fma(r * r2, ps, r);
    double pc = -1.5619206968586225e-16;
    pc = fma(pc, r2, 4.779477332387385e-14);
    pc = fma(pc, r2, -1.1470745597729725e-11);
    pc = fma(pc, r2, 2.08767569878681e-09);
    pc = fma(pc, r2, -2.755731922398589e-07);
    pc = fma(pc, r2, 2.48015873015873e-05);
    pc = fma(pc, r2, -0.001388888888888889);
    pc = fma(pc, r2, 0.041666666666666664);
    pc = fma(pc, r2, -0.5);
    const double c = fma(r2, pc, 1.0);
    const int q = (int)((long long)fmin(fmax(k, -0x1p52), 0x1p52) & 3);
    const double s_out = (q & 1) ? c : s, c_out = (q & 1) ? s : c;
    *sn = (q & 2) ? -s_out : s_out;
    *cs = ((q + 1) & 2) ? -c_out : c_out;
}

}  // namespace pf
