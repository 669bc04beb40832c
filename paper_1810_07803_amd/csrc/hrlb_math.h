// Elementary functions of the kernels that are written out here rather than taken from the device
// library, as host-and-device functions so that a CPU check can measure their accuracy
// (tests/exp_check.cpp).
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define HRLB_HD __host__ __device__
#else
#define HRLB_HD
#endif

namespace hrlb {

// e^x in FP64 for the projection of eq. (gx) and the viscosity law, by Cody and Waite's reduction
// x = k ln 2 + r, |r| <= ln(2)/2 (k = rint(x log2 e); ln 2 as the nearest double plus its remainder,
// each product taken off with one rounding), then the Taylor polynomial of e^r to degree 13 in
// Horner form (truncation below 2e-16 relative) and the scaling by 2^k.  Within an ulp of e^x over
// [-700, 700] against the long-double exponential (tests/exp_check.cpp); overflow to +inf and
// underflow to 0 as the scaling gives them; a non-finite argument gives NaN (only reached from a
// state that the residual check flags).  About half the instructions of the library's exp, which
// also handles the special arguments.
HRLB_HD inline double exp_cw(double x)
{
    constexpr double kLog2e = 1.4426950408889634, kLn2Hi = 0.6931471805599453, kLn2Lo = 2.3190468138462996e-17;
    const double k = rint(x * kLog2e);
    const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, x));
    double p = 1.6059043836821613e-10;   // 1/13!
    p = fma(p, r, 2.08767569878681e-09);  // 1/12!
    p = fma(p, r, 2.505210838544172e-08);
    p = fma(p, r, 2.755731922398589e-07);
    p = fma(p, r, 2.7557319223985893e-06);
    p = fma(p, r, 2.48015873015873e-05);
    p = fma(p, r, 0.0001984126984126984);
    p = fma(p, r, 0.001388888888888889);
    p = fma(p, r, 0.008333333333333333);
    p = fma(p, r, 0.041666666666666664);
    p = fma(p, r, 0.16666666666666666);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)fmin(fmax(k, -2100.0), 2100.0));  // clamped: the conversion is defined everywhere
}

}  // namespace hrlb
