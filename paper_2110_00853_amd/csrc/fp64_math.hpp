// FP64 elementary functions of the device thermodynamics: reciprocal,
// square root, natural logarithm and exponential, written out so that the
// passes spend few vector instructions on them.  Built with
// CM_LIBM_THERMO defined, the same names call the HIP library's IEEE
// division, sqrt, log and exp instead (a switch for accuracy comparisons;
// the default build uses the forms below).
#pragma once

#include <hip/hip_runtime.h>

namespace cm {

#ifdef CM_LIBM_THERMO

__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float frcp(float x) { return 1.0f / x; }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double ln_pos(double x) { return log(x); }
__device__ __forceinline__ double exp_fin(double y) { return exp(y); }

#else

// FP64 reciprocal and square root from the hardware estimates refined by
// Newton-Raphson (reciprocal) and Goldschmidt (square root) steps: within an
// ulp of the correctly rounded results, at a third of the instructions of
// the IEEE sequences.  Arguments are positive and finite.
__device__ __forceinline__ double frcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float frcp(float x) { return 1.0f / x; }

__device__ __forceinline__ double fsqrt(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}
__device__ __forceinline__ float fsqrt(float x) { return sqrtf(x); }

// FP64 natural logarithm and exponential for the thermodynamics (theta_v
// and the saturation vapour pressure), each within a few ulp of the
// correctly rounded result over the arguments the kernels pass.  The
// logarithm takes positive, finite, normal x = m 2^e with m in
// [1/sqrt2, sqrt2) and sums ln m = 2 atanh(s), s = (m-1)/(m+1), |s| <= 0.172,
// to the s^23 term; the exponential takes |y| < 700, reduces y = k ln2 + r,
// |r| <= ln2/2, and sums the Taylor series to the r^13 term.  No special
// cases: the arguments they see are far from the ends of the range.  The
// series coefficients come from a constant table (wave-uniform loads, kept
// in scalar registers) and enter as multiplicands of powers of the reduced
// argument, summed smallest first: a Horner step would need each
// coefficient as its vector addend, which the compiler copies into vector
// registers before every use.
static __constant__ double c_lnexp[24] = {
    // 1/(2n+1), n = 11 .. 1 (the last one is not read)
    1.0 / 23, 1.0 / 21, 1.0 / 19, 1.0 / 17, 1.0 / 15, 1.0 / 13, 1.0 / 11, 1.0 / 9, 1.0 / 7, 1.0 / 5, 1.0 / 3,
    // 1/n!, n = 13 .. 2
    1.0 / 6227020800.0, 1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0, 1.0 / 362880.0, 1.0 / 40320.0,
    1.0 / 5040.0, 1.0 / 720.0, 1.0 / 120.0, 1.0 / 24.0, 1.0 / 6.0, 0.5,
    0.0};
constexpr double LN2_HI = 6.93147180369123816490e-01, LN2_LO = 1.90821492927058770002e-10;

__device__ __forceinline__ double ln_pos(double x)
{
    int e;
    double m = frexp(x, &e);  // [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    // with f = m - 1 (exact) and s = f/(2+f): 2s = f - s f and
    // s f = (f^2/2)(1 - s), so ln m = 2s (1 + s^2 p) = f - (f^2/2 - s (f^2/2 + 2 s^2 p)):
    // the exact f carries the result, and the rounding of s enters only a
    // term about s^2 times smaller
    const double f = m - 1.0;
    const double sv = f * frcp(2.0 + f);
    const double s2 = sv * sv;
    // p = sum over n = 1 .. 11 of s2^(n-1) / (2n+1)
    double pw[10];
    pw[0] = s2;
#pragma unroll
    for (int n = 1; n < 10; ++n) pw[n] = pw[n - 1] * s2;
    double p = c_lnexp[0] * pw[9];
#pragma unroll
    for (int n = 1; n < 10; ++n) p = fma(c_lnexp[n], pw[9 - n], p);
    p = p + 1.0 / 3;
    const double hf = 0.5 * f * f;
    const double ek = (double)e;
    return fma(ek, LN2_HI, f - (hf - fma(sv, fma(2.0 * s2, p, hf), ek * LN2_LO)));
}

__device__ __forceinline__ double exp_fin(double y)
{
    const double k = rint(y * 1.44269504088896340736);
    double r = fma(-k, LN2_HI, y);
    r = fma(-k, LN2_LO, r);
    // exp(r) = 1 + r + sum over n = 2 .. 13 of r^n / n!
    double pr[13];
    pr[0] = r;
#pragma unroll
    for (int n = 1; n < 13; ++n) pr[n] = pr[n - 1] * r;
    double q = c_lnexp[11] * pr[12];
#pragma unroll
    for (int n = 12; n < 23; ++n) q = fma(c_lnexp[n], pr[23 - n], q);
    q = (q + r) + 1.0;
    return ldexp(q, (int)k);
}

#endif  // CM_LIBM_THERMO

}  // namespace cm
