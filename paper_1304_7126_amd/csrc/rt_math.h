// rt_math.h -- natural logarithms in FP64 for the App. E rate coefficients.
//
// Every attempt of the thermochemistry (App. A) evaluates four ln T and
// five ln(1 + u) of the Hui & Gnedin fits (App. E.2, E.3); the library
// routines carry extended-precision intermediates that cost about twice the
// instructions of the methods below, which stay within about 1.2 ulp (ln)
// and 1.5 ulp (ln(1 + u)) of the exact values, far inside what the
// subcycled solver needs.
//
//   ln x: x = 2^e m with m in [sqrt(1/2), sqrt(2)); with f = m - 1 (exact)
//   and s = f / (m + 1), ln m = 2 atanh(s) = 2s + 2s^3/3 + 2s^5/5 + ...,
//   |s| <= 3 - 2 sqrt(2), so the odd series to s^21 leaves a truncation
//   below 2^-55 relative.  Since 2s = f - s f, ln m = f - s (f - 2 z q(z))
//   with z = s^2 and q(z) = 1/3 + z/5 + ... + z^9/21: the rounding of s then
//   enters only through the small term s (...).  q is nested as
//   (1/3)(1 + (3/5) z (1 + (5/7) z (1 + ...))): every addend is 1, an inline
//   operand, and the ratios multiply z from scalar registers, where the
//   compiler rematerialises them instead of holding ten FP64 constants in
//   vector registers across the subcycling loop.  ln x = e ln 2 + ln m with
//   ln 2 split into a 32-bit head and its remainder.
//   ln(1 + u): w = 1 + u rounded, c = u - (w - 1) its rounding error (exact
//   for u >= 0), ln(1 + u) = ln w + c / w to first order in c, with 1/w
//   from the reduced mantissa (no second division).
//
// Written with explicit fma() and no other multiply feeding an add, so the
// same source gives the same bits compiled for the host (where its accuracy
// is tested against extended precision) and for the device.
#pragma once
#include <math.h>

namespace rtm1 {

constexpr double RM_LN2_HI = 6.93147180369123816490e-01;  // ln 2 to 32 significant bits
constexpr double RM_LN2_LO = 1.90821492927058770002e-10;  // ln 2 - RM_LN2_HI
constexpr double RM_SQRT_HALF = 0.70710678118654752440;

// ln x for finite x > 0; also returns the reduced mantissa's f = m - 1 and
// the exponent e
__host__ __device__ __forceinline__ double log_core(double x, double &f, int &e)
{
    double m = frexp(x, &e);  // m in [1/2, 1)
    const bool lo = m < RM_SQRT_HALF;
    m = lo ? m + m : m;
    e = lo ? e - 1 : e;
    f = m - 1.0;
    const double s = f / (m + 1.0);
    const double z = s * s;
    // t = 3 q(z)
    double t = fma(19.0 / 21.0 * z, 1.0, 1.0);
    t = fma(17.0 / 19.0 * z, t, 1.0);
    t = fma(15.0 / 17.0 * z, t, 1.0);
    t = fma(13.0 / 15.0 * z, t, 1.0);
    t = fma(11.0 / 13.0 * z, t, 1.0);
    t = fma(9.0 / 11.0 * z, t, 1.0);
    t = fma(7.0 / 9.0 * z, t, 1.0);
    t = fma(5.0 / 7.0 * z, t, 1.0);
    t = fma(3.0 / 5.0 * z, t, 1.0);
    const double d = fma(-2.0 / 3.0 * z, t, f);
    const double lnm = fma(-s, d, f);
    const double ef = (double)e;
    return fma(ef, RM_LN2_HI, fma(ef, RM_LN2_LO, lnm));
}

__host__ __device__ __forceinline__ double rt_log(double x)
{
    double f;
    int e;
    const double y = log_core(x, f, e);
    // zero, negative, infinite and NaN arguments as the library log
    return x > 0.0 && x < INFINITY ? y : (x == 0.0 ? -INFINITY : (x > 0.0 ? x : NAN));
}

// ln(1 + u) for u >= 0 (the fits' (lambda/lambda_0)^q), with the library's
// results for infinity and NaN; u < 0 is outside its domain (a further
// select for it pushed the chemistry kernels past their register budget).
// The correction c / w = c 2^-e / m takes 1/m as 1 - f + f^2, within 5% on
// the reduced range: c is below half an ulp of w, so that costs under 0.05
// ulp.
__host__ __device__ __forceinline__ double rt_log1p(double u)
{
    const double w = 1.0 + u;
    const double c = u - (w - 1.0);
    double f;
    int e;
    const double y = log_core(w, f, e);
    const double yc = fma(ldexp(c, -e), fma(f, f, 1.0 - f), y);
    return w == 1.0 ? u : (w < INFINITY ? yc : w);
}

}  // namespace rtm1
