// FP64 exponential and logarithm for the chemistry's rate fits.
//
// The network coefficients take 27 exponentials and logarithms per
// substep; the general library routines handle every special case of the
// IEEE formats at several times the cost of the finite, positive arguments
// that occur here.  These follow the classical reduction methods (Cody &
// Waite 1980; Tang 1989, 1990):
//   exp(x) = 2^n exp(r), n = rint(x / ln 2), r = x - n ln 2 with ln 2 split
//            into a short and a long part, |r| <= ln(2)/2, and exp(r) from
//            its Taylor series to degree 13 (truncation < 2e-16);
//   log(x) = e ln 2 + 2 atanh(s), x = m 2^e with m in [sqrt(1/2), sqrt(2)),
//            s = (m - 1)/(m + 1), |s| <= 0.1716, and atanh from its series
//            to s^23 (truncation < 1e-18).
// Both are accurate to a few units in the last place on their domain
// (checked against the C library over the ranges the rates use).
// Arguments: rt_exp any finite x (underflows to 0 below -745.2, overflows
// above 709.78); rt_log finite x > 0.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace rtk {

__host__ __device__ inline double rt_exp(double x) {
    if (x > 709.782712893384) return HUGE_VAL;
    if (x < -745.2) return 0.0;
    constexpr double kLog2e = 1.4426950408889634074;
    constexpr double kLn2Hi = 6.93147180369123816490e-01;   // 32 leading bits of ln 2
    constexpr double kLn2Lo = 1.90821492927058770002e-10;   // ln 2 - kLn2Hi
    const double n = rint(x * kLog2e);
    const double r = fma(-n, kLn2Lo, fma(-n, kLn2Hi, x));
    // sum_{k=0}^{13} r^k / k!  (Horner)
    double p = 1.0 / 6227020800.0;                 // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);              // 1/12!
    p = fma(p, r, 1.0 / 39916800.0);               // 1/11!
    p = fma(p, r, 1.0 / 3628800.0);                // 1/10!
    p = fma(p, r, 1.0 / 362880.0);                 // 1/9!
    p = fma(p, r, 1.0 / 40320.0);                  // 1/8!
    p = fma(p, r, 1.0 / 5040.0);                   // 1/7!
    p = fma(p, r, 1.0 / 720.0);                    // 1/6!
    p = fma(p, r, 1.0 / 120.0);                    // 1/5!
    p = fma(p, r, 1.0 / 24.0);                     // 1/4!
    p = fma(p, r, 1.0 / 6.0);                      // 1/3!
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}

__host__ __device__ inline double rt_log(double x) {
    constexpr double kSqrtHalf = 0.70710678118654752440;
    constexpr double kLn2Hi = 6.93147180369123816490e-01;
    constexpr double kLn2Lo = 1.90821492927058770002e-10;
    int e;
    double m = frexp(x, &e);                        // x = m 2^e, m in [1/2, 1)
    if (m < kSqrtHalf) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    // 2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ... + s^22/23)
    double q = 1.0 / 23.0;
    q = fma(q, s2, 1.0 / 21.0);
    q = fma(q, s2, 1.0 / 19.0);
    q = fma(q, s2, 1.0 / 17.0);
    q = fma(q, s2, 1.0 / 15.0);
    q = fma(q, s2, 1.0 / 13.0);
    q = fma(q, s2, 1.0 / 11.0);
    q = fma(q, s2, 1.0 / 9.0);
    q = fma(q, s2, 1.0 / 7.0);
    q = fma(q, s2, 1.0 / 5.0);
    q = fma(q, s2, 1.0 / 3.0);
    const double lnm = fma(2.0 * s * s2, q, 2.0 * s);  // 2 s + 2 s^3 q
    const double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, lnm));
}

}  // namespace rtk
