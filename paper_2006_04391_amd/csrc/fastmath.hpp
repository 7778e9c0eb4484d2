// fastmath.hpp -- FP64 reciprocal, reciprocal square root, log and exp for
// the hot path, accurate to a few units in the last place (not correctly
// rounded). The material-point solve needs its transcendental results to
// about 1e-14 relative, far inside the 1e-10 parity bar, but calls them in
// every Newton residual, so the general-purpose library sequences (which
// also handle every special case and round correctly) dominate the
// instruction count.
//
// Methods (textbook, written from the mathematics):
//  * rcp / rsqrt: the hardware estimate (v_rcp_f64 / v_rsq_f64, relative
//    error below 2^-22) refined by one third-order step: with e = 1 - x r
//    (rcp) or e = 1 - x r^2 (rsqrt), 1/x = r / (1 - e) = r (1 + e + e^2 + ...)
//    and 1/sqrt(x) = r (1 - e)^(-1/2) = r (1 + e/2 + 3e^2/8 + ...), each
//    truncated after e^2 (truncation below 2^-64); three dependent
//    operations after the estimate instead of the four to six of two
//    Newton-Raphson steps;
//  * log: x = 2^k m with m in [sqrt(1/2), sqrt(2)), s = (m - 1)/(m + 1),
//    log m = 2 atanh s = 2 (s + s^3/3 + s^5/5 + ...) summed to s^23
//    (|s| <= 0.1716, truncation < 1e-17), log x = k ln2 + log m with ln2
//    split in a high and a low part;
//  * exp: x = k ln2 + r, k = rint(x / ln2), |r| <= ln2/2, exp r by its
//    Taylor series to r^13 (truncation < 5e-18), scaled by 2^k.
// Domain: rcp, rsqrt for finite x > 0; log for finite x > 0 (subnormal x
// handled by a pre-scale); exp for any x (underflow to 0, overflow to inf);
// pow_pos for finite x > 0.
// Host and device run the same refinement and polynomial code; only the
// initial estimate of rcp / rsqrt differs (hardware on the device, a
// single-precision estimate on the host), which the refinement removes to
// within an ulp.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#ifndef AD_FN
#define AD_FN __host__ __device__ __forceinline__
#endif

namespace automat {
namespace fm {

// Polynomial coefficients and reduction constants live in a small table in
// the constant address space rather than in the instruction stream: the
// compiler cannot fold them (the table is externally initialised), so it
// reads them with uniform scalar loads into scalar registers instead of
// materializing every constant in vector registers. Scalar loads also stay
// out of the vector-memory counter, so the math never waits on outstanding
// field loads or stores.
#ifndef AUTOMAT_FM_TABLE_SPACE
#define AUTOMAT_FM_TABLE_SPACE __constant__
#endif
#if defined(__HIP_DEVICE_COMPILE__)
#define AUTOMAT_FM_TABLE static AUTOMAT_FM_TABLE_SPACE
#else
#define AUTOMAT_FM_TABLE static
#endif
// [0..10] 1/23, 1/21, ..., 1/3 (log series); [11..24] 1/13!, ..., 1/1!, 1
// (exp series); [25] ln2 high part, [26] ln2 low part, [27] 1/ln2,
// [28] sqrt(1/2)
AUTOMAT_FM_TABLE double fm_tab[29] = {
    1.0 / 23.0, 1.0 / 21.0, 1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0, 1.0 / 11.0,
    1.0 / 9.0, 1.0 / 7.0, 1.0 / 5.0, 1.0 / 3.0,
    1.0 / 6227020800.0, 1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0,
    1.0 / 362880.0, 1.0 / 40320.0, 1.0 / 5040.0, 1.0 / 720.0, 1.0 / 120.0, 1.0 / 24.0,
    1.0 / 6.0, 0.5, 1.0, 1.0,
    0x1.62e42fefa3800p-1, 0x1.ef35793c76730p-45, 1.4426950408889634074,
    0.70710678118654752440};

AD_FN double rcp_estimate(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcp(x);
#else
    int k;
    const double m = ::frexp(x, &k);  // keep the float estimate in range
    return ::ldexp((double)(1.0f / (float)m), -k);
#endif
}

AD_FN double rsq_estimate(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsq(x);
#else
    int k;
    double m = ::frexp(x, &k);
    if (k & 1) {
        m *= 2.0;
        k -= 1;
    }
    return ::ldexp((double)(1.0f / ::sqrtf((float)m)), -k / 2);
#endif
}

// 1 / x for finite x != 0
AD_FN double rcp(double x) {
    const double r = rcp_estimate(x);
    const double e = ::fma(-x, r, 1.0);
    return ::fma(r, ::fma(e, e, e), r);
}

// 1 / sqrt(x) for finite x > 0
AD_FN double rsqrt(double x) {
    const double r = rsq_estimate(x);
    const double e = ::fma(-x, r * r, 1.0);
    return ::fma(r * e, ::fma(0.375, e, 0.5), r);
}

#if defined(__HIP_DEVICE_COMPILE__)
typedef __attribute__((address_space(4))) const double tab_t;
// a fresh (opaque) pointer to the table at every call: the compiler cannot
// hoist the coefficient loads out of the Newton loop and keep them in
// scalar registers across it; they are reloaded (scalar cache) where used
AD_FN tab_t *table() {
    tab_t *T = (tab_t *)fm_tab;
    asm volatile("" : "+s"(T));
    return T;
}
#else
AD_FN const double *table() { return fm_tab; }
#endif

// natural logarithm for finite x > 0
AD_FN double log(double x) {
    const auto *T = table();
    const bool tiny = x < 0x1p-1000;
    if (tiny) x *= 0x1p+200;
    int k;
    double m = ::frexp(x, &k);            // x = m 2^k, m in [0.5, 1)
    if (m < T[28]) {                      // move m to [sqrt(1/2), sqrt(2))
        m *= 2.0;
        k -= 1;
    }
    const double s = (m - 1.0) * rcp(m + 1.0);
    const double z = s * s;
    // 2 atanh(s) = 2 s (1 + z (1/3 + z/5 + ... + z^10/23)); the inner
    // polynomial by Estrin's scheme (dependency depth 5 instead of 10)
    const double z2 = z * z, z4 = z2 * z2, z8 = z4 * z4;
    const double q0 = ::fma(T[9], z, T[10]), q1 = ::fma(T[7], z, T[8]);
    const double q2 = ::fma(T[5], z, T[6]), q3 = ::fma(T[3], z, T[4]);
    const double q4 = ::fma(T[1], z, T[2]);
    const double s0 = ::fma(q1, z2, q0), s1 = ::fma(q3, z2, q2), s2 = ::fma(T[0], z2, q4);
    const double p = ::fma(s2, z8, ::fma(s1, z4, s0));
    const double lm = ::fma(2.0 * s * z, p, 2.0 * s);
    const double kd = (double)(tiny ? k - 200 : k);
    return ::fma(kd, T[25], ::fma(kd, T[26], lm));
}

// exponential
AD_FN double exp(double x) {
    const auto *T = table();
    if (x < -745.2) return 0.0;
    if (x > 709.8) return HUGE_VAL;
    const double kd = ::rint(x * T[27]);
    const double r = ::fma(-kd, T[26], ::fma(-kd, T[25], x));
    // Taylor series of e^r to r^13 by Estrin's scheme (coefficient of r^k
    // is T[24 - k]; dependency depth 5 instead of 13)
    const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
    const double q0 = ::fma(T[23], r, T[24]), q1 = ::fma(T[21], r, T[22]);
    const double q2 = ::fma(T[19], r, T[20]), q3 = ::fma(T[17], r, T[18]);
    const double q4 = ::fma(T[15], r, T[16]), q5 = ::fma(T[13], r, T[14]);
    const double q6 = ::fma(T[11], r, T[12]);
    const double s0 = ::fma(q1, r2, q0), s1 = ::fma(q3, r2, q2), s2 = ::fma(q5, r2, q4);
    const double t1 = ::fma(q6, r4, s2);
    const double p = ::fma(t1, r8, ::fma(s1, r4, s0));
    return ::ldexp(p, (int)kd);
}

// x^e for finite x > 0 as exp(e log x), for every exponent: the power-law
// exponent is a material parameter that is varied and differentiated, so no
// exponent takes a separate path.
AD_FN double pow_pos(double x, double e) { return exp(e * log(x)); }

}  // namespace fm
}  // namespace automat
