// kx_math.h -- FP64 elementary functions for the gfx950 kernels.
//
// gfx950 has no FP64 exponential or logarithm instruction, so these are
// software sequences.  They assume finite arguments (inputs are checked by the
// preconditions of the entry points), which removes the special-case
// handling of a general-purpose libm:
//
//  kexp(x):  Cody-Waite reduction x = n ln2 + r (two-part ln 2), |r| <= ln2/2,
//            then the degree-13 Taylor polynomial of e^r (truncation error
//            below 5e-18 relative on that interval) and a scale by 2^n.
//  krcp(d):  v_rcp_f64 (about 24 correct bits on gfx950) followed by two
//            Newton-Raphson steps r <- r + r (1 - d r).
//  krsqrt(x): v_rsq_f64 followed by two Newton steps r <- r (3 - x r^2) / 2.
//  kln(x):   x = 2^e m with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),
//            s = (m - 1) / (m + 1), |s| <= 0.1716, from the odd series
//            2 (s + s^3/3 + ... + s^21/21) (truncation below 1e-18 relative),
//            plus e ln 2 with ln 2 in two parts.  Positive normal x only.
//
// The polynomial steps are written as VOP3 v_fma_f64 whose constant operand is
// a scalar register pair: the coefficients then live in SGPRs (materialised by
// cheap scalar moves) instead of occupying vector registers for the whole
// kernel, and the two-address v_fmac form's per-use copies are avoided.
#pragma once

#include <hip/hip_runtime.h>

namespace kx {

// a * b + c with a wave-uniform addend c read straight from scalar registers.
__device__ __forceinline__ double fma_s(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

__device__ __forceinline__ float fmaf_s(float a, float b, float c)
{
    float d;
    asm("v_fma_f32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

__device__ __forceinline__ double kexp(double x)
{
    const double n = __builtin_rint(x * 1.4426950408889634074);
    double r = __builtin_fma(-n, 6.93147180559945286227e-01, x);
    r = __builtin_fma(-n, 2.31904681384629955842e-17, r);
    double p = 1.0 / 6227020800.0;      // 1/13!
    p = fma_s(p, r, 1.0 / 479001600.0);  // 1/12!
    p = fma_s(p, r, 1.0 / 39916800.0);
    p = fma_s(p, r, 1.0 / 3628800.0);
    p = fma_s(p, r, 1.0 / 362880.0);
    p = fma_s(p, r, 1.0 / 40320.0);
    p = fma_s(p, r, 1.0 / 5040.0);
    p = fma_s(p, r, 1.0 / 720.0);
    p = fma_s(p, r, 1.0 / 120.0);
    p = fma_s(p, r, 1.0 / 24.0);
    p = fma_s(p, r, 1.0 / 6.0);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_ldexp(p, (int)n);
}

__device__ __forceinline__ double krcp(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// One Newton step only: about 2^-48 relative error (v_rcp_f64's ~2^-24
// squared), used where the result feeds a sum of positive terms.
__device__ __forceinline__ double krcp1(double d)
{
    const double r = __builtin_amdgcn_rcp(d);
    return __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
}

__device__ __forceinline__ double kln(double x)
{
    int e;
    double m = __builtin_frexp(x, &e);  // m in [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double f = m - 1.0;  // exact
    const double s = f * krcp(m + 1.0);
    const double z = s * s;
    double q = 1.0 / 21.0;
    q = fma_s(q, z, 1.0 / 19.0);
    q = fma_s(q, z, 1.0 / 17.0);
    q = fma_s(q, z, 1.0 / 15.0);
    q = fma_s(q, z, 1.0 / 13.0);
    q = fma_s(q, z, 1.0 / 11.0);
    q = fma_s(q, z, 1.0 / 9.0);
    q = fma_s(q, z, 1.0 / 7.0);
    q = fma_s(q, z, 1.0 / 5.0);
    q = __builtin_fma(q, z, 1.0 / 3.0);
    const double s2 = s + s;
    const double lnm = __builtin_fma(s2 * z, q, s2);
    const double de = (double)e;
    return __builtin_fma(de, 6.93147180559945286227e-01,
                         __builtin_fma(de, 2.31904681384629955842e-17, lnm));
}

__device__ __forceinline__ double krsqrt(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    r = r * __builtin_fma(-h * r, r, 1.5);
    return r * __builtin_fma(-h * r, r, 1.5);
}

}  // namespace kx
