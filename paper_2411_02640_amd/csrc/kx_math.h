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
//
// The polynomial steps are written as VOP3 v_fma_f64 so that the compiler keeps
// each coefficient in a register that is never overwritten (the two-address
// v_fmac form otherwise copies every coefficient before each use).
#pragma once

#include <hip/hip_runtime.h>

namespace kx {

__device__ __forceinline__ double fma3(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

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
    p = fma3(p, r, 1.0 / 479001600.0);  // 1/12!
    p = fma3(p, r, 1.0 / 39916800.0);
    p = fma3(p, r, 1.0 / 3628800.0);
    p = fma3(p, r, 1.0 / 362880.0);
    p = fma3(p, r, 1.0 / 40320.0);
    p = fma3(p, r, 1.0 / 5040.0);
    p = fma3(p, r, 1.0 / 720.0);
    p = fma3(p, r, 1.0 / 120.0);
    p = fma3(p, r, 1.0 / 24.0);
    p = fma3(p, r, 1.0 / 6.0);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_ldexp(p, (int)n);
}

// 10^x = e^(x ln 10) with ln 10 split in two parts.
__device__ __forceinline__ double kexp10(double x)
{
    const double hi = x * 2.30258509299404568402;
    const double lo = __builtin_fma(x, 2.30258509299404568402, -hi) +
                      x * -2.17075622338224935e-16;
    return kexp(hi) * (1.0 + lo);
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

__device__ __forceinline__ double krsqrt(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    r = r * __builtin_fma(-h * r, r, 1.5);
    return r * __builtin_fma(-h * r, r, 1.5);
}

}  // namespace kx
