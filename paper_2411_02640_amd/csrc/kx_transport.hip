// kx_transport.hip -- mixture-averaged transport and mixture thermo on gfx950.
//
// One grid point per lane.  Every mechanism constant is wave-uniform, so the
// compiler keeps it in scalar registers (one scalar load serves 64 points).
// The quadratic sums run over a block of kKB species k held in registers
// while j streams over all species; X_j is recomputed from Y_j (a coalesced,
// L2-resident re-read) instead of being held per lane.
//
//  * pure species (App. A.3 "Polynomial fits"): eta_k, lambda_k, D_kj as
//    polynomials in u = (ln T - L0)/h (Horner), D_kj divided by p/p_atm;
//  * Wilke / Bird viscosity with the squared bracket expanded:
//      sum_j X_j phi_kj = sum_j c1 X_j + 2 s_k sum_j c1 c2 X_j r_j
//                         + s_k^2 sum_j c1 c2^2 X_j r_j^2,
//    s_k = sqrt(eta_k), r_j = 1/sqrt(eta_j), c1 = (8 (1 + W_k/W_j))^(-1/2),
//    c2 = (W_j/W_k)^(1/4) -- three FMAs per pair, all terms positive;
//  * Mathur conductivity; eq:mix_diff for D_km with the full (k, j) matrix
//    evaluated (no symmetric reuse, so nothing but kKB accumulators is live).
#include <float.h>

#include "kx_internal.h"
#include "kx_math.h"

namespace kx {
namespace {

constexpr int kBlock = 256;

// Horner evaluation of a wave-uniform polynomial (coefficients in scalar
// registers, constant term first) at a per-lane point.
__device__ __forceinline__ double fma_u(double a, double b, double c) { return fma_s(a, b, c); }
__device__ __forceinline__ float fma_u(float a, float b, float c) { return fmaf_s(a, b, c); }

template <int ORDER, class F>
__device__ __forceinline__ F horner(const F *__restrict__ c, F u, int order)
{
    if (ORDER > 1) {
        F r = u * c[ORDER - 1] + c[ORDER - 2];
#pragma unroll
        for (int o = ORDER - 3; o >= 0; --o) r = fma_u(r, u, c[o]);
        return r;
    }
    if (ORDER == 1) return c[0];
    F r = c[order - 1];
    for (int o = order - 2; o >= 0; --o) r = fma_u(r, u, c[o]);
    return r;
}

// FP64 path.  KIND is the diffusion fit kind (0: D_kj, 1: 1/D_kj).
template <int ORDER, int KIND>
__global__ __launch_bounds__(kBlock) void transport_f64(MechDev m, int64_t n,
                                                        const double *__restrict__ T,
                                                        const double *__restrict__ P,
                                                        const double *__restrict__ Y,
                                                        double *__restrict__ mu,
                                                        double *__restrict__ lam,
                                                        double *__restrict__ Dmix)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int ns = m.ns, order = m.fit_order;
    const double Ti = T[i], pi = P[i];
    const double u = (log(Ti) - m.fit_L0) * m.inv_fit_h;
    const double pr = pi / kPatm;
    const double *Yi = Y + i;

    double sYW = 0.0;
    for (int k = 0; k < ns; ++k) sYW += Yi[(int64_t)k * n] * m.sp[k].inv_W;
    const double xf = 1.0 / sYW;  // X_k = Y_k / W_k * xf

    double s1 = 0.0, s2 = 0.0, wbar = 0.0;
    for (int k = 0; k < ns; ++k) {
        const double X = Yi[(int64_t)k * n] * m.sp[k].inv_W * xf;
        const double lk = horner<ORDER>(m.cond + k * order, u, order);
        s1 = fma(X, lk, s1);
        s2 = fma(X, krcp(lk), s2);
        wbar = fma(X, m.W[k], wbar);
    }
    lam[i] = 0.5 * (s1 + krcp(s2));

    const int nkb = (ns + kKB - 1) / kKB;
    double visc = 0.0;
    for (int kb = 0; kb < nkb; ++kb) {
        double S1[kKB], S2[kKB], S3[kKB];
#pragma unroll
        for (int kk = 0; kk < kKB; ++kk) S1[kk] = S2[kk] = S3[kk] = 0.0;
        const double *wl = m.wilke + (size_t)kb * ns * kKB * 3;
        double ynext = Yi[0];
        for (int j = 0; j < ns; ++j, wl += kKB * 3) {
            const double yj = ynext;
            if (j + 1 < ns) ynext = Yi[(int64_t)(j + 1) * n];
            const double Xj = yj * m.sp[j].inv_W * xf;
            const double rj = krsqrt(horner<ORDER>(m.visc + j * order, u, order));
            const double v = Xj * rj, w = v * rj;
#pragma unroll
            for (int kk = 0; kk < kKB; ++kk) {
                S1[kk] = fma(wl[3 * kk + 0], Xj, S1[kk]);
                S2[kk] = fma(wl[3 * kk + 1], v, S2[kk]);
                S3[kk] = fma(wl[3 * kk + 2], w, S3[kk]);
            }
        }
#pragma unroll
        for (int kk = 0; kk < kKB; ++kk) {
            const int k = kb * kKB + kk;
            if (k < ns) {
                const double ek = horner<ORDER>(m.visc + k * order, u, order);
                const double sk = ek * krsqrt(ek);
                const double den = fma(ek, S3[kk], fma(2.0 * sk, S2[kk], S1[kk]));
                const double Xk = Yi[(int64_t)k * n] * m.sp[k].inv_W * xf;
                visc = fma(Xk * ek, krcp(den), visc);
            }
        }
    }
    mu[i] = visc;

    for (int kb = 0; kb < nkb; ++kb) {
        double acc[kKB];
#pragma unroll
        for (int kk = 0; kk < kKB; ++kk) acc[kk] = 0.0;
        const double *dfb = m.dfit + (size_t)kb * ns * kKB * order;
        // sum_{j != k} X_j / D_kj for the kKB species of this block.  Padding
        // rows (k >= ns) hold a fit identically 1; the j-range that contains
        // the block's own species masks the diagonal term.
        auto pairs = [&](int j0, int j1, bool diag) {
            double ynext = j0 < j1 ? Yi[(int64_t)j0 * n] : 0.0;
            for (int j = j0; j < j1; ++j) {
                const double yj = ynext;
                if (j + 1 < j1) ynext = Yi[(int64_t)(j + 1) * n];
                const double Xj = yj * m.sp[j].inv_W * xf;
                const double *df = dfb + (size_t)j * kKB * order;
#pragma unroll
                for (int kk = 0; kk < kKB; ++kk) {
                    const double f = horner<ORDER>(df + kk * order, u, order);
                    const double x = (diag && kb * kKB + kk == j) ? 0.0 : Xj;
                    acc[kk] = fma(x, KIND == 0 ? krcp(f) : f, acc[kk]);
                }
            }
        };
        const int jd0 = kb * kKB, jd1 = min(jd0 + kKB, ns);
        pairs(0, jd0, false);
        pairs(jd0, jd1, true);
        pairs(jd1, ns, false);
#pragma unroll
        for (int kk = 0; kk < kKB; ++kk) {
            const int k = kb * kKB + kk;
            if (k < ns) {
                const double Xk = Yi[(int64_t)k * n] * m.sp[k].inv_W * xf;
                double D;
                if (acc[kk] == 0.0) {
                    const double f = horner<ORDER>(m.ddiag + k * order, u, order);
                    D = (KIND == 0) ? f / pr : 1.0 / (f * pr);
                } else {
                    // sum_{j!=k} X_j / D_kj = (p/p_atm) acc for either fit kind
                    D = (wbar - Xk * m.W[k]) / (wbar * acc[kk] * pr);
                }
                Dmix[(int64_t)k * n + i] = D;
            }
        }
    }
}

// Mixed path: fits and mixing sums in FP32 with FP32 accumulation; the
// D_km numerator (W-bar - X_k W_k)/W-bar in FP64.
template <int ORDER>
__global__ __launch_bounds__(kBlock) void transport_mixed(MechDev m, int64_t n,
                                                          const double *__restrict__ T,
                                                          const double *__restrict__ P,
                                                          const double *__restrict__ Y,
                                                          double *__restrict__ mu,
                                                          double *__restrict__ lam,
                                                          double *__restrict__ Dmix)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int ns = m.ns, order = m.fit_order;
    const double Ti = T[i], pi = P[i];
    const float u = (float)((log(Ti) - m.fit_L0) * m.inv_fit_h);
    const float pr = (float)(pi / kPatm);
    const double *Yi = Y + i;

    double sYW = 0.0;
    for (int k = 0; k < ns; ++k) sYW += Yi[(int64_t)k * n] * m.sp[k].inv_W;
    const double xf = 1.0 / sYW;

    float s1 = 0.0f, s2 = 0.0f;
    double wbar = 0.0;
    for (int k = 0; k < ns; ++k) {
        const double Xd = Yi[(int64_t)k * n] * m.sp[k].inv_W * xf;
        const float X = (float)Xd;
        const float lk = horner<ORDER>(m.cond32 + k * order, u, order);
        s1 = fmaf(X, lk, s1);
        s2 += __fdividef(X, lk);
        wbar += Xd * m.W[k];
    }
    lam[i] = (double)(0.5f * (s1 + 1.0f / s2));

    const int nkb = (ns + kKB - 1) / kKB;
    float visc = 0.0f;
    for (int kb = 0; kb < nkb; ++kb) {
        float S1[kKB], S2[kKB], S3[kKB];
#pragma unroll
        for (int kk = 0; kk < kKB; ++kk) S1[kk] = S2[kk] = S3[kk] = 0.0f;
        const float *wl = m.wilke32 + (size_t)kb * ns * kKB * 3;
        double ynext = Yi[0];
        for (int j = 0; j < ns; ++j, wl += kKB * 3) {
            const double yj = ynext;
            if (j + 1 < ns) ynext = Yi[(int64_t)(j + 1) * n];
            const float Xj = (float)(yj * m.sp[j].inv_W * xf);
            const float rj = rsqrtf(horner<ORDER>(m.visc32 + j * order, u, order));
            const float v = Xj * rj, w = v * rj;
#pragma unroll
            for (int kk = 0; kk < kKB; ++kk) {
                S1[kk] = fmaf(wl[3 * kk + 0], Xj, S1[kk]);
                S2[kk] = fmaf(wl[3 * kk + 1], v, S2[kk]);
                S3[kk] = fmaf(wl[3 * kk + 2], w, S3[kk]);
            }
        }
#pragma unroll
        for (int kk = 0; kk < kKB; ++kk) {
            const int k = kb * kKB + kk;
            if (k < ns) {
                const float ek = horner<ORDER>(m.visc32 + k * order, u, order);
                const float sk = sqrtf(ek);
                const float den = fmaf(sk * sk, S3[kk], fmaf(2.0f * sk, S2[kk], S1[kk]));
                const float Xk = (float)(Yi[(int64_t)k * n] * m.sp[k].inv_W * xf);
                visc += __fdividef(Xk * ek, den);
            }
        }
    }
    mu[i] = (double)visc;

    for (int kb = 0; kb < nkb; ++kb) {
        float acc[kKB];
#pragma unroll
        for (int kk = 0; kk < kKB; ++kk) acc[kk] = 0.0f;
        const float *df = m.dfit32 + (size_t)kb * ns * kKB * order;
        double ynext = Yi[0];
        for (int j = 0; j < ns; ++j, df += kKB * order) {
            const double yj = ynext;
            if (j + 1 < ns) ynext = Yi[(int64_t)(j + 1) * n];
            const float Xj = (float)(yj * m.sp[j].inv_W * xf);
#pragma unroll
            for (int kk = 0; kk < kKB; ++kk) {
                const int k = kb * kKB + kk;
                if (k < ns && k != j) {
                    const float f = horner<ORDER>(df + kk * order, u, order);
                    acc[kk] += (m.diff_kind == 0) ? __fdividef(Xj, f) : Xj * f;
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < kKB; ++kk) {
            const int k = kb * kKB + kk;
            if (k < ns) {
                const double Xk = Yi[(int64_t)k * n] * m.sp[k].inv_W * xf;
                double D;
                if (acc[kk] == 0.0f) {
                    const float f = horner<ORDER>(m.ddiag32 + k * order, u, order);
                    D = (m.diff_kind == 0) ? (double)(f / pr) : (double)(1.0f / (f * pr));
                } else {
                    const double num = (wbar - Xk * m.W[k]) / wbar;
                    D = num / (double)(acc[kk] * pr);
                }
                Dmix[(int64_t)k * n + i] = D;
            }
        }
    }
}

// Mixture thermo (App. A.1): cp_k = Cp_k/W_k, h_k = H_k/W_k, cp = sum Y_k cp_k.
__global__ __launch_bounds__(kBlock) void thermo_kernel(MechDev m, int64_t n,
                                                        const double *__restrict__ T,
                                                        const double *__restrict__ Y,
                                                        double *__restrict__ cpk,
                                                        double *__restrict__ hk,
                                                        double *__restrict__ cpmix)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double Ti = T[i], invT = 1.0 / Ti;
    double cp = 0.0;
    for (int k = 0; k < m.ns; ++k) {
        const DevSpecies &S = m.sp[k];
        const double *a = (Ti < S.t_mid) ? S.nasa_lo : S.nasa_hi;
        const double cpr = fma(Ti, fma(Ti, fma(Ti, fma(Ti, a[4], a[3]), a[2]), a[1]), a[0]);
        const double c = cpr * kRu * S.inv_W;
        if (cpk) cpk[(int64_t)k * n + i] = c;
        if (hk) {
            const double hrt =
                fma(Ti, fma(Ti, fma(Ti, fma(Ti, a[4] * 0.2, a[3] * 0.25), a[2] * (1.0 / 3.0)),
                            a[1] * 0.5),
                    a[0]) +
                a[5] * invT;
            hk[(int64_t)k * n + i] = hrt * kRu * Ti * S.inv_W;
        }
        cp = fma(Y[(int64_t)k * n + i], c, cp);
    }
    if (cpmix) cpmix[i] = cp;
}

}  // namespace

kx_status launch_transport(const kx_mech *mech, int64_t n, const double *T, const double *p,
                           const double *Y, double *mu, double *lam, double *Dmix,
                           int precision, hipStream_t s)
{
    const MechDev &m = mech->dev;
    const int64_t nblk = (n + kBlock - 1) / kBlock;
    if (nblk > 0x7fffffff) return fail(KX_EINVAL, "transport: n too large");
    const bool o5 = m.fit_order == 5;
    if (precision == KX_MIXED) {
        auto k = o5 ? transport_mixed<5> : transport_mixed<0>;
        hipLaunchKernelGGL(k, dim3((unsigned)nblk), dim3(kBlock), 0, s, m, n, T, p, Y, mu,
                           lam, Dmix);
    } else {
        auto k = m.diff_kind == 0 ? (o5 ? transport_f64<5, 0> : transport_f64<0, 0>)
                                  : (o5 ? transport_f64<5, 1> : transport_f64<0, 1>);
        hipLaunchKernelGGL(k, dim3((unsigned)nblk), dim3(kBlock), 0, s, m, n, T, p, Y, mu,
                           lam, Dmix);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "transport kernel launch");
    return ok();
}

kx_status launch_thermo(const kx_mech *mech, int64_t n, const double *T, const double *Y,
                        double *cpk, double *hk, double *cpmix, hipStream_t s)
{
    const int64_t nblk = (n + kBlock - 1) / kBlock;
    if (nblk > 0x7fffffff) return fail(KX_EINVAL, "thermo: n too large");
    hipLaunchKernelGGL(thermo_kernel, dim3((unsigned)nblk), dim3(kBlock), 0, s, mech->dev, n,
                       T, Y, cpk, hk, cpmix);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "thermo kernel launch");
    return ok();
}

}  // namespace kx
