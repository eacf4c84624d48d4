// kx_transport.hip -- mixture-averaged transport and mixture thermo on gfx950.
//
// Each lane evaluates P grid points.  Every mechanism constant is
// wave-uniform, so it is read with scalar loads into scalar registers and used
// directly as an instruction operand; one fetched coefficient serves the P
// points of all 64 lanes.  The quadratic sums run over a block of KB species k
// held in registers while j streams over all species; X_j is recomputed from
// Y_j (a coalesced re-read) instead of being held per lane.
//
//  * pure species (App. A.3 "Polynomial fits"): eta_k, lambda_k, D_kj as
//    polynomials in u = (ln T - L0)/h (Horner), D_kj divided by p/p_atm;
//  * Wilke / Bird viscosity with phi_kj = c1_kj (1 + sigma_k rho_j)^2, where
//    c1_kj = (8 (1 + W_k/W_j))^(-1/2), sigma_k = sqrt(eta_k) / W_k^(1/4) and
//    rho_j = W_j^(1/4) / sqrt(eta_j): (W_j/W_k)^(1/4) separates into
//    per-species factors, so each pair reads one coefficient;
//  * Mathur conductivity; eq:mix_diff for D_km with the full (k, j) matrix
//    evaluated (no symmetric reuse, so only the KB accumulators are live),
//    1/D_kj by v_rcp_f64 and one Newton step (each term of this positive
//    sum then carries about 2^-48 relative error).
#include <float.h>

#include <type_traits>

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

// Mixture-averaged transport for P points per lane.  F is the arithmetic
// type of the fits and mixing sums (double: FP64 path; float: mixed path);
// KIND is the diffusion fit kind (0: D_kj, 1: 1/D_kj); KB species k are held
// in registers per step of the j loop, which serves the Wilke and the D_km
// sums together.  Every uniform coefficient fetched by a scalar load feeds
// P lanes' worth of arithmetic.
template <class F> __device__ __forceinline__ F rcp_fast(F x);
template <> __device__ __forceinline__ double rcp_fast<double>(double x) { return krcp1(x); }
template <> __device__ __forceinline__ float rcp_fast<float>(float x)
{
    return __builtin_amdgcn_rcpf(x);
}
template <class F> __device__ __forceinline__ F rsqrt_acc(F x);
template <> __device__ __forceinline__ double rsqrt_acc<double>(double x) { return krsqrt(x); }
template <> __device__ __forceinline__ float rsqrt_acc<float>(float x) { return rsqrtf(x); }
template <class F> __device__ __forceinline__ F rcp_acc(F x);
template <> __device__ __forceinline__ double rcp_acc<double>(double x) { return krcp(x); }
template <> __device__ __forceinline__ float rcp_acc<float>(float x) { return 1.0f / x; }

template <class F> struct Tabs;
template <> struct Tabs<double> {
    static __device__ const double *visc(const MechDev &m) { return m.visc; }
    static __device__ const double *cond(const MechDev &m) { return m.cond; }
    static __device__ const double *wq(const MechDev &m) { return m.wq; }
    static __device__ const double *wilke(const MechDev &m) { return m.wilke; }
    static __device__ const double *dfit(const MechDev &m) { return m.dfit; }
    static __device__ const double *ddiag(const MechDev &m) { return m.ddiag; }
};
template <> struct Tabs<float> {
    static __device__ const float *visc(const MechDev &m) { return m.visc32; }
    static __device__ const float *cond(const MechDev &m) { return m.cond32; }
    static __device__ const float *wq(const MechDev &m) { return m.wq32; }
    static __device__ const float *wilke(const MechDev &m) { return m.wilke32; }
    static __device__ const float *dfit(const MechDev &m) { return m.dfit32; }
    static __device__ const float *ddiag(const MechDev &m) { return m.ddiag32; }
};

// One tile of kBlock * P points starting at point `base` of arrays with n
// points (species rows of stride n).
template <class F, int ORDER, int KIND, int P, int KB>
__device__ __forceinline__ void transport_tile(const MechDev &m, int64_t n, int64_t base,
                                               const double *__restrict__ T,
                                               const double *__restrict__ Pp,
                                               const double *__restrict__ Y,
                                               double *__restrict__ mu,
                                               double *__restrict__ lam,
                                               double *__restrict__ Dmix)
{
    using Tb = Tabs<F>;
    const int ns = m.ns, order = m.fit_order;
    // point q of this lane: i[q] (clamped to n - 1 past the end; not stored)
    int64_t idx[P];
    bool act[P];
    F u[P];
    double pr[P], xf[P], wbar[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int64_t ir = base + threadIdx.x + (int64_t)kBlock * q;
        act[q] = ir < n;
        idx[q] = act[q] ? ir : n - 1;
        const double Ti = T[idx[q]];
        u[q] = (F)((log(Ti) - m.fit_L0) * m.inv_fit_h);
        pr[q] = Pp[idx[q]] / kPatm;
    }
    auto Yat = [&](int k, int q) { return Y[(int64_t)k * n + idx[q]]; };

    // X_k = (Y_k / W_k) xf; W-bar = sum_k X_k W_k; Mathur conductivity
    {
        double sYW[P];
#pragma unroll
        for (int q = 0; q < P; ++q) sYW[q] = 0.0;
        for (int k = 0; k < ns; ++k) {
            const double iw = m.sp[k].inv_W;
#pragma unroll
            for (int q = 0; q < P; ++q) sYW[q] = fma(Yat(k, q), iw, sYW[q]);
        }
        F s1[P], s2[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            xf[q] = 1.0 / sYW[q];
            wbar[q] = 0.0;
            s1[q] = s2[q] = (F)0;
        }
        for (int k = 0; k < ns; ++k) {
            const double iw = m.sp[k].inv_W, Wk = m.W[k];
            const F *cf = Tb::cond(m) + k * order;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const double X = Yat(k, q) * iw * xf[q];
                const F lk = horner<ORDER>(cf, u[q], order);
                s1[q] = fma((F)X, lk, s1[q]);
                s2[q] = fma((F)X, rcp_acc(lk), s2[q]);
                wbar[q] = fma(X, Wk, wbar[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < P; ++q)
            if (act[q]) lam[idx[q]] = (double)((F)0.5 * (s1[q] + rcp_acc(s2[q])));
    }

    F visc[P];
#pragma unroll
    for (int q = 0; q < P; ++q) visc[q] = (F)0;
    const int nkb = (ns + KB - 1) / KB;
    for (int kb = 0; kb < nkb; ++kb) {
        // table rows of this block inside the kKB-blocked tables
        const int tb = (kb * KB) / kKB, toff = (kb * KB) % kKB;
        F sig[P][KB], den[P][KB], acc[P][KB];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            const int k = kb * KB + kk;
            const bool valid = k < ns;
            const int kc = valid ? k : 0;
            const F wk = Tb::wq(m)[kc];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const F ek = horner<ORDER>(Tb::visc(m) + kc * order, u[q], order);
                // sigma_k = sqrt(eta_k) / W_k^(1/4)
                sig[q][kk] = valid ? ek * rsqrt_acc(ek) * rcp_acc(wk) : (F)0;
                den[q][kk] = acc[q][kk] = (F)0;
            }
        }
        const F *c1b = Tb::wilke(m) + (size_t)tb * ns * kKB + toff;
        const F *dfb = Tb::dfit(m) + ((size_t)tb * ns * kKB + toff) * order;
        auto steps = [&](int j0, int j1, bool diag) {
            for (int j = j0; j < j1; ++j) {
                const double iw = m.sp[j].inv_W;
                const F wj = Tb::wq(m)[j];
                const F *vj = Tb::visc(m) + j * order;
                F Xj[P], rho[P];
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    Xj[q] = (F)(Yat(j, q) * iw * xf[q]);
                    // rho_j = W_j^(1/4) / sqrt(eta_j)
                    rho[q] = wj * rsqrt_acc(horner<ORDER>(vj, u[q], order));
                }
                const F *c1 = c1b + (size_t)j * kKB;
                const F *df = dfb + (size_t)j * kKB * order;
#pragma unroll
                for (int kk = 0; kk < KB; ++kk) {
                    const F c = c1[kk];
                    const bool self = diag && kb * KB + kk == j;
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        // Wilke: X_j phi_kj = c1 X_j (1 + sigma_k rho_j)^2
                        const F t = fma(sig[q][kk], rho[q], (F)1);
                        const F xt = Xj[q] * t;
                        den[q][kk] = fma(c, xt * t, den[q][kk]);
                        // D_km: X_j / D_kj (j != k)
                        const F f = horner<ORDER>(df + kk * order, u[q], order);
                        const F x = self ? (F)0 : Xj[q];
                        acc[q][kk] = fma(x, KIND == 0 ? rcp_fast(f) : f, acc[q][kk]);
                    }
                }
            }
        };
        const int jd0 = kb * KB, jd1 = min(jd0 + KB, ns);
        steps(0, jd0, false);
        steps(jd0, jd1, true);
        steps(jd1, ns, false);
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            const int k = kb * KB + kk;
            if (k < ns) {
                const double iw = m.sp[k].inv_W, Wk = m.W[k];
                const F *ek_c = Tb::visc(m) + k * order;
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const double Xk = Yat(k, q) * iw * xf[q];
                    const F ek = horner<ORDER>(ek_c, u[q], order);
                    visc[q] = fma((F)Xk * ek, rcp_acc(den[q][kk]), visc[q]);
                    double D;
                    if (acc[q][kk] == (F)0) {
                        const F f = horner<ORDER>(Tb::ddiag(m) + k * order, u[q], order);
                        D = (KIND == 0) ? (double)f / pr[q] : 1.0 / ((double)f * pr[q]);
                    } else {
                        // sum_{j!=k} X_j / D_kj = (p/p_atm) acc for either fit kind;
                        // the numerator (W-bar - X_k W_k)/W-bar is formed in FP64
                        D = (wbar[q] - Xk * Wk) / (wbar[q] * (double)acc[q][kk] * pr[q]);
                    }
                    if (act[q]) Dmix[(int64_t)k * n + idx[q]] = D;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < P; ++q)
        if (act[q]) mu[idx[q]] = (double)visc[q];
}

template <class F, int ORDER, int KIND, int P, int KB>
__global__ __launch_bounds__(kBlock) void transport_kernel(MechDev m, int64_t n,
                                                           const double *__restrict__ T,
                                                           const double *__restrict__ Pp,
                                                           const double *__restrict__ Y,
                                                           double *__restrict__ mu,
                                                           double *__restrict__ lam,
                                                           double *__restrict__ Dmix)
{
    transport_tile<F, ORDER, KIND, P, KB>(m, n, (int64_t)blockIdx.x * kBlock * P, T, Pp, Y, mu,
                                          lam, Dmix);
}

// Batched requests (see rates_batch_kernel): tiles of kBlock * P points.
template <class F, int ORDER, int KIND, int P, int KB>
__global__ __launch_bounds__(kBlock) void transport_batch_kernel(MechDev m,
                                                                 const WorkList *__restrict__ wl,
                                                                 int *__restrict__ counter)
{
    __shared__ int tile;
    const int ntiles = wl->ntiles[1];
    for (;;) {
        if (threadIdx.x == 0) tile = atomicAdd(counter, 1);
        __syncthreads();
        const int t = tile;
        __syncthreads();
        if (t >= ntiles) break;
        int r = 0;
        while (r + 1 < wl->nitems && wl->start[1][r + 1] <= t) ++r;
        const WorkItem it = wl->items[r];
        transport_tile<F, ORDER, KIND, P, KB>(m, it.n,
                                              (int64_t)(t - wl->start[1][r]) * kBlock * P, it.T,
                                              it.p, it.Y, it.mu, it.lam, it.Dmix);
    }
}

__global__ void zero_kernel(int *p, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
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

// Points per lane and k-block size, measured on the 53-species workload:
// FP64 is bound by the scalar-coefficient stream, so four points share each
// fetched coefficient; the FP32 path carries half the registers per value and
// prefers wider k-blocks.
template <class F> struct TransportShape;
template <> struct TransportShape<double> {
    static constexpr int P = 4, KB = 4;
};
template <> struct TransportShape<float> {
    static constexpr int P = 2, KB = 8;
};

}  // namespace

int transport_tile_points(int precision)
{
    return kBlock * (precision == KX_MIXED ? TransportShape<float>::P : TransportShape<double>::P);
}

namespace {
template <class F>
kx_status go_transport(const MechDev &m, int64_t n, const double *T, const double *p,
                       const double *Y, double *mu, double *lam, double *Dmix, hipStream_t s)
{
    constexpr int PP = TransportShape<F>::P, KB = TransportShape<F>::KB;
    const int64_t per = (int64_t)kBlock * PP;
    const int64_t nblk = (n + per - 1) / per;
    if (nblk > 0x7fffffff) return fail(KX_EINVAL, "transport: n too large");
    const bool o5 = m.fit_order == 5;
    auto k = m.diff_kind == 0
                 ? (o5 ? transport_kernel<F, 5, 0, PP, KB> : transport_kernel<F, 0, 0, PP, KB>)
                 : (o5 ? transport_kernel<F, 5, 1, PP, KB> : transport_kernel<F, 0, 1, PP, KB>);
    hipLaunchKernelGGL(k, dim3((unsigned)nblk), dim3(kBlock), 0, s, m, n, T, p, Y, mu, lam,
                       Dmix);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "transport kernel launch");
    return ok();
}

template <class F>
kx_status go_transport_batch(const MechDev &m, const WorkList *wl, int *counter, int grid,
                             hipStream_t s)
{
    constexpr int PP = TransportShape<F>::P, KB = TransportShape<F>::KB;
    const bool o5 = m.fit_order == 5;
    auto k = m.diff_kind == 0 ? (o5 ? transport_batch_kernel<F, 5, 0, PP, KB>
                                    : transport_batch_kernel<F, 0, 0, PP, KB>)
                              : (o5 ? transport_batch_kernel<F, 5, 1, PP, KB>
                                    : transport_batch_kernel<F, 0, 1, PP, KB>);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, s, m, wl, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "transport batch kernel launch");
    return ok();
}
}  // namespace

kx_status launch_transport(const kx_mech *mech, int64_t n, const double *T, const double *p,
                           const double *Y, double *mu, double *lam, double *Dmix,
                           int precision, hipStream_t s)
{
    if (precision == KX_MIXED)
        return go_transport<float>(mech->dev, n, T, p, Y, mu, lam, Dmix, s);
    return go_transport<double>(mech->dev, n, T, p, Y, mu, lam, Dmix, s);
}

kx_status launch_transport_batch(const MechDev &m, const WorkList *wl, int *counter,
                                 int precision, int grid, hipStream_t s)
{
    if (precision == KX_MIXED) return go_transport_batch<float>(m, wl, counter, grid, s);
    return go_transport_batch<double>(m, wl, counter, grid, s);
}

kx_status launch_zero(int *p, int count, hipStream_t s)
{
    hipLaunchKernelGGL(zero_kernel, dim3((count + 63) / 64), dim3(64), 0, s, p, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "zero kernel launch");
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
