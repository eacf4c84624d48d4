// kx_transport.hip -- mixture-averaged transport and mixture thermo on gfx950.
//
// Three evaluations of the same sums (App. A.3):
//  * the matrix-core kernel (tables holding fits of 1/D_kj and at least 24
//    species): the pair sums as products of fixed matrices with per-point
//    stacks on 16x16x4 MFMAs, described where it is defined below;
//  * the vector-ALU kernel (tables of D_kj fits, or fewer species): each lane
//    evaluates P grid points, every mechanism constant is wave-uniform and read
//    with scalar loads into scalar registers, used directly as an instruction
//    operand (one fetched coefficient serves the P points of all 64 lanes); the
//    quadratic sums run over a block of KB species k held in registers while j
//    streams over all species, and X_j is recomputed from Y_j (a coalesced
//    re-read) instead of being held per lane;
//  * the symmetric evaluation of D_kj fits (KX_DKJ_SYMMETRIC, §2.2.2 / §2.3.2),
//    described where it is defined below.
// Common to them:
//  * pure species (App. A.3 "Polynomial fits"): eta_k, lambda_k, D_kj as
//    polynomials in u = (ln T - L0)/h (Horner), D_kj divided by p/p_atm;
//  * Wilke / Bird viscosity with phi_kj = c1_kj (1 + sigma_k rho_j)^2, where
//    c1_kj = (8 (1 + W_k/W_j))^(-1/2), sigma_k = sqrt(eta_k) / W_k^(1/4) and
//    rho_j = W_j^(1/4) / sqrt(eta_j): (W_j/W_k)^(1/4) separates into
//    per-species factors, so each pair reads one coefficient;
//  * Mathur conductivity; eq:mix_diff for D_km, the reciprocals of the
//    positive sums by v_rcp_f64 and one Newton step (about 2^-48 relative).
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

// The same with per-lane coefficients (vector registers).
template <int ORDER, class F>
__device__ __forceinline__ F horner_v(const F *__restrict__ c, F u, int order)
{
    const int o = ORDER > 0 ? ORDER : order;
    F r = c[o - 1];
    for (int q = o - 2; q >= 0; --q) r = fma(r, u, c[q]);
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
// Reciprocals in the matrix-core kernel, where each result is a term of a sum
// of positive terms or a factor of one output: FP64 from v_rcp_f64 with one
// Newton step (about 2^-48 relative; FP64 vector instructions also cost the
// matrix pipe, so the second step is left out), FP32 from v_rcp_f32 with one
// Newton step (about 1 ulp, without the IEEE division's scaling and fix-up
// steps).
template <class F> __device__ __forceinline__ F rcp_mfma(F x);
template <> __device__ __forceinline__ double rcp_mfma<double>(double x) { return krcp1(x); }
template <> __device__ __forceinline__ float rcp_mfma<float>(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

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

// ---------------------------------------------------------------------------
// Symmetric evaluation of the D_kj fits (§2.2.2, §2.3.2: D_kj = D_jk, so half
// of the polynomial evaluations can be skipped).  With tables of D_kj fits
// (kind 0) every pair costs a polynomial and a reciprocal; here each unordered
// pair {k, j} is evaluated once and its 1/D_kj enters both sums
// S_k = sum_{j != k} X_j / D_kj and S_j.  One wave per workgroup, one point per
// lane (64 points).  S_j of a pair belongs to a species whose row is finished
// later, so the sums of every species are kept per lane in LDS (ns x 64
// values; each lane its own column).  The k rows are taken KB at a time with
// S_k in registers: pairs (k, j) with j before the block were added to S_k's
// LDS entry when j's block ran, pairs inside the block update the block's
// registers, and pairs with j after the block add X_k / D_kj to S_j's entry.
// The Wilke sums take the ordered pairs (phi_kj != phi_jk) as the full kernel.
template <class F, int ORDER, int KB>
__global__ __launch_bounds__(kWave) void transport_sym_kernel(MechDev m, int64_t n,
                                                              const double *__restrict__ T,
                                                              const double *__restrict__ Pp,
                                                              const double *__restrict__ Y,
                                                              double *__restrict__ mu,
                                                              double *__restrict__ lam,
                                                              double *__restrict__ Dmix)
{
    using Tb = Tabs<F>;
    extern __shared__ double smem_d[];
    F *sj = reinterpret_cast<F *>(smem_d);  // [ns][kWave]: S_j of this lane's point
    const int lane = threadIdx.x;
    const int ns = m.ns, order = m.fit_order;
    const int64_t ir = (int64_t)blockIdx.x * kWave + lane;
    const bool act = ir < n;
    const int64_t i = act ? ir : n - 1;
    const double Ti = T[i];
    const F u = (F)((kln(Ti) - m.fit_L0) * m.inv_fit_h);
    const double pr = Pp[i] / kPatm;
    auto Yat = [&](int k) { return Y[(int64_t)k * n + i]; };

    // X_k = (Y_k / W_k) xf; W-bar = sum_k X_k W_k; Mathur conductivity
    double xf, wbar = 0.0;
    {
        double sYW = 0.0;
        for (int k = 0; k < ns; ++k) sYW = fma(Yat(k), m.sp[k].inv_W, sYW);
        xf = 1.0 / sYW;
        F s1 = (F)0, s2 = (F)0;
        for (int k = 0; k < ns; ++k) {
            const double X = Yat(k) * m.sp[k].inv_W * xf;
            const F lk = horner<ORDER>(Tb::cond(m) + k * order, u, order);
            s1 = fma((F)X, lk, s1);
            s2 = fma((F)X, rcp_acc(lk), s2);
            wbar = fma(X, m.W[k], wbar);
            sj[k * kWave + lane] = (F)0;
        }
        if (act) lam[i] = (double)((F)0.5 * (s1 + rcp_acc(s2)));
    }

    F visc = (F)0;
    const int nkb = (ns + KB - 1) / KB;
    for (int kb = 0; kb < nkb; ++kb) {
        const int k0 = kb * KB, k1 = min(k0 + KB, ns);
        const int tb = k0 / kKB, toff = k0 % kKB;
        F sig[KB], den[KB], acc[KB], xk[KB];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            const int k = k0 + kk;
            const bool valid = k < ns;
            const int kc = valid ? k : 0;
            const F ek = horner<ORDER>(Tb::visc(m) + kc * order, u, order);
            sig[kk] = valid ? ek * rsqrt_acc(ek) * rcp_acc(Tb::wq(m)[kc]) : (F)0;
            den[kk] = (F)0;
            acc[kk] = valid ? sj[kc * kWave + lane] : (F)0;
            xk[kk] = valid ? (F)(Yat(kc) * m.sp[kc].inv_W * xf) : (F)0;
        }
        const F *c1b = Tb::wilke(m) + (size_t)tb * ns * kKB + toff;
        const F *dfb = Tb::dfit(m) + ((size_t)tb * ns * kKB + toff) * order;
        // pairs inside the block: (k0 + a, k0 + b), a < b
#pragma unroll
        for (int a = 0; a < KB; ++a)
#pragma unroll
            for (int b = a + 1; b < KB; ++b)
                if (k0 + b < ns) {
                    const F f = horner<ORDER>(dfb + ((size_t)(k0 + b) * kKB + a) * order, u,
                                              order);
                    const F g = rcp_fast(f);
                    acc[a] = fma(xk[b], g, acc[a]);
                    acc[b] = fma(xk[a], g, acc[b]);
                }
        for (int j = 0; j < ns; ++j) {
            const F wj = Tb::wq(m)[j];
            const F Xj = (F)(Yat(j) * m.sp[j].inv_W * xf);
            const F rho = wj * rsqrt_acc(horner<ORDER>(Tb::visc(m) + j * order, u, order));
            const F *c1 = c1b + (size_t)j * kKB;
#pragma unroll
            for (int kk = 0; kk < KB; ++kk) {
                // Wilke: X_j phi_kj = c1 X_j (1 + sigma_k rho_j)^2, every ordered pair
                const F t = fma(sig[kk], rho, (F)1);
                den[kk] = fma(c1[kk], Xj * t * t, den[kk]);
            }
            if (j >= k1) {
                const F *df = dfb + (size_t)j * kKB * order;
                F s = (F)0;
#pragma unroll
                for (int kk = 0; kk < KB; ++kk) {
                    const F g = rcp_fast(horner<ORDER>(df + kk * order, u, order));
                    acc[kk] = fma(Xj, g, acc[kk]);
                    s = fma(xk[kk], g, s);  // xk = 0 past the last species
                }
                sj[j * kWave + lane] += s;
            }
        }
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            const int k = k0 + kk;
            if (k < ns) {
                const double Xk = Yat(k) * m.sp[k].inv_W * xf;
                const F ek = horner<ORDER>(Tb::visc(m) + k * order, u, order);
                visc = fma((F)Xk * ek, rcp_acc(den[kk]), visc);
                double D;
                if (acc[kk] == (F)0) {
                    const F f = horner<ORDER>(Tb::ddiag(m) + k * order, u, order);
                    D = (double)f / pr;
                } else {
                    D = (wbar - Xk * m.W[k]) / (wbar * (double)acc[kk] * pr);
                }
                if (act) Dmix[(int64_t)k * n + i] = D;
            }
        }
    }
    if (act) mu[i] = (double)visc;
}

// ---------------------------------------------------------------------------
// Matrix-core form (tables holding fits of 1/D_kj, the form the paper's
// generated code evaluates).  With g_kj(u) = 1/D_kj(1 atm) = sum_n d_kjn u^n,
//     S_k = sum_{j != k} X_j g_kj = sum_n sum_j d_kjn (u^n X_j),
// a product of the fixed matrix [G_0 | ... | G_{N-1}] (G_n[k][j] = d_kjn, zero
// diagonal) with the per-point stack (u^n X_j).  The Wilke denominator, with
// t_kj = 1 + sigma_k rho_j and sigma_k = 1 / rho_k,
//     sum_j c1_kj X_j t_kj^2 = A_k + 2 sigma_k B_k + sigma_k^2 C_k,
// needs the products of the fixed matrix c1 with X, X rho and X rho^2 (all
// terms positive, so the expansion loses nothing).  A workgroup of four waves
// takes NP points: X and rho go to LDS, each wave runs 16x16x4 MFMAs for its
// blocks of 16 species k, and the epilogue forms mu, D_km per (k, point).

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <class F> struct Mfma;
template <> struct Mfma<double> {
    using V = v4d;
    static __device__ __forceinline__ V op(double a, double b, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row of the 16x16 result held by lane l in element r
    static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
    static __device__ const double *gfrag(const MechDev &m) { return m.gfrag; }
    static __device__ const double *c1frag(const MechDev &m) { return m.c1frag; }
};
template <> struct Mfma<float> {
    using V = v4f;
    static __device__ __forceinline__ V op(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
    static __device__ const float *gfrag(const MechDev &m) { return m.gfrag32; }
    static __device__ const float *c1frag(const MechDev &m) { return m.c1frag32; }
};

constexpr int kMfmaPad = 2;  // LDS row padding of the X / rho tiles (elements)

// Per-point values shared by the phases of a tile.
struct MfmaPoint {
    double u, xf, wbar, pr;
};

template <class F, int NP>
__host__ __device__ constexpr size_t mfma_lds_bytes_np(int kstep)
{
    // X and rho tiles, point table, partial sums (per (group, point) in the
    // prologue: 3 sums, and the normalisation sum in a slot of its own; 16 per
    // point for mu)
    return 2 * (size_t)(4 * kstep) * (NP + kMfmaPad) * sizeof(F) + NP * sizeof(MfmaPoint) +
           (size_t)4 * kBlock * sizeof(double);
}

// `tid` is threadIdx.x; the batch kernel passes it through an opaque move in
// each trip of its tile loop, so that the tile's lane-dependent addresses are
// not hoisted out of the loop (kept live across tiles they cost the kernel
// its occupancy).  LOOP: the workgroup takes another tile after this one (its
// LDS is then reused).
template <class F, int NP, int ORDER, bool LOOP>
__device__ __forceinline__ void transport_mfma_tile(int tid, const MechDev &m, int64_t n,
                                                    int64_t base,
                                                    const double *__restrict__ T,
                                                    const double *__restrict__ Pp,
                                                    const double *__restrict__ Y,
                                                    double *__restrict__ mu,
                                                    double *__restrict__ lam,
                                                    double *__restrict__ Dmix)
{
    using Tb = Tabs<F>;
    using MF = Mfma<F>;
    using V = typename MF::V;
    constexpr int NB = NP / 16;          // 16-point column blocks
    constexpr int NG = kBlock / NP;      // species groups of the prologue
    constexpr int LD = NP + kMfmaPad;    // LDS row stride of the tiles
    const int ns = m.ns, order = ORDER > 0 ? ORDER : m.fit_order;
    const int KS = m.kstep, MB = m.mblk, Kp = 4 * KS;
    const int t = tid, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);

    extern __shared__ double smem_d[];
    F *Xs = reinterpret_cast<F *>(smem_d);
    F *Rs = Xs + (size_t)Kp * LD;
    MfmaPoint *pt = reinterpret_cast<MfmaPoint *>(Rs + (size_t)Kp * LD);
    double *part = reinterpret_cast<double *>(pt + NP);  // [NG][3][NP], then mu's [16][NP]
    double *part1 = part + 3 * kBlock;                   // [NG][NP]: sum of Y_j / W_j

    // ---- prologue: thread = (point p, species group g)
    const int p = t % NP;
    // with 64-point tiles the species group is the wave: uniform, so the
    // per-species coefficients below come from scalar loads
    const int g = NP == 64 ? __builtin_amdgcn_readfirstlane(t / NP) : t / NP;
    const int64_t ip = min(base + p, n - 1);  // points past n repeat the last one
    const double Tp = T[ip];
    const double up = (kln(Tp) - m.fit_L0) * m.inv_fit_h;
    // every Y load of this thread is issued before the first is used (a
    // thread covers at most kJmax species: ns <= 4 NP for the chosen NP)
    constexpr int kJmax = 16;
    double yw[kJmax];
#pragma unroll
    for (int q = 0; q < kJmax; ++q) {
        const int j = g + NG * q;
        yw[q] = j < ns ? Y[(int64_t)j * n + ip] : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kJmax; ++q) {
        const int j = g + NG * q;
        if (j < ns) {
            yw[q] *= m.sp[j].inv_W;  // Y_j / W_j
            s += yw[q];
        }
    }
    part1[g * NP + p] = s;
    __syncthreads();
    double sYW = 0.0;
#pragma unroll
    for (int q = 0; q < NG; ++q) sYW += part1[q * NP + p];
    const double xf = krcp(sYW);
    if (t < NP) {
        MfmaPoint P;
        P.u = up;
        P.xf = xf;
        P.wbar = 0.0;  // the epilogue adds the group partials
        P.pr = Pp[ip] * (1.0 / kPatm);
        pt[p] = P;
    }
    double wb = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < kJmax; ++q) {
        const int j = g + NG * q;
        if (j >= Kp) break;
        if (j < ns) {
            const double X = yw[q] * xf;  // FP64 X_j for W-bar and the Mathur sums
            wb = fma(X, m.W[j], wb);
            const F lj = NP == 64 ? horner<ORDER>(Tb::cond(m) + j * order, (F)up, order)
                                  : horner_v<ORDER>(Tb::cond(m) + j * order, (F)up, order);
            s1 = fma(X, (double)lj, s1);
            s2 = fma(X, (double)rcp_mfma(lj), s2);
            const F ej = NP == 64 ? horner<ORDER>(Tb::visc(m) + j * order, (F)up, order)
                                  : horner_v<ORDER>(Tb::visc(m) + j * order, (F)up, order);
            Xs[(size_t)j * LD + p] = (F)X;
            Rs[(size_t)j * LD + p] = Tb::wq(m)[j] * rsqrt_acc(ej);  // rho_j
        } else {
            Xs[(size_t)j * LD + p] = (F)0;
            Rs[(size_t)j * LD + p] = (F)1;
        }
    }
    part[(g * 3 + 0) * NP + p] = wb;
    part[(g * 3 + 1) * NP + p] = s1;
    part[(g * 3 + 2) * NP + p] = s2;
    __syncthreads();
    if (t < NP && base + p < n) {
        double a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            a1 += part[(q * 3 + 1) * NP + p];
            a2 += part[(q * 3 + 2) * NP + p];
        }
        lam[base + p] = 0.5 * (a1 + krcp(a2));  // Mathur
    }

    // ---- products on the matrix cores: wave w takes row blocks w, w + 4, ...
    const int col = lane & 15, jr = lane >> 4;
    F uc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) uc[nb] = (F)pt[16 * nb + col].u;
    double mup[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) mup[nb] = 0.0;
    const F *gf = MF::gfrag(m), *cf = MF::c1frag(m);
    constexpr int MO = ORDER > 0 ? ORDER : kMaxFitOrder;  // A fragments per K-step
    const size_t ostride = (size_t)MB * KS * 64;           // between fit orders
    for (int mb = w; mb < MB; mb += 4) {
        V S[NB], A[NB], B[NB], C[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) S[nb] = A[nb] = B[nb] = C[nb] = V{0, 0, 0, 0};
        // A fragments of the next K-step are in flight during this one
        const F *cfb = cf + (size_t)mb * KS * 64 + lane;
        const F *gfb = gf + (size_t)mb * KS * 64 + lane;
        F a1n = cfb[0], ggn[MO];
#pragma unroll
        for (int o = 0; o < MO; ++o)
            if (o < order) ggn[o] = gfb[o * ostride];
        for (int ks = 0; ks < KS; ++ks) {
            const F a1 = a1n;
            F gg[MO];
#pragma unroll
            for (int o = 0; o < MO; ++o) gg[o] = ggn[o];
            if (ks + 1 < KS) {
                a1n = cfb[(ks + 1) * 64];
#pragma unroll
                for (int o = 0; o < MO; ++o)
                    if (o < order) ggn[o] = gfb[o * ostride + (ks + 1) * 64];
            }
            const int j = 4 * ks + jr;
            F x[NB], r[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                x[nb] = Xs[(size_t)j * LD + 16 * nb + col];
                r[nb] = Rs[(size_t)j * LD + 16 * nb + col];
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const F xr = x[nb] * r[nb];
                A[nb] = MF::op(a1, x[nb], A[nb]);
                B[nb] = MF::op(a1, xr, B[nb]);
                C[nb] = MF::op(a1, xr * r[nb], C[nb]);
            }
            F bb[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) bb[nb] = x[nb];
#pragma unroll
            for (int o = 0; o < MO; ++o) {
                if (o < order) {
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        S[nb] = MF::op(gg[o], bb[nb], S[nb]);
                        bb[nb] *= uc[nb];
                    }
                }
            }
        }
        // ---- epilogue of this row block: element e of lane l is (k, point).
        // The Wilke denominator with sigma_k = 1/rho_k is
        //   A + sigma (2B + sigma C) = (A rho^2 + 2 B rho + C) / rho^2,
        // and the viscosity term X_k eta_k / den with eta_k = (W_k^(1/4) / rho_k)^2
        // becomes X_k W_k^(1/2) / (A rho^2 + 2 B rho + C): one reciprocal per
        // element, of a sum of positive terms.  In FP64, Z_k = X_k from the tile
        // and the row factor is W_k^(1/2); the mixed path (FP32 tile) forms
        // Z_k = Y_k W-bar' = X_k W_k in FP64 from the input, so its row factor
        // is W_k^(-1/2) and the D_km numerator W-bar - X_k W_k is W-bar - Z_k.
        constexpr bool F64 = std::is_same<F, double>::value;
        int krow[4];
        F rf[4];
        double wk[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            krow[e] = 16 * mb + MF::row(lane, e);
            const int kc = min(krow[e], ns - 1);
            const F q = Tb::wq(m)[kc];
            rf[e] = F64 ? q * q : (F)1 / (q * q);
            wk[e] = F64 ? m.W[kc] : 1.0;
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int pp = 16 * nb + col;
            const int64_t i = base + pp;
            const MfmaPoint P = pt[pp];
            double wbar = 0.0;
#pragma unroll
            for (int q = 0; q < NG; ++q) wbar += part[(q * 3 + 0) * NP + pp];
            double yk[4];
            if (!F64) {
                const int64_t ic = min(i, n - 1);
#pragma unroll
                for (int e = 0; e < 4; ++e) yk[e] = Y[(int64_t)min(krow[e], ns - 1) * n + ic];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = krow[e];
                if (k >= ns) continue;
                const F rho = Rs[(size_t)k * LD + pp];
                const F den = fma(fma(A[nb][e], rho, (F)2 * B[nb][e]), rho, C[nb][e]);
                const double Zk = F64 ? (double)Xs[(size_t)k * LD + pp] : yk[e] * P.xf;
                mup[nb] = fma(Zk, (double)(rf[e] * rcp_mfma(den)), mup[nb]);
                double D;
                if (S[nb][e] == (F)0) {
                    // no other species present: D_km -> D_kk
                    const F gk = horner_v<ORDER>(Tb::ddiag(m) + k * order, (F)P.u, order);
                    D = 1.0 / ((double)gk * P.pr);
                } else {
                    D = (wbar - Zk * wk[e]) * krcp1(wbar * (double)S[nb][e] * P.pr);
                }
                if (i < n) Dmix[(int64_t)k * n + i] = D;
            }
        }
    }
    // mu: 16 partial sums per point (4 waves x 4 row groups), fixed order
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) part[(w * 4 + jr) * NP + 16 * nb + col] = mup[nb];
    __syncthreads();
    if (t < NP && base + t < n) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) v += part[q * NP + t];
        mu[base + t] = v;
    }
    if (LOOP) __syncthreads();  // LDS reused by the next tile
}

template <class F, int NP, int ORDER>
__global__ __launch_bounds__(kBlock) void transport_mfma_kernel(MechDev m, int64_t n,
                                                                const double *__restrict__ T,
                                                                const double *__restrict__ Pp,
                                                                const double *__restrict__ Y,
                                                                double *__restrict__ mu,
                                                                double *__restrict__ lam,
                                                                double *__restrict__ Dmix)
{
    transport_mfma_tile<F, NP, ORDER, false>(threadIdx.x, m, n, (int64_t)blockIdx.x * NP, T, Pp, Y, mu,
                                      lam, Dmix);
}

// At most 256 VGPRs (two waves per SIMD): the FP64 form for fits of any order
// would otherwise take 258 and run one wave per SIMD.
template <class F, int NP, int ORDER>
__global__ __launch_bounds__(kBlock, 2) void transport_mfma_batch_kernel(
    MechDev m, const WorkList *__restrict__ wl, int *__restrict__ counter)
{
    __shared__ int tile;
    const int ntiles = wl->ntiles[1];
    int r = 0;  // item of the previous tile
    for (;;) {
        if (threadIdx.x == 0) tile = atomicAdd(counter, 1);
        __syncthreads();
        // wave-uniform (the compiler then keeps the item's pointers in scalar
        // registers; read as a per-lane value they cost the tile its occupancy)
        const int t = __builtin_amdgcn_readfirstlane(tile);
        __syncthreads();
        if (t >= ntiles) break;
        r = work_item_of(wl, 1, t, r);
        const WorkItem it = wl->items[r];
        int tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
        transport_mfma_tile<F, NP, ORDER, true>(tid, m, it.n, (int64_t)(t - wl->start[1][r]) * NP, it.T,
                                          it.p, it.Y, it.mu, it.lam, it.Dmix);
    }
}

// Batched requests, one tile per workgroup (grid = the batch's transport
// tiles).  Uniform per workgroup, so a workgroup past the last tile returns
// before any barrier.
template <class F, int NP, int ORDER>
__global__ __launch_bounds__(kBlock) void transport_mfma_items_kernel(
    MechDev m, const WorkList *__restrict__ wl)
{
    const int t = (int)blockIdx.x;
    if (t >= wl->ntiles[1]) return;
    const int r = work_item_ballot(wl, 1, t);
    const WorkItem it = wl->items[r];
    transport_mfma_tile<F, NP, ORDER, false>(threadIdx.x, m, it.n, (int64_t)(t - wl->start[1][r]) * NP,
                                      it.T, it.p, it.Y, it.mu, it.lam, it.Dmix);
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
    int r = 0;  // item of the previous tile
    for (;;) {
        if (threadIdx.x == 0) tile = atomicAdd(counter, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(tile);  // wave-uniform
        __syncthreads();
        if (t >= ntiles) break;
        r = work_item_of(wl, 1, t, r);
        const WorkItem it = wl->items[r];
        transport_tile<F, ORDER, KIND, P, KB>(m, it.n,
                                              (int64_t)(t - wl->start[1][r]) * kBlock * P, it.T,
                                              it.p, it.Y, it.mu, it.lam, it.Dmix);
    }
}

template <class F, int ORDER, int KIND, int P, int KB>
__global__ __launch_bounds__(kBlock) void transport_items_kernel(MechDev m,
                                                                 const WorkList *__restrict__ wl)
{
    const int t = (int)blockIdx.x;
    if (t >= wl->ntiles[1]) return;
    const int r = work_item_ballot(wl, 1, t);
    const WorkItem it = wl->items[r];
    transport_tile<F, ORDER, KIND, P, KB>(m, it.n, (int64_t)(t - wl->start[1][r]) * kBlock * P,
                                          it.T, it.p, it.Y, it.mu, it.lam, it.Dmix);
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

// Points per matrix-core tile: the largest of 64, 32, 16 whose LDS (X and rho
// tiles) stays within 80 KB, i.e. two workgroups per CU.
// The prologue gives each thread at most 16 species (256 / NP groups), so NP
// also bounds the species count: NP = 64 up to 64 species, 32 up to 128.
template <class F> int mfma_np(const MechDev &m)
{
    const int kp = 4 * m.kstep;
    if (kp <= 64 && mfma_lds_bytes_np<F, 64>(m.kstep) <= 80 * 1024) return 64;
    if (kp <= 128 && mfma_lds_bytes_np<F, 32>(m.kstep) <= 80 * 1024) return 32;
    return 16;
}

template <class F> size_t mfma_lds(const MechDev &m, int np)
{
    return np == 64 ? mfma_lds_bytes_np<F, 64>(m.kstep)
                    : (np == 32 ? mfma_lds_bytes_np<F, 32>(m.kstep)
                                : mfma_lds_bytes_np<F, 16>(m.kstep));
}

// Below about two dozen species the padded 16 x 4 MFMA tiles are mostly empty
// and the vector-ALU kernel is faster.
constexpr int kMfmaMinSpecies = 24;
bool use_mfma(const MechDev &m)
{
    return m.diff_kind == 1 && m.gfrag != nullptr && m.ns >= kMfmaMinSpecies;
}

// FORM 0: direct launch, 1: work-stealing batch, 2: one tile per workgroup
template <class F, int FORM> const void *mfma_kernel(const MechDev &m, int np)
{
    const bool o5 = m.fit_order == 5;
#define KX_PICK(NPV)                                                                        \
    (FORM == 1 ? (o5 ? (const void *)transport_mfma_batch_kernel<F, NPV, 5>                 \
                     : (const void *)transport_mfma_batch_kernel<F, NPV, 0>)                \
     : FORM == 2 ? (o5 ? (const void *)transport_mfma_items_kernel<F, NPV, 5>               \
                       : (const void *)transport_mfma_items_kernel<F, NPV, 0>)              \
                 : (o5 ? (const void *)transport_mfma_kernel<F, NPV, 5>                     \
                       : (const void *)transport_mfma_kernel<F, NPV, 0>))
    return np == 64 ? KX_PICK(64) : (np == 32 ? KX_PICK(32) : KX_PICK(16));
#undef KX_PICK
}

template <class F, int FORM> kx_status mfma_prepare(const MechDev &m, size_t *lds)
{
    const int np = mfma_np<F>(m);
    *lds = mfma_lds<F>(m, np);
    if (*lds > 160 * 1024)
        return fail(KX_EUNSUPPORTED, "transport: mechanism too large for the LDS tiles");
    hipError_t e = hipFuncSetAttribute(mfma_kernel<F, FORM>(m, np),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)*lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute (transport)");
    return KX_OK;
}

}  // namespace

int transport_tile_points(const MechDev &m, int precision)
{
    if (use_mfma(m)) return precision == KX_MIXED ? mfma_np<float>(m) : mfma_np<double>(m);
    return kBlock * (precision == KX_MIXED ? TransportShape<float>::P : TransportShape<double>::P);
}

kx_status prepare_transport_batch(const MechDev &m, int precision)
{
    if (!use_mfma(m)) return KX_OK;
    size_t lds = 0;
    return precision == KX_MIXED ? mfma_prepare<float, 1>(m, &lds)
                                 : mfma_prepare<double, 1>(m, &lds);
}

namespace {
template <class F>
kx_status go_transport(const MechDev &m, int64_t n, const double *T, const double *p,
                       const double *Y, double *mu, double *lam, double *Dmix, bool sym,
                       hipStream_t s)
{
    if (sym && m.diff_kind == 0) {
        // one wave per 64 points, the per-lane sums of every species in LDS
        const size_t lds = (size_t)m.ns * kWave * sizeof(F);
        if (lds > 160 * 1024) return fail(KX_EUNSUPPORTED, "transport: symmetric D_kj sums "
                                                           "of this many species exceed the LDS");
        constexpr int KB = 8;
        auto k = m.fit_order == 5 ? transport_sym_kernel<F, 5, KB> : transport_sym_kernel<F, 0, KB>;
        hipError_t e = hipFuncSetAttribute((const void *)k,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute (symmetric transport)");
        const int64_t nblk = (n + kWave - 1) / kWave;
        if (nblk > 0x7fffffff) return fail(KX_EINVAL, "transport: n too large");
        hipLaunchKernelGGL(k, dim3((unsigned)nblk), dim3(kWave), lds, s, m, n, T, p, Y, mu, lam,
                           Dmix);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "symmetric transport kernel launch");
        return ok();
    }
    if (use_mfma(m)) {
        size_t lds = 0;
        kx_status st = mfma_prepare<F, 0>(m, &lds);
        if (st != KX_OK) return st;
        const int np = mfma_np<F>(m);
        const int64_t nblk = (n + np - 1) / np;
        if (nblk > 0x7fffffff) return fail(KX_EINVAL, "transport: n too large");
        void *args[] = {(void *)&m, (void *)&n, (void *)&T, (void *)&p, (void *)&Y,
                        (void *)&mu, (void *)&lam, (void *)&Dmix};
        hipError_t e = hipLaunchKernel(mfma_kernel<F, 0>(m, np), dim3((unsigned)nblk),
                                       dim3(kBlock), args, lds, s);
        if (e != hipSuccess) return hip_fail(e, "transport kernel launch");
        return ok();
    }
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
    if (use_mfma(m)) {
        const int np = mfma_np<F>(m);
        const size_t lds = mfma_lds<F>(m, np);
        void *args[] = {(void *)&m, (void *)&wl, (void *)&counter};
        hipError_t e = hipLaunchKernel(mfma_kernel<F, 1>(m, np), dim3(grid), dim3(kBlock),
                                       args, lds, s);
        if (e != hipSuccess) return hip_fail(e, "transport batch kernel launch");
        return ok();
    }
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
template <class F>
kx_status go_transport_items(const MechDev &m, const WorkList *wl, int64_t ntiles, hipStream_t s)
{
    if (ntiles <= 0) return ok();
    if (ntiles > 0x7fffffff) return fail(KX_EINVAL, "transport: too many tiles");
    if (use_mfma(m)) {
        size_t lds = 0;
        kx_status st = mfma_prepare<F, 2>(m, &lds);
        if (st != KX_OK) return st;
        const int np = mfma_np<F>(m);
        void *args[] = {(void *)&m, (void *)&wl};
        hipError_t e = hipLaunchKernel(mfma_kernel<F, 2>(m, np), dim3((unsigned)ntiles),
                                       dim3(kBlock), args, lds, s);
        if (e != hipSuccess) return hip_fail(e, "transport items kernel launch");
        return ok();
    }
    constexpr int PP = TransportShape<F>::P, KB = TransportShape<F>::KB;
    const bool o5 = m.fit_order == 5;
    auto k = m.diff_kind == 0 ? (o5 ? transport_items_kernel<F, 5, 0, PP, KB>
                                    : transport_items_kernel<F, 0, 0, PP, KB>)
                              : (o5 ? transport_items_kernel<F, 5, 1, PP, KB>
                                    : transport_items_kernel<F, 0, 1, PP, KB>);
    hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(kBlock), 0, s, m, wl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "transport items kernel launch");
    return ok();
}
}  // namespace

kx_status launch_transport_items(const MechDev &m, const WorkList *wl, int64_t ntiles,
                                 int precision, hipStream_t s)
{
    if (precision == KX_MIXED) return go_transport_items<float>(m, wl, ntiles, s);
    return go_transport_items<double>(m, wl, ntiles, s);
}

kx_status launch_transport(const kx_mech *mech, int64_t n, const double *T, const double *p,
                           const double *Y, double *mu, double *lam, double *Dmix,
                           int precision, hipStream_t s)
{
    const bool sym = (precision & KX_DKJ_SYMMETRIC) != 0;
    if ((precision & ~KX_DKJ_SYMMETRIC) == KX_MIXED)
        return go_transport<float>(mech->dev, n, T, p, Y, mu, lam, Dmix, sym, s);
    return go_transport<double>(mech->dev, n, T, p, Y, mu, lam, Dmix, sym, s);
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
