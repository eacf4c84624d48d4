// kx_rates.hip -- species net production rates on gfx950.
//
// Work decomposition (one wave per grid point at a time).  A workgroup of four
// waves owns a tile of `tp` consecutive points: the tile of Y is staged
// through LDS with coalesced row loads, and the same LDS tile later receives
// wdot and is written back with coalesced row stores.  For each of its points
// a wave runs three phases, with lanes spread over species, then reactions,
// then species again:
//
//  1. species (lane = k): C_k, the Gibbs energy g_k = G_k/RT of eq:Ck (range by
//     T_mid), a_k = (p_atm/RT) exp(-g_k) and b_k = C_k / a_k into wave-private
//     LDS.  With these, prod_k C_k^nu' = A' B' and prod_k C_k^nu'' / K_c = A' B''
//     (A' = prod_reac a^nu', B' = prod_reac b^nu', B'' = prod_prod b^nu''), since
//     K_c = prod_k a_k^(nu''-nu') by eq:K_p and K_c = K_p (p_atm/RT)^(sum nu).
//     So K_c needs one exponential per species instead of one per reaction and
//     the rate of progress needs no division:
//         R_i = c_i k_f A' (B' - B'')                   (eq:r_i, eq:c_i)
//     and B' - B'' is the near-equilibrium difference, formed in FP64.
//  2. reactions (lane = reaction): k_f (eq:arrhenius, with the beta = E_R = 0
//     shortcut of eq:k_f), [X]_i, the Lindemann / Troe factor (eq:blend) and
//     R_i into a wave-private LDS array, one chunk of reactions at a time.
//  3. species (lane = k): wdot_k = sum_i nu_ki R_i gathered from a species-major
//     list of (reaction, nu) pairs -- a fixed summation order, so results are
//     deterministic; the mixed path accumulates with Neumaier compensation.
#include <float.h>

#include "kx_internal.h"

namespace kx {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kSPL = kMaxSpecies / kWave;  // species per lane

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v)
{
    // xor butterfly: every lane forms the same sums (a + b == b + a), so all
    // lanes end with the bit-identical total.
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double ipow(double x, int nu)
{
    double r = x;
    for (int j = 1; j < nu; ++j) r *= x;
    return r;
}

// exp(x) for the mixed path: the argument stays in FP64, is reduced by n ln 2
// in FP64 and only exp(r), |r| <= ln2/2, is evaluated in FP32.
__device__ __forceinline__ double exp_mixed(double x)
{
    const double nd = rint(x * 1.4426950408889634);
    const double r = fma(-nd, 6.93147180559945286e-01, x);
    const float er = __expf((float)r);
    return ldexp((double)er, (int)nd);
}

template <bool MIXED>
__device__ __forceinline__ double arrhenius(double lnA, double beta, double ER, double lnT,
                                            double invT)
{
    const double x = fma(beta, lnT, fma(-ER, invT, lnA));
    return MIXED ? exp_mixed(x) : exp(x);
}

// Troe blending factor (eq:blend, base-10 logarithms).
__device__ __forceinline__ double troe_F64(const DevAux &ax, double T, double invT, double Pr)
{
    double Fc = (1.0 - ax.troe_alpha) * exp(-T * ax.troe_inv_T3) +
                ax.troe_alpha * exp(-T * ax.troe_inv_T1);
    if (ax.has_T2) Fc += exp(-ax.troe_T2 * invT);
    const double lFc = log10(Fc);
    const double c = -0.4 - 0.67 * lFc;
    const double nn = 0.75 - 1.27 * lFc;
    const double x = log10(fmax(Pr, DBL_MIN)) + c;
    const double f1 = x / (nn - 0.14 * x);
    return exp10(lFc / (1.0 + f1 * f1));
}

// FP32 Troe blend from log10 P_r (computed by the caller without overflow).
__device__ __forceinline__ float troe_F32(const DevAux &ax, float T, float invT, float lPr)
{
    const float al = (float)ax.troe_alpha;
    float Fc = (1.0f - al) * __expf(-T * (float)ax.troe_inv_T3) +
               al * __expf(-T * (float)ax.troe_inv_T1);
    if (ax.has_T2) Fc += __expf(-(float)ax.troe_T2 * invT);
    const float lFc = log10f(Fc);
    const float c = -0.4f - 0.67f * lFc;
    const float nn = 0.75f - 1.27f * lFc;
    const float x = lPr + c;
    const float f1 = x / (nn - 0.14f * x);
    return exp10f(lFc / (1.0f + f1 * f1));
}

// log10 of a positive double over its whole range, in FP32 arithmetic.
__device__ __forceinline__ float log10_wide(double v)
{
    int ex;
    const double mant = frexp(fmax(v, DBL_MIN), &ex);
    return (__log2f((float)mant) + (float)ex) * 0.30102999566398120f;
}

// Rate of progress R_i of one reaction (lane-private work).
template <bool MIXED>
__device__ __forceinline__ double rate_of_progress(const MechDev &m, const DevRxn &rx,
                                                   const double *__restrict__ sa,
                                                   const double *__restrict__ sb,
                                                   double Ti, double lnT, double invT,
                                                   double Mconc)
{
    const double kf = (rx.flags & kFlagKfConst)
                          ? rx.A
                          : arrhenius<MIXED>(rx.lnA, rx.beta, rx.ER, lnT, invT);
    double Ap = 1.0, Bp = 1.0, Bpp = 1.0;
#pragma unroll
    for (int q = 0; q < kMaxSide; ++q) {
        if (rx.rnu[q]) {
            const int k = rx.rsp[q];
            Ap *= ipow(sa[k], rx.rnu[q]);
            Bp *= ipow(sb[k], rx.rnu[q]);
        }
        if (rx.pnu[q]) Bpp *= ipow(sb[rx.psp[q]], rx.pnu[q]);
    }
    double c = 1.0;
    if (rx.type != KX_RXN_ELEMENTARY) {
        const DevAux ax = m.aux[rx.aux];
        if (MIXED) {
            float Xf = (float)(ax.eff_default * Mconc);
            for (int e = 0; e < ax.eff_cnt; ++e) {
                const DevEff f = m.eff[ax.eff_off + e];
                Xf += (float)f.dalpha * (float)(sa[f.sp] * sb[f.sp]);
            }
            const double X = (double)Xf;
            c = X;
            if (rx.type != KX_RXN_THREEBODY) {
                // k_0 / k_inf spans many decades: P_r and P_r/(1+P_r) in FP64,
                // the Troe blend in FP32 from a range-safe log10 P_r.
                const double k0 = arrhenius<true>(ax.lnA0, ax.beta0, ax.ER0, lnT, invT);
                const double Pr = k0 * X / kf;
                const float F = (rx.type == KX_RXN_TROE)
                                    ? troe_F32(ax, (float)Ti, (float)invT, log10_wide(Pr))
                                    : 1.0f;
                c = Pr / (1.0 + Pr) * (double)F;
            }
        } else {
            double X = ax.eff_default * Mconc;
            for (int e = 0; e < ax.eff_cnt; ++e) {
                const DevEff f = m.eff[ax.eff_off + e];
                X += f.dalpha * (sa[f.sp] * sb[f.sp]);
            }
            c = X;
            if (rx.type != KX_RXN_THREEBODY) {
                const double k0 = arrhenius<false>(ax.lnA0, ax.beta0, ax.ER0, lnT, invT);
                const double Pr = k0 * X / kf;
                const double F =
                    (rx.type == KX_RXN_TROE) ? troe_F64(ax, Ti, invT, Pr) : 1.0;
                c = Pr / (1.0 + Pr) * F;
            }
        }
    }
    const double br = (rx.flags & kFlagReversible) ? (Bp - Bpp) : Bp;
    return c * kf * Ap * br;
}

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void rates_kernel(MechDev m, int64_t n,
                                                       const double *__restrict__ T,
                                                       const double *__restrict__ P,
                                                       const double *__restrict__ Y,
                                                       double *__restrict__ wdot, int tp)
{
    extern __shared__ double lds[];
    const int ns = m.ns;
    const int ys = tp + 1;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    double *Yt = lds;
    double *sa = lds + (size_t)ns * ys + (size_t)wave * (2 * ns + m.chunk);
    double *sb = sa + ns;
    double *sq = sb + ns;

    const int64_t i0 = (int64_t)blockIdx.x * tp;
    const int npts = (int)min((int64_t)tp, n - i0);
    for (int e = threadIdx.x; e < ns * tp; e += kBlock) {
        const int k = e / tp, c = e - k * tp;
        Yt[k * ys + c] = (c < npts) ? Y[(int64_t)k * n + i0 + c] : 0.0;
    }
    __syncthreads();

    for (int pl = wave; pl < npts; pl += kWavesPerBlock) {
        const int64_t i = i0 + pl;
        const double Ti = T[i], pi = P[i];
        const double lnT = log(Ti), invT = 1.0 / Ti;
        const double RT = kRu * Ti;
        const double P0 = kPatm / RT;
        const double Mconc = pi / RT;

        // ---- phase 1: species
        double yk[kSPL];
        double part = 0.0;
#pragma unroll
        for (int s = 0; s < kSPL; ++s) {
            const int k = lane + kWave * s;
            yk[s] = 0.0;
            if (k < ns) {
                yk[s] = Yt[k * ys + pl];
                part += yk[s] * m.sp[k].inv_W;
            }
        }
        const double sumYW = wave_sum(part);
        const double cfac = Mconc / sumYW;
#pragma unroll
        for (int s = 0; s < kSPL; ++s) {
            const int k = lane + kWave * s;
            if (k < ns) {
                const DevSpecies &S = m.sp[k];
                const double *g = (Ti < S.t_mid) ? S.g_lo : S.g_hi;
                const double poly = Ti * fma(Ti, fma(Ti, fma(Ti, g[4], g[3]), g[2]), g[1]);
                const double gk = fma(g[0], 1.0 - lnT, poly) + fma(g[5], invT, g[6]);
                const double ak = P0 * exp(-gk);
                const double Ck = yk[s] * S.inv_W * cfac;
                sa[k] = ak;
                sb[k] = Ck / ak;
            }
        }
        wave_sync();

        // ---- phases 2 and 3, one chunk of reactions at a time
        double acc[kSPL], cmp[kSPL];
#pragma unroll
        for (int s = 0; s < kSPL; ++s) acc[s] = cmp[s] = 0.0;
        for (int c = 0; c < m.nchunks; ++c) {
            const int base = c * m.chunk;
            const int cnt = min(m.chunk, m.nr - base);
            for (int r = lane; r < cnt; r += kWave) {
                const DevRxn rx = m.rxn[base + r];
                sq[r] = rate_of_progress<MIXED>(m, rx, sa, sb, Ti, lnT, invT, Mconc);
            }
            wave_sync();
            const int32_t *gp = m.gptr + (size_t)c * (ns + 1);
#pragma unroll
            for (int s = 0; s < kSPL; ++s) {
                const int k = lane + kWave * s;
                if (k < ns) {
                    const int e1 = gp[k + 1];
                    for (int e = gp[k]; e < e1; ++e) {
                        const int32_t v = m.gent[e];
                        const double t = (double)(int8_t)(v & 0xFF) * sq[v >> 8];
                        if (MIXED) {
                            const double sum = acc[s] + t;
                            cmp[s] += (fabs(acc[s]) >= fabs(t)) ? (acc[s] - sum) + t
                                                                : (t - sum) + acc[s];
                            acc[s] = sum;
                        } else {
                            acc[s] += t;
                        }
                    }
                }
            }
            wave_sync();
        }
#pragma unroll
        for (int s = 0; s < kSPL; ++s) {
            const int k = lane + kWave * s;
            if (k < ns) Yt[k * ys + pl] = MIXED ? acc[s] + cmp[s] : acc[s];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ns * tp; e += kBlock) {
        const int k = e / tp, c = e - k * tp;
        if (c < npts) wdot[(int64_t)k * n + i0 + c] = Yt[k * ys + c];
    }
}

size_t rates_lds_bytes(const MechDev &m, int tp)
{
    return sizeof(double) *
           ((size_t)m.ns * (tp + 1) + (size_t)kWavesPerBlock * (2 * m.ns + m.chunk));
}

}  // namespace

kx_status launch_rates(const kx_mech *mech, int64_t n, const double *T, const double *p,
                       const double *Y, double *wdot, int precision, hipStream_t s)
{
    const MechDev &m = mech->dev;
    // Largest tile (64, 32 or 16 points) that leaves room for three workgroups
    // per CU (160 KB of LDS), else two, else one.
    int tp = 16;
    const size_t limits[3] = {53 * 1024, 80 * 1024, 160 * 1024};
    bool found = false;
    for (size_t lim : limits) {
        for (int cand : {64, 32, 16}) {
            if (rates_lds_bytes(m, cand) <= lim) {
                tp = cand;
                found = true;
                break;
            }
        }
        if (found) break;
    }
    const size_t lds = rates_lds_bytes(m, tp);
    if (lds > 160 * 1024)
        return fail(KX_EUNSUPPORTED, "production rates: mechanism too large for LDS");
    const int64_t nblk = (n + tp - 1) / tp;
    if (nblk > 0x7fffffff) return fail(KX_EINVAL, "production rates: n too large");
    auto kern = precision == KX_MIXED ? rates_kernel<true> : rates_kernel<false>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute (rates)");
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(kBlock), lds, s, m, n, T, p, Y, wdot,
                       tp);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "rates kernel launch");
    return ok();
}

}  // namespace kx
