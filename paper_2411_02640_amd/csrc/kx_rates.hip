// kx_rates.hip -- species net production rates on gfx950.
//
// Work decomposition (one wave per grid point at a time).  A workgroup is one
// wave that owns a tile of `tp` consecutive points: the tile of Y is staged
// through LDS with coalesced row loads, and the same LDS tile later receives
// wdot and is written back with coalesced row stores.  For each of its points
// the wave runs three phases, with lanes spread over species, then reactions,
// then species again:
//
//  1. species (lane = k): C_k, the Gibbs energy g_k = G_k/RT of eq:Ck (range by
//     T_mid), a_k = (p_atm/RT) exp(-g_k) and b_k = C_k / a_k into LDS as one
//     16-byte pair per species.  With these, prod_k C_k^nu' = A' B' and prod_k C_k^nu'' / K_c = A' B''
//     (A' = prod_reac a^nu', B' = prod_reac b^nu', B'' = prod_prod b^nu''), since
//     K_c = prod_k a_k^(nu''-nu') by eq:K_p and K_c = K_p (p_atm/RT)^(sum nu).
//     So K_c needs one exponential per species instead of one per reaction and
//     the rate of progress needs no division:
//         R_i = c_i k_f A' (B' - B'')                   (eq:r_i, eq:c_i)
//     and B' - B'' is the near-equilibrium difference, formed in FP64.
//  2. reactions (lane = reaction): k_f (eq:arrhenius, with the beta = E_R = 0
//     shortcut of eq:k_f), [X]_i, the Lindemann / Troe factor (eq:blend) and
//     R_i into an LDS array, one chunk of reactions at a time.  Each reaction
//     side is three molecule slots (unused ones hit a dummy species with
//     a = b = 1), so the products A', B', B'' are branch-free.
//  3. species (lane = k): wdot_k = sum_i nu_ki R_i gathered from a species-major
//     list of (reaction, nu) pairs -- a fixed summation order, so results are
//     deterministic; the mixed path accumulates with Neumaier compensation.
#include <float.h>

#include <type_traits>

#include "kx_internal.h"
#include "kx_math.h"

namespace kx {
namespace {


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
    return MIXED ? exp_mixed(x) : kexp(x);
}

// Troe blending factor (eq:blend, base-10 logarithms).
__device__ __forceinline__ double troe_F64(const DevAux &ax, double T, double invT, double Pr)
{
    double Fc = (1.0 - ax.troe_alpha) * kexp(-T * ax.troe_inv_T3) +
                ax.troe_alpha * kexp(-T * ax.troe_inv_T1);
    if (ax.has_T2) Fc += kexp(-ax.troe_T2 * invT);
    const double lFc = log10(Fc);
    const double c = -0.4 - 0.67 * lFc;
    const double nn = 0.75 - 1.27 * lFc;
    const double x = log10(fmax(Pr, DBL_MIN)) + c;
    const double f1 = x * krcp(nn - 0.14 * x);
    return kexp10(lFc * krcp(1.0 + f1 * f1));
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

// Per-point factors of one species in LDS: {a_k, b_k}, 16 bytes.
struct Pair {
    double a, b;
};

__device__ __forceinline__ Pair load_pair(const char *pb, int off)
{
    return *reinterpret_cast<const Pair *>(pb + off);
}

__device__ __forceinline__ double load_b(const char *pb, int off)
{
    return *reinterpret_cast<const double *>(pb + off + 8);
}

// One reaction record held in registers: the three 16-byte words of DevRxn.
struct RxnWords {
    uint4 w0, w1, w2;
};

__device__ __forceinline__ double as_double(unsigned lo, unsigned hi)
{
    return __hiloint2double((int)hi, (int)lo);
}

// [X]_i = default [M] + sum over listed species of (alpha - default) C_k.
__device__ __forceinline__ double third_body(const MechDev &m, const DevAux &ax,
                                             const char *__restrict__ pb, double Mconc)
{
    double X = ax.eff_default * Mconc;
#pragma unroll
    for (int e = 0; e < kInlineEff; ++e) {
        const Pair s = load_pair(pb, ax.eoff[e]);
        X = fma(ax.dalpha[e], s.a * s.b, X);
    }
    for (int e = 0; e < ax.ext_cnt; ++e) {
        const DevEff f = m.eff[ax.ext_off + e];
        const Pair s = load_pair(pb, 16 * f.sp);
        X = fma(f.dalpha, s.a * s.b, X);
    }
    return X;
}

// Rate of progress R_i = c_i k_f A' (B' - B'') of one reaction (lane-private).
template <bool MIXED>
__device__ __forceinline__ double rate_of_progress(const MechDev &m, const RxnWords &w,
                                                   const char *__restrict__ pb, double Ti,
                                                   double lnT, double invT, double Mconc)
{
    const double lnA = as_double(w.w0.x, w.w0.y);
    const double beta = as_double(w.w0.z, w.w0.w);
    const double ER = as_double(w.w1.x, w.w1.y);
    const double A = as_double(w.w1.z, w.w1.w);
    const unsigned type = w.w2.w & 0xFFu;
    const unsigned flags = (w.w2.w >> 8) & 0xFFu;
    const unsigned aux = w.w2.w >> 16;

    double kf;
    if (flags & kFlagKfConst)
        kf = A;
    else
        kf = arrhenius<MIXED>(lnA, beta, ER, lnT, invT);
    const Pair r0 = load_pair(pb, w.w2.x & 0xFFFFu);
    const Pair r1 = load_pair(pb, w.w2.x >> 16);
    const Pair r2 = load_pair(pb, w.w2.y & 0xFFFFu);
    const double Ap = r0.a * r1.a * r2.a;
    const double Bp = r0.b * r1.b * r2.b;
    const double Bpp = load_b(pb, w.w2.y >> 16) * load_b(pb, w.w2.z & 0xFFFFu) *
                       load_b(pb, w.w2.z >> 16);
    double c = 1.0;
    if (type != KX_RXN_ELEMENTARY) {
        const DevAux ax = m.aux[aux];
        const double X = third_body(m, ax, pb, Mconc);
        c = X;
        if (type != KX_RXN_THREEBODY) {
            const double k0 = arrhenius<MIXED>(ax.lnA0, ax.beta0, ax.ER0, lnT, invT);
            const double Pr = k0 * X * krcp(kf);
            double F = 1.0;
            if (type == KX_RXN_TROE)
                F = MIXED ? (double)troe_F32(ax, (float)Ti, (float)invT, log10_wide(Pr))
                          : troe_F64(ax, Ti, invT, Pr);
            c = Pr * krcp(1.0 + Pr) * F;
        }
    }
    const double rev = (flags & kFlagReversible) ? 1.0 : 0.0;
    return c * kf * Ap * fma(-rev, Bpp, Bp);
}

// LDS layout of one workgroup (one wave):
//   pairs [ns + 1] {a, b}   (entry ns is the dummy species, {1, 1})
//   sq    [chunk + 1]       (rates of progress of the current chunk; the last
//                            element is the zero the gather padding reads)
//   Yt    [ns][tp + 1]      (Y tile in, wdot tile out)
// One tile of `npts` (<= tp) points starting at point i0 of arrays whose
// species rows have stride ld.  Called by the whole (one-wave) workgroup.
template <bool MIXED, int SPL>
__device__ __forceinline__ void rates_tile(const MechDev &m, int64_t ld, int64_t i0, int npts,
                                           int tp, const double *__restrict__ T,
                                           const double *__restrict__ P,
                                           const double *__restrict__ Y,
                                           double *__restrict__ wdot)
{
    extern __shared__ double lds[];
    const int ns = m.ns;
    const int ys = tp + 1;
    const int lane = threadIdx.x;
    double *pairs = lds;
    double *sq = lds + 2 * (ns + 1);
    double *Yt = sq + (m.chunk + 1);
    const char *pb = reinterpret_cast<const char *>(pairs);
    const char *qb = reinterpret_cast<const char *>(sq);

    for (int e = lane; e < ns * tp; e += kWave) {
        const int k = e / tp, c = e - k * tp;
        Yt[k * ys + c] = (c < npts) ? Y[(int64_t)k * ld + i0 + c] : 0.0;
    }
    if (lane == 0) {
        pairs[2 * ns] = 1.0;
        pairs[2 * ns + 1] = 1.0;
        sq[m.chunk] = 0.0;
    }
    __syncthreads();

    const int gw = kWave * m.gpass;
    for (int pl = 0; pl < npts; ++pl) {
        const int64_t i = i0 + pl;
        const double Ti = T[i], pi = P[i];
        const double lnT = log(Ti), invT = 1.0 / Ti;
        const double RT = kRu * Ti;
        const double P0 = kPatm / RT;
        const double Mconc = pi / RT;

        // ---- phase 1: species
        double yk[SPL];
        double part = 0.0;
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            const int k = lane + kWave * s;
            yk[s] = 0.0;
            if (k < ns) {
                yk[s] = Yt[k * ys + pl];
                part = fma(yk[s], m.sp[k].inv_W, part);
            }
        }
        const double cfac = Mconc / wave_sum(part);
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            const int k = lane + kWave * s;
            if (k < ns) {
                const DevSpecies &S = m.sp[k];
                const double *g = (Ti < S.t_mid) ? S.g_lo : S.g_hi;
                const double poly = Ti * fma(Ti, fma(Ti, fma(Ti, g[4], g[3]), g[2]), g[1]);
                const double gk = fma(g[0], 1.0 - lnT, poly) + fma(g[5], invT, g[6]);
                const double ak = P0 * kexp(-gk);
                const double Ck = yk[s] * S.inv_W * cfac;
                pairs[2 * k] = ak;
                pairs[2 * k + 1] = Ck * krcp(ak);
            }
        }
        wave_sync();

        // ---- phases 2 and 3, one chunk of reactions at a time
        double acc[SPL], cmp[SPL];
#pragma unroll
        for (int s = 0; s < SPL; ++s) acc[s] = cmp[s] = 0.0;
        for (int c = 0; c < m.nchunks; ++c) {
            const int base = c * m.chunk;
            const int cnt = min(m.chunk, m.nr - base);
            // 48-byte reaction records as three 16-byte loads, the next
            // iteration's record in flight while this one is evaluated
            const uint4 *rsrc = reinterpret_cast<const uint4 *>(m.rxn + base);
            RxnWords w;
            w.w0 = w.w1 = w.w2 = make_uint4(0, 0, 0, 0);
            if (lane < cnt) {
                w.w0 = rsrc[3 * lane];
                w.w1 = rsrc[3 * lane + 1];
                w.w2 = rsrc[3 * lane + 2];
            }
            for (int r = lane; r < cnt; r += kWave) {
                const RxnWords cur = w;
                const int rn = r + kWave;
                if (rn < cnt) {
                    w.w0 = rsrc[3 * rn];
                    w.w1 = rsrc[3 * rn + 1];
                    w.w2 = rsrc[3 * rn + 2];
                }
                sq[r] = rate_of_progress<MIXED>(m, cur, pb, Ti, lnT, invT, Mconc);
            }
            wave_sync();
            const int len = m.glen[c];  // a multiple of 8
            const int32_t *ge = m.gent + m.goff[c] + lane;
#pragma unroll
            for (int s = 0; s < SPL; ++s) {
                const int32_t *g = ge + kWave * s;
                for (int it = 0; it < len; it += 8) {
                    int32_t v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = g[(size_t)(it + u) * gw];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const double q = *reinterpret_cast<const double *>(qb + (v[u] >> 8));
                        const double t = (double)(int8_t)(v[u] & 0xFF) * q;
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
        for (int s = 0; s < SPL; ++s) {
            const int k = lane + kWave * s;
            if (k < ns) Yt[k * ys + pl] = MIXED ? acc[s] + cmp[s] : acc[s];
        }
    }
    __syncthreads();
    for (int e = lane; e < ns * tp; e += kWave) {
        const int k = e / tp, c = e - k * tp;
        if (c < npts) wdot[(int64_t)k * ld + i0 + c] = Yt[k * ys + c];
    }
    __syncthreads();  // the LDS tile may be reused by the next tile
}

template <bool MIXED, int SPL>
__global__ __launch_bounds__(kWave) void rates_kernel(MechDev m, int64_t n,
                                                      const double *__restrict__ T,
                                                      const double *__restrict__ P,
                                                      const double *__restrict__ Y,
                                                      double *__restrict__ wdot, int tp)
{
    const int64_t i0 = (int64_t)blockIdx.x * tp;
    rates_tile<MIXED, SPL>(m, n, i0, (int)min((int64_t)tp, n - i0), tp, T, P, Y, wdot);
}

// Batched requests: workgroups take tiles from a shared counter until the
// batch's tiles are exhausted (every workgroup exits once the counter passes
// the tile count).  Tile t belongs to the last item whose first tile is <= t.
template <bool MIXED, int SPL>
__global__ __launch_bounds__(kWave) void rates_batch_kernel(MechDev m,
                                                            const WorkList *__restrict__ wl,
                                                            int *__restrict__ counter, int tp)
{
    const int ntiles = wl->ntiles[0];
    for (;;) {
        int t = 0;
        if (threadIdx.x == 0) t = atomicAdd(counter, 1);
        t = __shfl(t, 0, kWave);
        if (t >= ntiles) break;
        int r = 0;
        while (r + 1 < wl->nitems && wl->start[0][r + 1] <= t) ++r;
        const WorkItem it = wl->items[r];
        const int64_t i0 = (int64_t)(t - wl->start[0][r]) * tp;
        rates_tile<MIXED, SPL>(m, it.n, i0, (int)min((int64_t)tp, it.n - i0), tp, it.T, it.p,
                               it.Y, it.wdot);
    }
}

size_t rates_lds_bytes(const MechDev &m, int tp)
{
    return sizeof(double) * (2 * (size_t)(m.ns + 1) + (m.chunk + 1) + (size_t)m.ns * (tp + 1));
}

}  // namespace

// Largest tile (16, 8 or 4 points per wave) whose LDS leaves room for at least
// eight waves per CU (160 KB of LDS).
int rates_tile_points(const MechDev &m)
{
    for (int cand : {16, 8, 4})
        if (rates_lds_bytes(m, cand) <= 20 * 1024) return cand;
    return 4;
}

namespace {
template <class K>
kx_status set_lds(K kern, size_t lds)
{
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute (rates)");
    return KX_OK;
}

// species per lane of the species and gather phases
int rates_spl(const MechDev &m) { return m.gpass <= 1 ? 1 : (m.gpass <= 2 ? 2 : 4); }
}  // namespace

kx_status launch_rates(const kx_mech *mech, int64_t n, const double *T, const double *p,
                       const double *Y, double *wdot, int precision, hipStream_t s)
{
    const MechDev &m = mech->dev;
    const int tp = rates_tile_points(m);
    const size_t lds = rates_lds_bytes(m, tp);
    if (lds > 160 * 1024)
        return fail(KX_EUNSUPPORTED, "production rates: mechanism too large for LDS");
    const int64_t nblk = (n + tp - 1) / tp;
    if (nblk > 0x7fffffff) return fail(KX_EINVAL, "production rates: n too large");
    const int spl = rates_spl(m);
    auto pick = [&](auto mixed) {
        constexpr bool M = decltype(mixed)::value;
        return spl == 1 ? rates_kernel<M, 1> : (spl == 2 ? rates_kernel<M, 2> : rates_kernel<M, 4>);
    };
    auto kern = precision == KX_MIXED ? pick(std::true_type{}) : pick(std::false_type{});
    kx_status st = set_lds(kern, lds);
    if (st != KX_OK) return st;
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(kWave), lds, s, m, n, T, p, Y, wdot,
                       tp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "rates kernel launch");
    return ok();
}

namespace {
auto pick_batch(const MechDev &m, int precision)
{
    const int spl = rates_spl(m);
    auto pick = [&](auto mixed) {
        constexpr bool M = decltype(mixed)::value;
        return spl == 1 ? rates_batch_kernel<M, 1>
                        : (spl == 2 ? rates_batch_kernel<M, 2> : rates_batch_kernel<M, 4>);
    };
    return precision == KX_MIXED ? pick(std::true_type{}) : pick(std::false_type{});
}
}  // namespace

kx_status prepare_rates_batch(const MechDev &m, int precision)
{
    const size_t lds = rates_lds_bytes(m, rates_tile_points(m));
    if (lds > 160 * 1024)
        return fail(KX_EUNSUPPORTED, "production rates: mechanism too large for LDS");
    return set_lds(pick_batch(m, precision), lds);
}

kx_status launch_rates_batch(const MechDev &m, const WorkList *wl, int *counter, int precision,
                             int grid, hipStream_t s)
{
    const int tp = rates_tile_points(m);
    const size_t lds = rates_lds_bytes(m, tp);
    hipLaunchKernelGGL(pick_batch(m, precision), dim3(grid), dim3(kWave), lds, s, m, wl,
                       counter, tp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "rates batch kernel launch");
    return ok();
}

}  // namespace kx
