// kx_rates.hip -- species net production rates on gfx950.
//
// Work decomposition.  A workgroup is one wave that owns a tile of `tp`
// consecutive points (8; 2 above 128 species): the tile's T and p are read
// first, the tile of Y is staged through LDS with coalesced row loads, and the
// same LDS tile later receives wdot and is written back with coalesced row
// stores.  The wave takes the tile's points four at a time (two above 128
// species) and runs three phases per step, with lanes spread over species,
// then (reaction, point) pairs, then species again:
//
//  1. species (lane = k, every point of the step): C_k, the Gibbs energy
//     g_k = G_k/RT of eq:Ck (range by T_mid; both ranges' coefficients read
//     once per step from a by-field table), a_k = (p_atm/RT) exp(-g_k) and
//     b_k = C_k / a_k into LDS as one 16-byte pair per species and point.
//     With these, prod_k C_k^nu' = A' B' and prod_k C_k^nu'' / K_c = A' B''
//     (A' = prod_reac a^nu', B' = prod_reac b^nu', B'' = prod_prod b^nu''), since
//     K_c = prod_k a_k^(nu''-nu') by eq:K_p and K_c = K_p (p_atm/RT)^(sum nu).
//     So K_c needs one exponential per species instead of one per reaction and
//     the rate of progress needs no division:
//         R_i = c_i k_f A' (B' - B'')                   (eq:r_i, eq:c_i)
//     and B' - B'' is the near-equilibrium difference, formed in FP64.
//  2. reactions (lanes 2r, 2r+1 = reaction r, each at half of the step's
//     points): k_f (eq:arrhenius, with the beta = E_R = 0 shortcut of eq:k_f),
//     [X]_i, the Lindemann / Troe factor (eq:blend) and R_i into LDS, one
//     chunk of reactions at a time; the 48-byte record is read and decoded
//     once per two rates of progress, a third-body reaction's efficiency data
//     loaded with it.  Reactions are sorted heaviest type first, so the
//     falloff code runs for 32 reactions per 64-lane iteration.  Each reaction
//     side is three molecule slots (unused ones hit a dummy species with
//     a = b = 1), so the products A', B', B'' are branch-free.
//  3. species (lane = k, every point of the step): wdot_k = sum_i nu_ki R_i
//     gathered from species-major lists of R slots (a net |nu| of 2 or 3 is
//     listed that many times); one 16-byte LDS read returns R_i at two points.
//     With four points per step a species has one list, each entry's sign in
//     its bit 31; with two, separate +R and -R lists.  The summation order is
//     fixed, so results are deterministic; the mixed path adds each two list
//     groups' sum with one Neumaier-compensated step.
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

// exp(x) for the mixed path: the argument stays in FP64, is reduced by n ln 2
// in FP64 and only exp(r), |r| <= ln2/2, is evaluated in FP32.
__device__ __forceinline__ double exp_mixed(double x)
{
    const double nd = rint(x * 1.4426950408889634);
    const double r = fma(-nd, 6.93147180559945286e-01, x);
    const float er = __expf((float)r);
    return ldexp((double)er, (int)nd);
}

// The falloff data of a reaction: k_0's Arrhenius parameters and the blend
// parameters (loaded with the third-body data, for the same reason).
struct Falloff {
    double lnA0, beta0, ER0;
    double fp[5];
    int has_T2;
};

__device__ __forceinline__ Falloff load_falloff(const DevAux &ax)
{
    Falloff f;
    f.lnA0 = ax.lnA0;
    f.beta0 = ax.beta0;
    f.ER0 = ax.ER0;
#pragma unroll
    for (int e = 0; e < 5; ++e) f.fp[e] = ax.fp[e];
    f.has_T2 = ax.has_T2;
    return f;
}

// Falloff blending factor F (eq:blend), Troe and SRI in one code path (so a
// wave mixing the two runs it once):
//   Troe  log10 F = log10 F_cent / (1 + f1^2), f1 = (l + c) / (n - 0.14 (l + c)),
//         F_cent = (1 - alpha) e^(-T/T***) + alpha e^(-T/T*) [+ e^(-T**/T)],
//         c = -0.4 - 0.67 log10 F_cent, n = 0.75 - 1.27 log10 F_cent;
//   SRI   F = d T^e B^X, B = a e^(-b/T) + e^(-T/c), X = 1 / (1 + l^2),
// with l = log10 P_r.  Both are ln F = ln B / (1 + w^2) + extra, where B is
// F_cent or the SRI bracket, w = f1 or l, and extra = 0 or ln d + e ln T.  The
// base-10 logarithms are formed from natural ones.
__device__ __forceinline__ double blend_F64(const Falloff &ax, bool sri, double T, double lnT,
                                            double invT, double lnPr)
{
    constexpr double kInvLn10 = 0.43429448190325182765;
    const double a0 = ax.fp[0], a1 = ax.fp[1], a2 = ax.fp[2], a3 = ax.fp[3], a4 = ax.fp[4];
    double B = (sri ? a0 : 1.0 - a0) * kexp(-a1 * (sri ? invT : T)) +
               (sri ? 1.0 : a0) * kexp(-T * a2);
    if (!sri && ax.has_T2) B += kexp(-a3 * invT);
    const double lnB = kln(fmax(B, DBL_MIN));
    const double lB = lnB * kInvLn10;
    const double x = fma(lnPr, kInvLn10, sri ? 0.0 : fma(-0.67, lB, -0.4));
    const double nn = sri ? 1.0 : fma(-1.27, lB, 0.75);
    const double w = x * krcp(fma(sri ? 0.0 : -0.14, x, nn));
    return kexp(fma(lnB, krcp(fma(w, w, 1.0)), sri ? fma(a4, lnT, a3) : 0.0));
}

// The same in FP32 from l = log10 P_r (computed by the caller without overflow).
__device__ __forceinline__ float blend_F32(const Falloff &ax, bool sri, float T, float lnT,
                                           float invT, float lPr)
{
    const float a0 = (float)ax.fp[0], a1 = (float)ax.fp[1], a2 = (float)ax.fp[2];
    const float a3 = (float)ax.fp[3], a4 = (float)ax.fp[4];
    float B = (sri ? a0 : 1.0f - a0) * __expf(-a1 * (sri ? invT : T)) +
              (sri ? 1.0f : a0) * __expf(-T * a2);
    if (!sri && ax.has_T2) B += __expf(-a3 * invT);
    const float lnB = __logf(fmaxf(B, FLT_MIN));
    const float lB = lnB * 0.43429448190325182765f;
    const float x = lPr + (sri ? 0.0f : -0.4f - 0.67f * lB);
    const float nn = sri ? 1.0f : 0.75f - 1.27f * lB;
    const float w = x / (nn - (sri ? 0.0f : 0.14f) * x);
    return __expf(lnB / (1.0f + w * w) + (sri ? a4 * lnT + a3 : 0.0f));
}

// Exponent ln k_f of a pressure-table reaction at ln p: linear in ln p between
// the neighbouring reference pressures, the nearest end point's value outside
// them (App. A.2, pressure-dependent reactions).
__device__ __forceinline__ double plog_exponent(const DevPlog *pl, int cnt, double lnT,
                                                double invT, double lnp)
{
    int j = 0;
    while (j + 1 < cnt && pl[j + 1].lnp <= lnp) ++j;
    const DevPlog &a = pl[j];
    const double x1 = fma(a.beta, lnT, fma(-a.ER, invT, a.lnA));
    if (j + 1 >= cnt || lnp <= a.lnp) return x1;
    const DevPlog &b = pl[j + 1];
    const double x2 = fma(b.beta, lnT, fma(-b.ER, invT, b.lnA));
    return fma(x2 - x1, (lnp - a.lnp) * a.inv_dlnp, x1);
}

// log10 of a positive double over its whole range, in FP32 arithmetic.
__device__ __forceinline__ float log10_wide(double v)
{
    int ex;
    const double mant = frexp(fmax(v, DBL_MIN), &ex);
    return (__log2f((float)mant) + (float)ex) * 0.30102999566398120f;
}

// Per-point factors of one species in LDS: {a_k, b_k}, 16 bytes, aligned so
// that one 16-byte LDS read fetches a pair (as two 8-byte halves it costs the
// LDS about twice the cycles).
struct alignas(16) Pair {
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

// The third-body data of a reaction: the default efficiency, the inline
// efficiencies (alpha - default) and their LDS offsets, and the count of
// further ones.  Loaded as one batch as soon as the reaction record is decoded,
// so that its memory latency overlaps the Arrhenius exponentials (loaded where
// the sum is formed, each of its dependent batches stalls the wave).
struct ThirdBody {
    double def;
    double dalpha[kInlineEff];
    unsigned eoff2[kInlineEff / 2];  // two 16-bit offsets per word (unpacked where used)
    int ext_off, ext_cnt;
};

__device__ __forceinline__ ThirdBody load_third_body(const DevAux &ax)
{
    ThirdBody t;
    t.def = ax.eff_default;
#pragma unroll
    for (int e = 0; e < kInlineEff; ++e) t.dalpha[e] = ax.dalpha[e];
    const unsigned *eo = reinterpret_cast<const unsigned *>(ax.eoff);
#pragma unroll
    for (int e = 0; e < kInlineEff / 2; ++e) t.eoff2[e] = eo[e];
    t.ext_off = ax.ext_off;
    t.ext_cnt = ax.ext_cnt;
    return t;
}

// [X]_i = default [M] + sum over listed species of (alpha - default) C_k.
__device__ __forceinline__ double third_body(const MechDev &m, const ThirdBody &tb,
                                             const char *__restrict__ pb, double Mconc)
{
    double X = tb.def * Mconc;
    // the reads are issued four at a time (left to itself the scheduler waits
    // for each read in turn; eight in flight would cost registers)
#pragma unroll
    for (int e0 = 0; e0 < kInlineEff; e0 += 4) {
        Pair s[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ee = e0 + e;
            s[e] = load_pair(pb, (tb.eoff2[ee / 2] >> (16 * (ee & 1))) & 0xFFFFu);
        }
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) X = fma(tb.dalpha[e0 + e], s[e].a * s[e].b, X);
    }
    for (int e = 0; e < tb.ext_cnt; ++e) {
        const DevEff f = m.eff[tb.ext_off + e];
        const Pair s = load_pair(pb, 16 * f.sp);
        X = fma(f.dalpha, s.a * s.b, X);
    }
    return X;
}

// The per-point values phase 2 needs.
struct PtVals {
    double T, lnT, invT, M, lnp;
};

// Rates of progress R_i = c_i k_f A' (B' - B'') of one reaction at the NPT
// points of this lane (lane-private).  The record is decoded once; the LDS
// reads of every point are issued before the first exponential, and the
// points' exponentials are independent, so their chains interleave.
template <bool MIXED, int NPT>
__device__ __forceinline__ void rates_of_progress(const MechDev &m, const RxnWords &w,
                                                  const char *const (&pb)[NPT],
                                                  const PtVals (&q)[NPT], double (&R)[NPT])
{
    const double lnA = as_double(w.w0.x, w.w0.y);
    const double beta = as_double(w.w0.z, w.w0.w);
    const double ER = as_double(w.w1.x, w.w1.y);
    const double A = as_double(w.w1.z, w.w1.w);
    const unsigned type = w.w2.w & 0xFFu;
    const unsigned flags = (w.w2.w >> 8) & 0xFFu;
    const unsigned aux = w.w2.w >> 16;
    const unsigned o0 = w.w2.x & 0xFFFFu, o1 = w.w2.x >> 16;
    const unsigned o3 = w.w2.y >> 16, o4 = w.w2.z & 0xFFFFu;

    const bool has_tb = type != KX_RXN_ELEMENTARY && type != KX_RXN_PLOG;
    const bool has_fo = has_tb && type != KX_RXN_THREEBODY;
    ThirdBody tb;
    Falloff fo;
    if (has_tb) tb = load_third_body(m.aux[aux]);

    // exponent of k_f (eq:k_f); k_f = A without an exponential when beta = E_R = 0
    // (such reactions are sorted together, so the branch is mostly wave-uniform),
    // or interpolated in ln p for a pressure-table reaction
    const bool kconst = (flags & kFlagKfConst) != 0;
    double xf[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j)
        xf[j] = kconst ? lnA : fma(beta, q[j].lnT, fma(-ER, q[j].invT, lnA));
    if (type == KX_RXN_PLOG) {
        const DevAux &ax = m.aux[aux];
#pragma unroll
        for (int j = 0; j < NPT; ++j)
            xf[j] = plog_exponent(m.plog + ax.plog_off, ax.plog_cnt, q[j].lnT, q[j].invT,
                                  q[j].lnp);
    }
    // the LDS reads go before the exponentials so that their latency hides behind them
    Pair r0[NPT], r1[NPT];
    double bp0[NPT], bp1[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        r0[j] = load_pair(pb[j], o0);
        r1[j] = load_pair(pb[j], o1);
        bp0[j] = load_b(pb[j], o3);
        bp1[j] = load_b(pb[j], o4);
    }
    double kf[NPT], Ap[NPT], Bp[NPT], Bpp[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        kf[j] = A;
        if (!kconst) kf[j] = MIXED ? exp_mixed(xf[j]) : kexp(xf[j]);
    }
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        Ap[j] = r0[j].a * r1[j].a;
        Bp[j] = r0[j].b * r1[j].b;
        Bpp[j] = bp0[j] * bp1[j];
    }
    // third molecule slots: skipped by the whole wave when none of its
    // reactions has three molecules on a side (the dummy species gives 1)
    const unsigned o2 = w.w2.y & 0xFFFFu, o5 = w.w2.z >> 16;
    const unsigned dummy = 16u * (unsigned)m.ns;
    if (__builtin_amdgcn_ballot_w64(o2 != dummy || o5 != dummy) != 0) {
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const Pair r2 = load_pair(pb[j], o2);
            Ap[j] *= r2.a;
            Bp[j] *= r2.b;
            Bpp[j] *= load_b(pb[j], o5);
        }
    }
    if (flags & kFlagOrders) {
        // explicit forward orders (irreversible): prod_k C_k^o_k, C_k = a_k b_k
        const DevAux &ax = m.aux[aux];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            double s = 0.0;
            bool zero = false;
#pragma unroll
            for (int e = 0; e < kMaxOrd; ++e) {
                const double o = ax.oval[e];
                if (o != 0.0) {
                    const Pair qq = load_pair(pb[j], ax.ooff[e]);
                    const double C = qq.a * qq.b;
                    zero = zero || !(C > 0.0);
                    s = fma(o, kln(fmax(C, DBL_MIN)), s);
                }
            }
            Ap[j] = zero ? 0.0 : kexp(s);
            Bp[j] = 1.0;
            Bpp[j] = 0.0;
        }
    }
    double c[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) c[j] = 1.0;
    if (has_tb) {
        // FP64: the falloff data is read before the third-body sums, whose LDS
        // reads and products then cover its memory latency (the mixed path
        // reads it where it is used: the earlier read measured slower there)
        if (!MIXED && has_fo) fo = load_falloff(m.aux[aux]);
        double X[NPT];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            X[j] = third_body(m, tb, pb[j], q[j].M);
            c[j] = X[j];
        }
        if (has_fo) {
            if (MIXED) fo = load_falloff(m.aux[aux]);
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                // P_r = k_0 [X] / k_inf = e0 [X] with e0 = exp(x_0 - x_inf) (no division)
                const double d0 =
                    fma(fo.beta0, q[j].lnT, fma(-fo.ER0, q[j].invT, fo.lnA0)) - xf[j];
                const double e0 = MIXED ? exp_mixed(d0) : kexp(d0);
                const double Pr = e0 * X[j];
                double F = 1.0;
                if (type == KX_RXN_TROE || type == KX_RXN_SRI) {
                    const bool sri = type == KX_RXN_SRI;
                    if (MIXED) {
                        F = (double)blend_F32(fo, sri, (float)q[j].T, (float)q[j].lnT,
                                              (float)q[j].invT, log10_wide(Pr));
                    } else {
                        // ln max(P_r, DBL_MIN) without forming the logarithm of P_r
                        const double lnPr =
                            fmax(d0 + kln(fmax(X[j], DBL_MIN)), -708.39641853226410622);
                        F = blend_F64(fo, sri, q[j].T, q[j].lnT, q[j].invT, lnPr);
                    }
                }
                // eq:c_i: P_r/(1+P_r) F; chemically activated: F/(1+P_r) with k_0 =
                // e0 k_inf in r_i, i.e. c k_inf = e0 F/(1+P_r) k_inf
                const double g = krcp(1.0 + Pr) * F;
                c[j] = (flags & kFlagChemAct) ? e0 * g : Pr * g;
            }
        }
    }
    const double rev = (flags & kFlagReversible) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < NPT; ++j) R[j] = c[j] * kf[j] * Ap[j] * fma(-rev, Bpp[j], Bp[j]);
}

// Gibbs energy g = G/RT of one species at one temperature (eq:Ck with the
// coefficients pre-scaled: g = c0 (1 - ln T) + c1 T + ... + c4 T^4 + c5 / T + c6).
__device__ __forceinline__ double gibbs(const double (&g)[7], double T, double lnT, double invT)
{
    const double poly = T * fma(T, fma(T, fma(T, g[4], g[3]), g[2]), g[1]);
    return fma(g[0], 1.0 - lnT, poly) + fma(g[5], invT, g[6]);
}

template <bool MIXED>
__device__ __forceinline__ void accumulate(double &acc, double &cmp, double t)
{
    if (MIXED) {
        const double sum = acc + t;
        cmp += (fabs(acc) >= fabs(t)) ? (acc - sum) + t : (t - sum) + acc;
        acc = sum;
    } else {
        acc += t;
    }
}

// Two groups' partial sums ga, gb per trip of a gather loop: FP64 adds each to
// the running sum as it is formed (first_of_pair, then second_of_pair); the
// mixed path adds their sum with one compensated step (the two groups' plain
// sum carries FP64 rounding, far below the mixed path's error).
template <bool MIXED, int PS>
__device__ __forceinline__ void first_of_pair(double (&acc)[PS], const double (&ga)[PS])
{
    if (!MIXED) {
#pragma unroll
        for (int j = 0; j < PS; ++j) acc[j] += ga[j];
    }
}

template <bool MIXED, int PS>
__device__ __forceinline__ void second_of_pair(double (&acc)[PS], double (&cmp)[PS],
                                               const double (&ga)[PS], const double (&gb)[PS])
{
#pragma unroll
    for (int j = 0; j < PS; ++j) {
        if (MIXED)
            accumulate<true>(acc[j], cmp[j], ga[j] + gb[j]);
        else
            acc[j] += gb[j];
    }
}

// Points per workgroup tile: 8 (64-byte row segments of Y and wdot; tiles that
// share a 128-byte line run on the same XCD, see xcd_tile); 2 for mechanisms
// of more than 128 species, whose Y tile would otherwise crowd the LDS.
__host__ __device__ constexpr int rates_tile_points_for(int spl) { return spl == 4 ? 2 : 8; }

// Points per step: four for mechanisms of up to 128 species (each lane of the
// reaction phase evaluates its reaction at two points, so a reaction record is
// read and decoded once per two rates of progress), two above (the per-point
// LDS arrays of a 4-point step would crowd the LDS).
__host__ __device__ constexpr int rates_step_points_for(int spl) { return spl == 4 ? 2 : 4; }

// Byte distance between the two halves of the rate-of-progress array of a
// 4-point step: slot s of the chunk holds R at points 0 and 1 at 16 s and at
// points 2 and 3 at kSqHalf + 16 s, so one gather offset addresses both halves
// (the second through the LDS instruction's immediate offset).
constexpr int kSqHalf = 16 * (kChunkMax + 1);

// Per-point constants of a tile, computed once per point (lane = point).
struct PointConst {
    double T, lnT, invT, M;  // temperature, ln T, 1/T, [M] = p / RT
    double P0, cf;           // p_atm / RT; C_k = Y_k / W_k * cf with cf = [M] W-bar
    double lnp, pad;         // ln p (pressure-table reactions)
};

// LDS layout of one workgroup (one wave), PS = points per step:
//   sq    rates of progress of the current chunk for the points of a step:
//         PS = 2: [chunk + 1][2], the two points side by side;
//         PS = 4: two such arrays kSqHalf bytes apart (points 0, 1 and 2, 3);
//         slot `chunk` is zero and absorbs the gather padding; at byte 0 so that
//         the gather offsets are LDS addresses
//   pairs [PS][ns + 1] {a, b} per point (entry ns is the dummy species, {1, 1})
//   pc    [tp]              PointConst of the tile's points
//   Yt    [ns][tp + 1]      Y tile in, wdot tile out (coalesced row loads/stores)
// One tile of `npts` (<= tp) points starting at point i0 of arrays whose
// species rows have stride ld, PS points per step:
//   phase 1 -- lane = species, every point of the step;
//   phase 2 -- lane = (reaction, point): lanes 2r and 2r+1 take reaction r, lane
//              2r + j for the points j (and j + 2 when PS = 4) of the step, so a
//              group of 32 falloff reactions fills a whole 64-lane iteration;
//   phase 3 -- lane = species: one 16-byte LDS read per list entry (two when
//              PS = 4) returns the rate of progress of the reaction at the points.
// A 16-byte LDS read at a byte address (the gather lists hold addresses
// relative to the dynamic LDS, which starts at 0 when the kernel has no static
// LDS; rates_tile<..., true> is only entered after checking that).
__device__ __forceinline__ double2 lds_read16(unsigned addr)
{
    typedef double v2d __attribute__((ext_vector_type(2)));
    const v2d v = *(const __attribute__((address_space(3))) v2d *)(size_t)addr;
    return make_double2(v.x, v.y);
}

__device__ __forceinline__ unsigned lds_base()
{
    extern __shared__ double lds[];
    return (unsigned)(size_t)(__attribute__((address_space(3))) double *)lds;
}

// ---- phase 3: wdot_k = sum_i nu_ki R_i for the PS points of a step, one
// chunk of reactions.  Lane = species (SPL per lane); a group is eight list
// entries, summed plainly per point (the mixed path compensates the running
// sum once per two groups).  All reads of a group (or of each half of it, for four
// points) are issued before the first sum (left to itself the scheduler waits
// for each read in turn), and two groups are handled per trip with
// alternating offset registers (the next group's offsets in flight).
//
// gather_signed: one list per species with the sign of each entry in bit 31,
// turned into the factor +-1 of an exact FMA (used with four points per step,
// where the +q and -q lists padded separately cost a third more reads).
template <bool MIXED, int SPL, bool DIRECT, int PS>
__device__ __forceinline__ void gather_signed(const MechDev &m, int c, int gw, int lane,
                                              const char *qb, double (&acc)[SPL][PS],
                                              double (&cmp)[SPL][PS])
{
    const int ngrp = m.gmgrp[c];
    const uint4 *ge = m.gment + ((size_t)m.gmoff[c] * gw + lane) * 2;
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
        const uint4 *g = ge + 2 * kWave * s;
        auto group = [&](const uint4 &v0, const uint4 &v1, double (&gs)[PS]) {
            const unsigned raw[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
            for (int h = 0; h < PS / 2; ++h) {
                double2 q2[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const unsigned off = raw[u] & 0x7fffffffu;
                    q2[u] = DIRECT ? lds_read16(off + h * kSqHalf)
                                   : *reinterpret_cast<const double2 *>(qb + off + h * kSqHalf);
                }
                __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);  // DS reads
                __builtin_amdgcn_sched_group_barrier(0x002, 24, 0);  // VALU
                auto sgn = [&](int u) {
                    return __hiloint2double((int)((raw[u] & 0x80000000u) | 0x3ff00000u), 0);
                };
                double g0 = q2[0].x * sgn(0), g1 = q2[0].y * sgn(0);
#pragma unroll
                for (int u = 1; u < 8; ++u) {
                    const double sg = sgn(u);
                    g0 = fma(q2[u].x, sg, g0);
                    g1 = fma(q2[u].y, sg, g1);
                }
                gs[2 * h] = g0;
                gs[2 * h + 1] = g1;
            }
        };
        uint4 a0 = make_uint4(0, 0, 0, 0), a1 = a0, b0 = a0, b1 = a0;
        if (ngrp > 0) {
            a0 = g[0];
            a1 = g[1];
        }
        int it = 0;
        for (; it + 1 < ngrp; it += 2) {
            b0 = g[(size_t)(it + 1) * 2 * gw];
            b1 = g[(size_t)(it + 1) * 2 * gw + 1];
            double ga[PS], gb[PS];
            group(a0, a1, ga);
            first_of_pair<MIXED, PS>(acc[s], ga);
            if (it + 2 < ngrp) {
                a0 = g[(size_t)(it + 2) * 2 * gw];
                a1 = g[(size_t)(it + 2) * 2 * gw + 1];
            }
            group(b0, b1, gb);
            second_of_pair<MIXED, PS>(acc[s], cmp[s], ga, gb);
        }
        if (it < ngrp) {
            double ga[PS];
            group(a0, a1, ga);
#pragma unroll
            for (int j = 0; j < PS; ++j) accumulate<MIXED>(acc[s][j], cmp[s][j], ga[j]);
        }
    }
}

// gather_split: a +q list and a -q list per species, each padded to whole
// groups (the group's sum is negated for the -q groups); two points per step.
template <bool MIXED, int SPL, bool DIRECT, int PS>
__device__ __forceinline__ void gather_split(const MechDev &m, int c, int gw, int lane,
                                             const char *qb, double (&acc)[SPL][PS],
                                             double (&cmp)[SPL][PS])
{
    const int npos = m.gpos[c], ngrp = npos + m.gneg[c];
    const uint4 *ge = m.gent + ((size_t)m.goff[c] * gw + lane) * 2;
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
        const uint4 *g = ge + 2 * kWave * s;
        auto group = [&](const uint4 &v0, const uint4 &v1, int it, double (&gs)[PS]) {
            const unsigned off[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
            double2 q2[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                q2[u] = DIRECT ? lds_read16(off[u])
                               : *reinterpret_cast<const double2 *>(qb + off[u]);
            __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);  // DS reads
            __builtin_amdgcn_sched_group_barrier(0x002, 16, 0);  // VALU
            double g0 = q2[0].x, g1 = q2[0].y;
#pragma unroll
            for (int u = 1; u < 8; ++u) {
                g0 += q2[u].x;
                g1 += q2[u].y;
            }
            if (it >= npos) {
                g0 = -g0;
                g1 = -g1;
            }
            gs[0] = g0;
            gs[1] = g1;
        };
        uint4 a0 = make_uint4(0, 0, 0, 0), a1 = a0, b0 = a0, b1 = a0;
        if (ngrp > 0) {
            a0 = g[0];
            a1 = g[1];
        }
        int it = 0;
        for (; it + 1 < ngrp; it += 2) {
            b0 = g[(size_t)(it + 1) * 2 * gw];
            b1 = g[(size_t)(it + 1) * 2 * gw + 1];
            double ga[PS], gb[PS];
            group(a0, a1, it, ga);
            first_of_pair<MIXED, PS>(acc[s], ga);
            if (it + 2 < ngrp) {
                a0 = g[(size_t)(it + 2) * 2 * gw];
                a1 = g[(size_t)(it + 2) * 2 * gw + 1];
            }
            group(b0, b1, it + 1, gb);
            second_of_pair<MIXED, PS>(acc[s], cmp[s], ga, gb);
        }
        if (it < ngrp) {
            double ga[PS];
            group(a0, a1, it, ga);
#pragma unroll
            for (int j = 0; j < PS; ++j) accumulate<MIXED>(acc[s][j], cmp[s][j], ga[j]);
        }
    }
}

// `lane` is threadIdx.x; the batch kernel passes it through an opaque move in
// each trip of its tile loop, so that the tile's lane-dependent addresses are
// not hoisted out of the loop (kept live across tiles they cost registers).
template <bool MIXED, int SPL, bool DIRECT>
__device__ __forceinline__ void rates_tile(int lane, const MechDev &m, int64_t ld, int64_t i0,
                                           int npts,
                                           int tp, const double *__restrict__ T,
                                           const double *__restrict__ P,
                                           const double *__restrict__ Y,
                                           double *__restrict__ wdot)
{
    extern __shared__ double lds[];
    constexpr int TP = rates_tile_points_for(SPL);  // == tp
    constexpr int PS = rates_step_points_for(SPL);  // points per step
    constexpr int NPT = PS / 2;                     // points per lane in phase 2
    constexpr int NGW = kWave / TP;                 // species groups of the W-bar pass
    const int ns = m.ns;
    const int ys = TP + 1;
    double *sq = lds;
    double *pairs = sq + (PS == 4 ? 2 * kSqHalf / 8 : 2 * (m.chunk + 1));
    PointConst *pc = reinterpret_cast<PointConst *>(pairs + 2 * PS * (ns + 1));
    double *Yt = reinterpret_cast<double *>(pc + TP);
    const char *qb = reinterpret_cast<const char *>(sq);
    (void)tp;

    // the temperature and pressure of the tile's points are read first, so
    // that their memory latency overlaps the Y tile's
    double Tl = 0.0, Pl = 0.0;
    if (lane < TP) {
        const int64_t i = i0 + min(lane, npts - 1);
        Tl = T[i];
        Pl = P[i];
    }
    // the tile's Y, eight row loads per lane in flight before the first LDS
    // store (a loop of load-wait-store would pay one memory latency per row)
    constexpr int kLd = 8;
    for (int e0 = lane; e0 < ns * TP; e0 += kLd * kWave) {
        double v[kLd];
#pragma unroll
        for (int u = 0; u < kLd; ++u) {
            const int e = e0 + u * kWave, k = e / TP, c = e % TP;
            v[u] = (e < ns * TP && c < npts) ? Y[(int64_t)k * ld + i0 + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kLd; ++u) {
            const int e = e0 + u * kWave;
            if (e < ns * TP) Yt[(e / TP) * ys + e % TP] = v[u];
        }
    }
    __syncthreads();
    {
        // sum_k Y_k / W_k = 1 / W-bar: lane = (point, species group); the
        // group partials meet in the (still unused) rate-of-progress array.
        // The 1/W_k of eight species are loaded before they are used.
        const int c = lane % TP, g = lane / TP;
        const int cc = min(c, npts - 1);  // padding points repeat the last one
        double part = 0.0;
        for (int k0 = g; k0 < ns; k0 += kLd * NGW) {
            double iw[kLd];
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int k = k0 + u * NGW;
                iw[u] = k < ns ? m.gsoa[((size_t)(k / kWave) * 16 + 15) * kWave + k % kWave] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kLd; ++u) {
                const int k = k0 + u * NGW;
                if (k < ns) part = fma(Yt[k * ys + cc], iw[u], part);
            }
        }
        sq[g * TP + c] = part;
    }
    __syncthreads();
    if (lane < TP) {
        double wsum = 0.0;
#pragma unroll
        for (int g = 0; g < NGW; ++g) wsum += sq[g * TP + lane];
        PointConst q;
        q.T = Tl;
        q.lnT = kln(q.T);
        q.invT = krcp(q.T);
        const double invRT = krcp(kRu * q.T);
        q.M = Pl * invRT;
        q.P0 = kPatm * invRT;
        q.cf = q.M * krcp(wsum);
        q.lnp = kln(Pl);
        q.pad = 0.0;
        pc[lane] = q;
    }
    __syncthreads();
    if (lane < PS) {
        pairs[2 * ns + 2 * (ns + 1) * lane] = 1.0;
        pairs[2 * ns + 2 * (ns + 1) * lane + 1] = 1.0;
    }
    if (lane < 2) {
        sq[2 * m.chunk + lane] = 0.0;
        if (PS == 4) sq[kSqHalf / 8 + 2 * m.chunk + lane] = 0.0;
    }

    const int jl = lane & 1;   // point of this lane in phase 2 (and jl + 2)
    const int rl = lane >> 1;  // reaction slot of this lane in phase 2
    const char *pbl[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j)
        pbl[j] = reinterpret_cast<const char *>(pairs + 2 * (ns + 1) * (jl + 2 * j));
    const int gw = kWave * m.gpass;
    for (int pl = 0; pl < npts; pl += PS) {
        // ---- phase 1: species (every point of the step per lane)
        PointConst ps[PS];
#pragma unroll
        for (int j = 0; j < PS; ++j) ps[j] = pc[pl + j];
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            const int k = lane + kWave * s;
            if (k < ns) {
                // both temperature ranges' coefficients are read once per step
                // and selected per point (one read per point would cost the
                // vector-memory unit four times as many loads), from the
                // by-field table (a wave's read is one contiguous row)
                const double *gs = m.gsoa + (size_t)s * 16 * kWave + lane;
                // the same rows every step: read them per step (kept in
                // registers across the steps they would cost spills)
                asm volatile("" : "+v"(gs));
                double glo[7], ghi[7];
#pragma unroll
                for (int e = 0; e < 7; ++e) {
                    glo[e] = gs[e * kWave];
                    ghi[e] = gs[(7 + e) * kWave];
                }
                const double tmid = gs[14 * kWave], iw = gs[15 * kWave];
#pragma unroll
                for (int j = 0; j < PS; ++j) {
                    const PointConst &q = ps[j];
                    double g[7];
                    const bool lo = q.T < tmid;
#pragma unroll
                    for (int e = 0; e < 7; ++e) g[e] = lo ? glo[e] : ghi[e];
                    const double ak = q.P0 * kexp(-gibbs(g, q.T, q.lnT, q.invT));
                    const double Ck = Yt[k * ys + pl + j] * iw * q.cf;
                    double *pr = pairs + 2 * (ns + 1) * j + 2 * k;
                    pr[0] = ak;
                    pr[1] = Ck * krcp(ak);
                }
            }
        }
        wave_sync();
        // the points of this lane in phase 2
        PtVals qv[NPT];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const PointConst &q = pc[pl + jl + 2 * j];  // LDS (a lane-dependent index)
            qv[j] = PtVals{q.T, q.lnT, q.invT, q.M, q.lnp};
        }

        // ---- phases 2 and 3, one chunk of reactions at a time
        double acc[SPL][PS], cmp[SPL][PS];
#pragma unroll
        for (int s = 0; s < SPL; ++s)
#pragma unroll
            for (int j = 0; j < PS; ++j) acc[s][j] = cmp[s][j] = 0.0;
        for (int c = 0; c < m.nchunks; ++c) {
            const int base = c * m.chunk;
            const int cnt = min(m.chunk, m.nr - base);
            // 48-byte reaction records as three 16-byte loads, the next
            // iteration's record in flight while this one is evaluated
            const uint4 *rsrc = reinterpret_cast<const uint4 *>(m.rxn + base);
            RxnWords w;
            w.w0 = w.w1 = w.w2 = make_uint4(0, 0, 0, 0);
            if (rl < cnt) {
                w.w0 = rsrc[3 * rl];
                w.w1 = rsrc[3 * rl + 1];
                w.w2 = rsrc[3 * rl + 2];
            }
            for (int r = rl; r < cnt; r += kWave / 2) {
                const RxnWords cur = w;
                const int rn = r + kWave / 2;
                if (rn < cnt) {
                    w.w0 = rsrc[3 * rn];
                    w.w1 = rsrc[3 * rn + 1];
                    w.w2 = rsrc[3 * rn + 2];
                }
                double R[NPT];
                rates_of_progress<MIXED, NPT>(m, cur, pbl, qv, R);
                sq[2 * r + jl] = R[0];
                if (PS == 4) sq[kSqHalf / 8 + 2 * r + jl] = R[NPT - 1];
            }
            wave_sync();
            if (PS == 4)
                gather_signed<MIXED, SPL, DIRECT, PS>(m, c, gw, lane, qb, acc, cmp);
            else
                gather_split<MIXED, SPL, DIRECT, PS>(m, c, gw, lane, qb, acc, cmp);
            wave_sync();
        }
        // the rates of progress were stored as points (0, 1) and (2, 3); the
        // accumulators follow the same order
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            const int k = lane + kWave * s;
            if (k < ns) {
#pragma unroll
                for (int j = 0; j < PS; ++j)
                    Yt[k * ys + pl + j] = MIXED ? acc[s][j] + cmp[s][j] : acc[s][j];
            }
        }
    }
    __syncthreads();
    for (int e = lane; e < ns * TP; e += kWave) {
        const int k = e / TP, c = e % TP;
        if (c < npts) wdot[(int64_t)k * ld + i0 + c] = Yt[k * ys + c];
    }
    __syncthreads();  // the LDS tile may be reused by the next tile
}

// Workgroups are dispatched to the eight XCDs round-robin (workgroup b runs on
// XCD b mod 8).  This bijection gives each XCD one contiguous range of tiles,
// so neighbouring tiles -- which share cache lines of Y and wdot -- meet in the
// same L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nblk)
{
    constexpr unsigned kXcd = 8;
    const unsigned x = b % kXcd, q = nblk / kXcd, r = nblk % kXcd;
    return x * q + min(x, r) + b / kXcd;
}

// DIRECT: the gather lists' offsets are LDS addresses, which holds when the
// kernel has no static LDS (its dynamic LDS then starts at address 0); the
// host checks the kernel's static LDS size and launches the DIRECT = false
// instance otherwise.
template <bool MIXED, int SPL, bool DIRECT>
__global__ __launch_bounds__(kWave, SPL == 1 ? 3 : 2) void rates_kernel(MechDev m, int64_t n,
                                                      const double *__restrict__ T,
                                                      const double *__restrict__ P,
                                                      const double *__restrict__ Y,
                                                      double *__restrict__ wdot, int tp)
{
    const int64_t i0 = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * tp;
    const int np = (int)min((int64_t)tp, n - i0);
    rates_tile<MIXED, SPL, DIRECT>(threadIdx.x, m, n, i0, np, tp, T, P, Y, wdot);
}

// Batched requests.  The batch's tiles are split into kXcds contiguous ranges,
// one per XCD (workgroup b runs on XCD b mod kXcds); a workgroup takes tiles
// of its own XCD's range from that range's counter (kTicketTiles consecutive
// tiles per ticket), so neighbouring tiles --
// which share cache lines of Y and wdot -- meet in the same L2 as in a direct
// launch, and then helps with the other ranges in turn.  Every workgroup
// exits after the last range is exhausted.  Tile t belongs to the last item
// whose first tile is <= t.
//
// Tiles per ticket: a ticket's atomic returns after the wave's next memory
// wait (the wait counter is in order), so each ticket costs the wave about one
// atomic round trip; four tiles per ticket spread it.
constexpr int kTicketTiles = 4;

template <bool MIXED, int SPL, bool DIRECT>
__global__ __launch_bounds__(kWave, SPL == 1 ? 3 : 2) void rates_batch_kernel(MechDev m,
                                                            const WorkList *__restrict__ wl,
                                                            int *__restrict__ counter, int tp)
{
    const int ntiles = wl->ntiles[0];
    const int x0 = (int)(blockIdx.x % kXcds);
    int r = 0;  // item of the previous tile
    for (int step = 0; step < kXcds; ++step) {
        const int x = (x0 + step) % kXcds;
        const int lo = (int)((int64_t)ntiles * x / kXcds);
        const int hi = (int)((int64_t)ntiles * (x + 1) / kXcds);
        int tn = 0;
        if (threadIdx.x == 0) tn = atomicAdd(counter + x, 1);
        int t0 = 0, k = kTicketTiles;  // tiles t0 .. t0 + kTicketTiles - 1 of a ticket
        for (;;) {
            if (k == kTicketTiles) {
                t0 = lo + kTicketTiles * __builtin_amdgcn_readfirstlane(tn);  // lane 0's ticket
                k = 0;
                // the next ticket is taken now, so its round trip overlaps these tiles
                if (t0 < hi && threadIdx.x == 0) tn = atomicAdd(counter + x, 1);
            }
            const int t = t0 + k++;
            if (t >= hi) break;
            r = work_item_of(wl, 0, t, r);
            const WorkItem it = wl->items[r];
            const int64_t i0 = (int64_t)(t - wl->start[0][r]) * tp;
            const int np = (int)min((int64_t)tp, it.n - i0);
            int lane;
            asm volatile("v_mov_b32 %0, %1" : "=v"(lane) : "v"((int)threadIdx.x));
            rates_tile<MIXED, SPL, DIRECT>(lane, m, it.n, i0, np, tp, it.T, it.p, it.Y, it.wdot);
        }
    }
}

// Batched requests, one tile per workgroup (grid = the batch's tiles, mapped
// to XCDs as in a direct launch; the item of tile t by work_item_ballot).
// Persistent workgroups that take tickets measured about a tenth slower per
// tile than this one-tile form.
template <bool MIXED, int SPL, bool DIRECT>
__global__ __launch_bounds__(kWave, SPL == 1 ? 3 : 2) void rates_items_kernel(
    MechDev m, const WorkList *__restrict__ wl, int tp)
{
    const int ntiles = wl->ntiles[0];
    const int t = (int)xcd_tile(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const int r = work_item_ballot(wl, 0, t);
    const WorkItem it = wl->items[r];
    const int64_t i0 = (int64_t)(t - wl->start[0][r]) * tp;
    const int np = (int)min((int64_t)tp, it.n - i0);
    rates_tile<MIXED, SPL, DIRECT>(threadIdx.x, m, it.n, i0, np, tp, it.T, it.p, it.Y, it.wdot);
}

size_t rates_lds_bytes(const MechDev &m, int tp)
{
    const int ps = rates_step_points_for(m.gpass);
    const size_t sq = ps == 4 ? 2 * (size_t)kSqHalf / 8 : 2 * (size_t)(m.chunk + 1);
    return sizeof(double) * (sq + 2 * (size_t)ps * (m.ns + 1) + 8 * (size_t)tp +
                             (size_t)m.ns * (tp + 1));
}

}  // namespace

int rates_tile_points(const MechDev &m) { return rates_tile_points_for(m.gpass); }

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

// The instance to launch: the DIRECT one when it has no static LDS.
template <class K>
K pick_direct(K direct, K indirect)
{
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, (const void *)direct) == hipSuccess && a.sharedSizeBytes == 0)
        return direct;
    return indirect;
}

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
        return spl == 1 ? pick_direct(rates_kernel<M, 1, true>, rates_kernel<M, 1, false>)
                        : (spl == 2 ? pick_direct(rates_kernel<M, 2, true>, rates_kernel<M, 2, false>)
                                    : pick_direct(rates_kernel<M, 4, true>, rates_kernel<M, 4, false>));
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
        return spl == 1
                   ? pick_direct(rates_batch_kernel<M, 1, true>, rates_batch_kernel<M, 1, false>)
                   : (spl == 2 ? pick_direct(rates_batch_kernel<M, 2, true>,
                                             rates_batch_kernel<M, 2, false>)
                               : pick_direct(rates_batch_kernel<M, 4, true>,
                                             rates_batch_kernel<M, 4, false>));
    };
    return precision == KX_MIXED ? pick(std::true_type{}) : pick(std::false_type{});
}
}  // namespace

namespace {
auto pick_items(const MechDev &m, int precision)
{
    const int spl = rates_spl(m);
    auto pick = [&](auto mixed) {
        constexpr bool M = decltype(mixed)::value;
        return spl == 1
                   ? pick_direct(rates_items_kernel<M, 1, true>, rates_items_kernel<M, 1, false>)
                   : (spl == 2 ? pick_direct(rates_items_kernel<M, 2, true>,
                                             rates_items_kernel<M, 2, false>)
                               : pick_direct(rates_items_kernel<M, 4, true>,
                                             rates_items_kernel<M, 4, false>));
    };
    return precision == KX_MIXED ? pick(std::true_type{}) : pick(std::false_type{});
}
}  // namespace

kx_status launch_rates_items(const MechDev &m, const WorkList *wl, int64_t ntiles, int precision,
                             hipStream_t s)
{
    if (ntiles <= 0) return ok();
    if (ntiles > 0x7fffffff) return fail(KX_EINVAL, "production rates: too many tiles");
    const int tp = rates_tile_points(m);
    const size_t lds = rates_lds_bytes(m, tp);
    if (lds > 160 * 1024)
        return fail(KX_EUNSUPPORTED, "production rates: mechanism too large for LDS");
    auto kern = pick_items(m, precision);
    kx_status st = set_lds(kern, lds);
    if (st != KX_OK) return st;
    hipLaunchKernelGGL(kern, dim3((unsigned)ntiles), dim3(kWave), lds, s, m, wl, tp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "rates items kernel launch");
    return ok();
}

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
