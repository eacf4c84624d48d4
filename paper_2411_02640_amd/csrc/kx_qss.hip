// kx_qss.hip -- production rates of a mechanism with quasi-steady-state (QSS)
// species on gfx950.  The paper lists QSS support as planned work (§4) without
// a formulation; the method here is the linearised QSSA of Lu & Law (J. Phys.
// Chem. A 110, 2006).  With at most one QSS molecule on either side of every
// reaction, each rate of progress is affine in the QSS concentrations C_Q, and
// the balances wdot_q = 0 form a linear system A C_Q = -b at every point.
//
// The mixture is that of the transported species: W-bar and C_k come from the
// non-QSS mass fractions (QSS entries of Y are not read), and the third-body
// sums run over transported species (a QSS species may not carry an
// efficiency; [M] = p/(R_u T) is their total concentration).
//
// Work decomposition: one workgroup of one wave per point.
//  1. species (thread = k): a_k = (p_atm/RT) e^{-g_k} (eq:K_p, eq:Ck) and C_k;
//     a QSS slot holds C = 1, so the products of phase 2 leave its factor out;
//  2. reactions (thread = r, every reaction of the mechanism): k_f, k_r =
//     k_f prod a' / prod a'', the modifier c_i (eq:c_i, eq:blend) and the two
//     products without the QSS factor, F'_r = c k_f prod C' and
//     B'_r = c k_r prod C'', into LDS;
//  3. QSS rows (thread = j): row j of [A | b] from the reactions in which the
//     net nu of QSS species j is not zero: the forward term goes to the column
//     of the reaction's QSS reactant (to b if it has none), the reverse term to
//     that of its QSS product;
//  4. elimination without row exchanges.  Up to 7 QSS species, [A | b] sits
//     in registers, one entry per lane (phase 3 sums each entry there), and
//     Gauss-Jordan steps read the pivot row and column by shuffles; beyond
//     that, rows in LDS (thread = row, one pivot per barrier) and back
//     substitution (one unknown per barrier).  Every column of A is
//     weakly diagonally dominant: a reaction that consumes a QSS molecule turns
//     it into at most one other QSS molecule, so the off-diagonal entries of a
//     column add up to at most its diagonal sink.  For such matrices
//     elimination keeps the pivots on the diagonal and is backward stable
//     (Golub & Van Loan, Matrix Computations, §3.4);
//  5. reactions (thread = r): R_r = F'_r C_s - B'_r C_t with s, t the QSS
//     species of the two sides (a factor 1 where a side has none);
//  6. species (thread = k): wdot_k = sum_r nu_kr R_r over the gather lists of
//     the rates kernel, summed in list order; the QSS rows are written as 0.
#include <hip/hip_runtime.h>
#include <float.h>

#include <algorithm>

#include "kx_internal.h"
#include "kx_math.h"

namespace kx {
namespace {

struct QPair {
    double a, C;
};

__device__ __forceinline__ double qgibbs(const DevSpecies &S, double T, double lnT, double invT)
{
    const double *g = (T < S.t_mid) ? S.g_lo : S.g_hi;
    const double poly = T * fma(T, fma(T, fma(T, g[4], g[3]), g[2]), g[1]);
    return fma(g[0], 1.0 - lnT, poly) + fma(g[5], invT, g[6]);
}

// Falloff blend F of eq:blend, Troe and SRI in one form (parameters as the
// table builder stores them: Troe alpha, 1/T***, 1/T*, T**; SRI a, b, 1/c,
// ln d, e).
__device__ __forceinline__ double qblend(const DevAux &ax, bool sri, double T, double lnT,
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

// Per-point scalars of phase 2: T, ln T, 1/T, [M] = p/(R_u T), ln p.
struct PointConst {
    double T, lnT, invT, Mc, lnp;
};

// Phase 2 for one reaction at one point: {F', B'} = c_i {k_f prod C', k_r prod
// C''} with the QSS slots counting 1 (k_f by eq:arrhenius or the pressure
// table, k_r = k_f prod a' / prod a'' by eq:K_p, c_i by eq:c_i and eq:blend).
__device__ __forceinline__ double2 reaction_terms(const MechDev &m, const DevRxn &R,
                                                  const QPair *sp, const PointConst &pc)
{
    const double Ti = pc.T, lnT = pc.lnT, invT = pc.invT, Mc = pc.Mc, lnp = pc.lnp;
    const unsigned type = R.type, flags = R.flags;
    const bool kconst = (flags & kFlagKfConst) != 0;
    double xf = kconst ? R.lnA : fma(R.beta, lnT, fma(-R.ER, invT, R.lnA));
    if (type == KX_RXN_PLOG) {
        const DevAux &ax = m.aux[R.aux];
        const DevPlog *pl = m.plog + ax.plog_off;
        const int cntp = ax.plog_cnt;
        int j = 0;
        while (j + 1 < cntp && pl[j + 1].lnp <= lnp) ++j;
        xf = fma(pl[j].beta, lnT, fma(-pl[j].ER, invT, pl[j].lnA));
        if (j + 1 < cntp && lnp > pl[j].lnp) {
            const double x2 =
                fma(pl[j + 1].beta, lnT, fma(-pl[j + 1].ER, invT, pl[j + 1].lnA));
            xf = fma((x2 - xf) * pl[j].inv_dlnp, lnp - pl[j].lnp, xf);
        }
    }
    const double kf = kconst ? R.A : kexp(xf);
    const QPair r0 = sp[R.roff[0] / 16], r1 = sp[R.roff[1] / 16], r2 = sp[R.roff[2] / 16];
    const QPair p0 = sp[R.poff[0] / 16], p1 = sp[R.poff[1] / 16], p2 = sp[R.poff[2] / 16];
    const bool rev = (flags & kFlagReversible) != 0;
    const double kr = rev ? kf * (r0.a * r1.a * r2.a) * krcp(p0.a * p1.a * p2.a) : 0.0;
    double F = kf * r0.C * r1.C * r2.C;
    const double B = kr * p0.C * p1.C * p2.C;
    if (flags & kFlagOrders) {  // no QSS species takes part (checked at create)
        const DevAux &ax = m.aux[R.aux];
        double S = 0.0;
        bool zero = false;
#pragma unroll
        for (int e = 0; e < kMaxOrd; ++e) {
            const double o = ax.oval[e], Ce = sp[ax.ooff[e] / 16].C;
            if (o != 0.0) {
                zero |= !(Ce > 0.0);
                S = fma(o, Ce > 0.0 ? kln(Ce) : 0.0, S);
            }
        }
        F = zero ? 0.0 : kf * kexp(S);
    }
    double cmod = 1.0;
    if (type != KX_RXN_ELEMENTARY && type != KX_RXN_PLOG) {
        const DevAux &ax = m.aux[R.aux];
        double X = ax.eff_default * Mc;
        for (int e = 0; e < kInlineEff; ++e) X = fma(ax.dalpha[e], sp[ax.eoff[e] / 16].C, X);
        for (int e = 0; e < ax.ext_cnt; ++e) {
            const DevEff f = m.eff[ax.ext_off + e];
            X = fma(f.dalpha, sp[f.sp].C, X);
        }
        if (type == KX_RXN_THREEBODY) {
            cmod = X;
        } else {
            const double d0 = fma(ax.beta0, lnT, fma(-ax.ER0, invT, ax.lnA0)) - xf;
            const double e0 = kexp(d0);
            const double Pr = e0 * X;
            double Fb = 1.0;
            if (type == KX_RXN_TROE || type == KX_RXN_SRI)
                Fb = qblend(ax, type == KX_RXN_SRI, Ti, lnT, invT,
                            fmax(d0 + kln(fmax(X, DBL_MIN)), -708.39641853226410622));
            const double h = krcp(1.0 + Pr);
            cmod = (flags & kFlagChemAct) ? e0 * Fb * h : Pr * Fb * h;
        }
    }
    return make_double2(cmod * F, cmod * B);
}

// Phases 3-4 with [A | b] in registers (nq (nq + 1) <= 64): lane l holds entry
// (j, c) = (l / (nq + 1), l % (nq + 1)), summed from row j's entries qe; then
// Gauss-Jordan steps on the diagonal read the pivot row and column by
// cross-lane shuffles (no LDS, no barrier), and x_j = -b'_j / a'_jj.
__device__ __forceinline__ void solve_in_registers(const MechDev &m, const int4 *qe,
                                                   const double2 *rec, double *x, int tid)
{
    const int nq = m.nq, ld = nq + 1;
    const bool act = tid < nq * ld;
    const int j = act ? tid / ld : nq - 1, c = act ? tid - j * ld : 0;
    double a = 0.0;
    if (act) {
        const int e0 = m.qrow_ptr[j], e1 = m.qrow_ptr[j + 1];
        for (int e = e0; e < e1; e += 4) {
            int4 en[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                en[u] = e + u < e1 ? qe[e + u] : make_int4(0, 0, -1, -1);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (e + u >= e1) break;
                const double2 fb = rec[en[u].x];
                const double nu = (double)en[u].y;
                if ((en[u].z >= 0 ? en[u].z : nq) == c) a = fma(nu, fb.x, a);
                if ((en[u].w >= 0 ? en[u].w : nq) == c) a = fma(-nu, fb.y, a);
            }
        }
    }
    for (int k = 0; k < nq; ++k) {
        const double akk = __shfl(a, k * ld + k, kWave);
        const double ajk = __shfl(a, j * ld + k, kWave);
        const double akc = __shfl(a, k * ld + c, kWave);
        if (act && j != k && c > k) a = fma(-(ajk / akk), akc, a);
    }
    const double ajj = __shfl(a, j * ld + j, kWave);
    if (act && c == nq) x[j] = -a / ajj;
}

// Phases 3-4 with the rows of [A | b] in LDS (thread = row): assembly, then
// elimination (one pivot per barrier) and back substitution (one unknown per
// barrier).
__device__ __forceinline__ void solve_in_lds(const MechDev &m, const int4 *qe,
                                             const double2 *rec, double *Am, double *x, int tid)
{
    const int nq = m.nq, ld = nq + 1;
    // ---- phase 3: row j of [A | b]
    if (tid < nq) {
        double *row = Am + tid * ld;
        for (int c = 0; c <= nq; ++c) row[c] = 0.0;
        // entries four at a time, their loads issued together
        const int e0 = m.qrow_ptr[tid], e1 = m.qrow_ptr[tid + 1];
        for (int e = e0; e < e1; e += 4) {
            int4 en[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                en[u] = e + u < e1 ? qe[e + u] : make_int4(0, 0, -1, -1);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (e + u >= e1) break;
                const double2 fb = rec[en[u].x];
                const double nu = (double)en[u].y;
                row[en[u].z >= 0 ? en[u].z : nq] += nu * fb.x;
                row[en[u].w >= 0 ? en[u].w : nq] -= nu * fb.y;
            }
        }
        x[tid] = -row[nq];
    }
    // ---- phase 4: elimination, then back substitution
    for (int k = 0; k < nq; ++k) {
        __syncthreads();
        if (tid > k && tid < nq) {
            double *row = Am + tid * ld;
            const double *pr = Am + k * ld;
            const double f = row[k] / pr[k];
            for (int c = k + 1; c < nq; ++c) row[c] = fma(-f, pr[c], row[c]);
            x[tid] = fma(-f, x[k], x[tid]);
        }
    }
    for (int k = nq - 1; k >= 0; --k) {
        __syncthreads();
        if (tid == k) x[k] = x[k] / Am[k * ld + k];
        __syncthreads();
        if (tid < k) x[tid] = fma(-Am[tid * ld + k], x[k], x[tid]);
    }
}

size_t qss_lds_bytes(const MechDev &m)
{
    const size_t ns = (size_t)m.ns, nr = (size_t)m.nr, nq = (size_t)m.nq;
    return sizeof(QPair) * (ns + 1)              // {a, C} per species (+dummy)
           + 2 * sizeof(double) * (size_t)m.nchunks * (m.chunk + 1)  // {F', B'}, then R,
                                                   // per chunk: chunk slots and a zero slot
           + sizeof(int4) * (size_t)m.nqent        // the balance rows' entries
           + sizeof(double) * (nq * (nq + 1) + nq);         // [A | b], x
}

// One wave (kWave threads) per point; see launch_qss.
__global__ __launch_bounds__(kWave) void qss_kernel(MechDev m, int64_t n,
                                                  const double *__restrict__ T,
                                                  const double *__restrict__ P,
                                                  const double *__restrict__ Y,
                                                  double *__restrict__ wdot,
                                                  double *__restrict__ Cq)
{
    extern __shared__ double lds[];
    constexpr int NT = kWave;
    const int ns = m.ns, nr = m.nr, nq = m.nq, tid = threadIdx.x;
    const int ld = nq + 1;  // row stride of [A | b]
    QPair *sp = reinterpret_cast<QPair *>(lds);
    double2 *rec = reinterpret_cast<double2 *>(sp + ns + 1);
    // chunk c owns rec[c (chunk + 1) ...]: its reactions (reaction r of the chunk
    // at base + c + r), then at offset chunk the zero slot that the padding
    // entries of the gather lists address (also for a partial last chunk)
    int4 *qe = reinterpret_cast<int4 *>(rec + m.nchunks * (m.chunk + 1));
    double *Am = reinterpret_cast<double *>(qe + m.nqent);
    double *x = Am + nq * ld;
    const int gw = kWave * m.gpass;
    // the entries of the balance rows are the same at every point: staged once
    for (int e = tid; e < m.nqent; e += NT) qe[e] = m.qrow_ent[e];
    __syncthreads();

    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const double Ti = T[i], pi = P[i];
        const double lnT = kln(Ti), invT = krcp(Ti);
        const double invRT = krcp(kRu * Ti);
        const double Mc = pi * invRT, P0 = kPatm * invRT, lnp = kln(pi);
        // W-bar over the transported species
        double part = 0.0;
        for (int k = tid; k < ns; k += NT)
            if (m.qidx[k] < 0) part = fma(Y[(int64_t)k * n + i], m.sp[k].inv_W, part);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
        const double cf = Mc * krcp(part);

        // ---- phase 1: species
        for (int k = tid; k < ns; k += NT) {
            const DevSpecies &S = m.sp[k];
            QPair q;
            q.a = P0 * kexp(-qgibbs(S, Ti, lnT, invT));
            q.C = m.qidx[k] < 0 ? Y[(int64_t)k * n + i] * S.inv_W * cf : 1.0;
            sp[k] = q;
        }
        if (tid == 0) {
            sp[ns].a = 1.0;
            sp[ns].C = 1.0;
        }
        __syncthreads();

        // ---- phase 2: one reaction per thread, chunk by chunk
        const PointConst pc{Ti, lnT, invT, Mc, lnp};
        for (int c = 0; c < m.nchunks; ++c) {
            const int base = c * m.chunk, cnt = min(m.chunk, nr - base);
            double2 *rc = rec + base + c;
            if (tid == 0) rc[m.chunk] = make_double2(0.0, 0.0);
            for (int rr = tid; rr < cnt; rr += NT) rc[rr] = reaction_terms(m, m.rxn[base + rr], sp, pc);
        }
        __syncthreads();

        // ---- phases 3-4: the QSS balances, then their solution x = C_Q
        if (nq * ld <= kWave)
            solve_in_registers(m, qe, rec, x, tid);
        else
            solve_in_lds(m, qe, rec, Am, x, tid);
        __syncthreads();
        if (Cq && tid < nq) Cq[(int64_t)tid * n + i] = x[tid];

        if (wdot) {
            // ---- phase 5: rates of progress with the QSS factors
            for (int c = 0; c < m.nchunks; ++c) {
                const int base = c * m.chunk, cnt = min(m.chunk, nr - base);
                for (int rr = tid; rr < cnt; rr += NT) {
                    const int2 q = m.qrx[base + rr];
                    double2 &f = rec[base + c + rr];
                    const double cs = q.x >= 0 ? x[q.x] : 1.0, ct = q.y >= 0 ? x[q.y] : 1.0;
                    f.x = fma(f.x, cs, -f.y * ct);
                }
            }
            __syncthreads();
            // ---- phase 6: wdot_k from the gather lists, chunk by chunk
            for (int k = tid; k < ns; k += NT) {
                double acc = 0.0;
                for (int c = 0; c < m.nchunks; ++c) {
                    const int base = c * m.chunk;
                    const int npos = m.gpos[c], ngrp = npos + m.gneg[c];
                    const uint4 *ge = m.gent + ((size_t)m.goff[c] * gw + k) * 2;
                    // list entries are byte offsets into the chunk's slots
                    const char *cb = reinterpret_cast<const char *>(rec + base + c);
                    // four groups per trip, their list loads issued together
                    for (int it0 = 0; it0 < ngrp; it0 += 4) {
                        uint4 v[8];
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const bool in = it0 + g < ngrp;
                            const size_t at = (size_t)(in ? it0 + g : it0) * 2 * gw;
                            v[2 * g] = ge[at];
                            v[2 * g + 1] = ge[at + 1];
                        }
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            if (it0 + g >= ngrp) break;
                            const unsigned off[8] = {v[2 * g].x, v[2 * g].y, v[2 * g].z,
                                                     v[2 * g].w, v[2 * g + 1].x, v[2 * g + 1].y,
                                                     v[2 * g + 1].z, v[2 * g + 1].w};
                            double s = 0.0;
#pragma unroll
                            for (int u = 0; u < 8; ++u)
                                s += *reinterpret_cast<const double *>(cb + off[u]);
                            acc += it0 + g < npos ? s : -s;
                        }
                    }
                }
                wdot[(int64_t)k * n + i] = m.qidx[k] < 0 ? acc : 0.0;
            }
        }
        __syncthreads();
    }
}

template <class K>
kx_status set_lds(K kern, size_t lds)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute (qss LDS)");
    return ok();
}
}  // namespace

kx_status launch_qss(const kx_mech *mech, int64_t n, const double *T, const double *p,
                     const double *Y, double *wdot, double *Cq, hipStream_t s)
{
    const MechDev &m = mech->dev;
    const size_t lds = qss_lds_bytes(m);
    if (lds > 160 * 1024)
        return fail(KX_EUNSUPPORTED, "QSS rates: mechanism too large for one workgroup's LDS");
    // One wave per point.  A point's work is a chain of dependent loads and
    // barriers rather than arithmetic, so more points in flight per CU beat more
    // threads per point: 2.8x faster than 256-thread groups on 53 species with
    // 6 QSS species (measured), and a one-wave barrier costs next to nothing.
    auto kern = qss_kernel;
    kx_status st = set_lds(kern, lds);
    if (st != KX_OK) return st;
    const unsigned grid = (unsigned)std::min<int64_t>(n, 32768);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave), lds, s, m, n, T, p, Y, wdot, Cq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "QSS rates kernel launch");
    return ok();
}

}  // namespace kx
