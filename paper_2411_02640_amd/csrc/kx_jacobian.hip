// kx_jacobian.hip -- analytical Jacobian of the species production rates on
// gfx950: J_kj = d wdot_k / d C_j at fixed temperature, the pressure following
// the concentrations (p = R_u T sum_k C_k).  The paper names the analytical
// Jacobian as the input of implicit (BDF) integrators (§1, §4).
//
// With R_i = c_i (F_i - B_i), F_i = k_f prod C^nu' (or prod C^o for explicit
// orders) and B_i = k_r prod C^nu'' (App. A.2, eq:r_i, eq:c_i):
//
//   d R_i / d C_j = c_i (dF_i/dC_j - dB_i/dC_j)                  mass action
//                 + (dc_i/d[X]_i) alpha_ji (F_i - B_i)            third body / falloff
//                 + c_i (F_i - B_i) (d ln k_f / d ln p) / [M]     pressure tables
//
// dF/dC of a molecule slot is k_f times the product of the other slots (exact
// also where a concentration is zero).  For falloff, P_r = e0 [X] with
// e0 = k_0/k_inf and, with g = d ln F / d ln P_r of the blend (eq:blend),
//   c = P_r/(1+P_r) F:        dc/d[X] = e0 F (1/(1+P_r)^2 + g/(1+P_r))
//   c = e0 F/(1+P_r) (chem. activated, referred to k_inf):
//                             dc/d[X] = e0 F (g/([X](1+P_r)) - e0/(1+P_r)^2).
//
// Work decomposition.  One workgroup of one or two waves per point; J is accumulated
// in LDS (row k owned by thread k, so no two threads write the same word):
//   1. species (thread = k): C_k, Gibbs g_k, a_k = (p_atm/RT) e^{-g_k}; zero row k;
//   2. reactions (thread = r, one chunk at a time): k_f, k_r = k_f A'/A'' (the
//      product of a over reactants over that over products is 1/K_c, eq:K_p),
//      the slot partials c dF/dC, c dB/dC, D = dc/d[X] (F - B) and the part
//      that is the same for every column j, into an LDS record per reaction;
//   3. species (thread = k): the chunk's gather lists (the +/- entries of the
//      production rates, repeated |nu| times) add nu_ki d R_i / d C_j into row k;
//   4. the matrix, plus the per-row constant, goes out as one contiguous block.
// Output layout: jac[(i * ns + k) * ns + j] -- one dense ns x ns matrix per
// point, the form batched linear solvers take.
#include <hip/hip_runtime.h>
#include <float.h>

#include <algorithm>

#include "kx_internal.h"
#include "kx_math.h"

namespace kx {
namespace {

constexpr int kJacMaxSpecies = 128;
// doubles per reaction record of phase 2: the partials, then a word packing the
// slots' species, type and flags, then the index of the reaction's DevAux
constexpr int kRec = 10;

struct JPair {
    double a, C;
};

__device__ __forceinline__ double jgibbs(const DevSpecies &S, double T, double lnT, double invT)
{
    const double *g = (T < S.t_mid) ? S.g_lo : S.g_hi;
    const double poly = T * fma(T, fma(T, fma(T, g[4], g[3]), g[2]), g[1]);
    return fma(g[0], 1.0 - lnT, poly) + fma(g[5], invT, g[6]);
}

// Falloff blend F (eq:blend, Troe and SRI in one form; see the rates kernel)
// and g = d ln F / d ln P_r.
__device__ __forceinline__ double jblend(const DevAux &ax, bool sri, double T, double lnT,
                                         double invT, double lnPr, double &g)
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
    const double den = fma(sri ? 0.0 : -0.14, x, nn);
    const double rden = krcp(den);
    const double w = x * rden;
    const double q = krcp(fma(w, w, 1.0));
    // d lnF/dw = -2 lnB w q^2; dw/dx = nn / den^2; dx/d ln P_r = 1 / ln 10
    g = -2.0 * lnB * w * q * q * nn * rden * rden * kInvLn10;
    return kexp(fma(lnB, q, sri ? fma(a4, lnT, a3) : 0.0));
}

size_t jac_lds_bytes(const MechDev &m)
{
    const size_t ns = (size_t)m.ns;
    return sizeof(double) * (ns * ns + ns + 2)           // J, row constants (+pad)
           + sizeof(JPair) * (ns + 1)                     // {a, C} per species (+dummy)
           + sizeof(double) * kRec * (size_t)(m.chunk + 1);  // records (+zero record)
}

// NT threads (one or two waves; thread k owns row k, ns <= NT)
template <int NT>
__global__ __launch_bounds__(NT) void jacobian_kernel(MechDev m, int64_t n,
                                                         const double *__restrict__ T,
                                                         const double *__restrict__ P,
                                                         const double *__restrict__ Y,
                                                         double *__restrict__ jac)
{
    extern __shared__ double lds[];
    const int ns = m.ns, nsq = ns * ns, tid = threadIdx.x;
    double *J = lds;
    double *rowc = J + nsq;
    // ns * ns + ns is even, so the pairs start 16-byte aligned after ns + 2 slots
    JPair *sp = reinterpret_cast<JPair *>(rowc + ns + 2);
    double *rec = reinterpret_cast<double *>(sp + ns + 1);
    const int gw = kWave * m.gpass;

    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const double Ti = T[i], pi = P[i];
        const double lnT = kln(Ti), invT = krcp(Ti);
        const double invRT = krcp(kRu * Ti);
        const double Mc = pi * invRT, P0 = kPatm * invRT, lnp = kln(pi);
        // W-bar: sum_k Y_k / W_k over the workgroup (the two waves meet in the
        // record area, which phase 2 fills only later)
        double part = 0.0;
        for (int k = tid; k < ns; k += NT) part = fma(Y[(int64_t)k * n + i], m.sp[k].inv_W, part);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
        if (NT > kWave) {
            if ((tid & (kWave - 1)) == 0) rec[tid / kWave] = part;
            __syncthreads();
            part = rec[0] + rec[1];
            __syncthreads();
        }
        const double cf = Mc * krcp(part);

        // ---- phase 1: species
        for (int k = tid; k < ns; k += NT) {
            {
                const DevSpecies &S = m.sp[k];
                JPair q;
                q.a = P0 * kexp(-jgibbs(S, Ti, lnT, invT));
                q.C = Y[(int64_t)k * n + i] * S.inv_W * cf;
                sp[k] = q;
                for (int j = 0; j < ns; ++j) J[k * ns + j] = 0.0;
                rowc[k] = 0.0;
            }
        }
        if (tid == 0) {
            sp[ns].a = 1.0;
            sp[ns].C = 1.0;
        }
        if (tid < kRec) rec[kRec * m.chunk + tid] = 0.0;
        __syncthreads();

        for (int c = 0; c < m.nchunks; ++c) {
            const int base = c * m.chunk;
            const int cnt = min(m.chunk, m.nr - base);
            // ---- phase 2: one reaction per thread
            for (int r = tid; r < cnt; r += NT) {
                const DevRxn &R = m.rxn[base + r];
                const unsigned type = R.type, flags = R.flags;
                const bool kconst = (flags & kFlagKfConst) != 0;
                double xf = kconst ? R.lnA : fma(R.beta, lnT, fma(-R.ER, invT, R.lnA));
                double slope = 0.0;  // d ln k_f / d ln p
                if (type == KX_RXN_PLOG) {
                    const DevAux &ax = m.aux[R.aux];
                    const DevPlog *pl = m.plog + ax.plog_off;
                    const int cntp = ax.plog_cnt;
                    int j = 0;
                    while (j + 1 < cntp && pl[j + 1].lnp <= lnp) ++j;
                    const double x1 = fma(pl[j].beta, lnT, fma(-pl[j].ER, invT, pl[j].lnA));
                    xf = x1;
                    if (j + 1 < cntp && lnp > pl[j].lnp) {
                        const double x2 =
                            fma(pl[j + 1].beta, lnT, fma(-pl[j + 1].ER, invT, pl[j + 1].lnA));
                        slope = (x2 - x1) * pl[j].inv_dlnp;
                        xf = fma(slope, lnp - pl[j].lnp, x1);
                    }
                }
                const double kf = kconst ? R.A : kexp(xf);
                const JPair r0 = sp[R.roff[0] / 16], r1 = sp[R.roff[1] / 16],
                            r2 = sp[R.roff[2] / 16];
                const JPair p0 = sp[R.poff[0] / 16], p1 = sp[R.poff[1] / 16],
                            p2 = sp[R.poff[2] / 16];
                const bool rev = (flags & kFlagReversible) != 0;
                // k_r = k_f prod_reac a / prod_prod a  (1/K_c from eq:K_p)
                const double kr =
                    rev ? kf * (r0.a * r1.a * r2.a) * krcp(p0.a * p1.a * p2.a) : 0.0;
                double F = kf * r0.C * r1.C * r2.C;
                const double B = kr * p0.C * p1.C * p2.C;
                double Pd[4] = {kf * r1.C * r2.C, kf * r0.C * r2.C, kf * r0.C * r1.C, 0.0};
                const double Qd[3] = {kr * p1.C * p2.C, kr * p0.C * p2.C, kr * p0.C * p1.C};
                if (flags & kFlagOrders) {
                    // F = k_f prod C^o over the listed species (irreversible)
                    const DevAux &ax = m.aux[R.aux];
                    double Cs[kMaxOrd], lnC[kMaxOrd], S = 0.0;
                    int nz = 0;
#pragma unroll
                    for (int e = 0; e < kMaxOrd; ++e) {
                        Cs[e] = sp[ax.ooff[e] / 16].C;
                        const bool use = ax.oval[e] != 0.0;
                        nz += (use && !(Cs[e] > 0.0)) ? 1 : 0;
                        lnC[e] = (use && Cs[e] > 0.0) ? kln(Cs[e]) : 0.0;
                        S = fma(use ? ax.oval[e] : 0.0, lnC[e], S);
                    }
                    F = nz ? 0.0 : kf * kexp(S);
#pragma unroll
                    for (int e = 0; e < kMaxOrd; ++e) {
                        const double o = ax.oval[e];
                        double d = 0.0;
                        if (o != 0.0) {
                            if (Cs[e] > 0.0) {
                                d = nz ? 0.0 : o * F * krcp(Cs[e]);
                            } else if (nz == 1) {  // only this species is absent
                                const double rest = kf * kexp(S);  // S excludes it
                                d = (o == 1.0) ? rest : (o > 1.0 ? 0.0 : __builtin_inf());
                            }
                        }
                        Pd[e] = d;
                    }
                }
                double cmod = 1.0, dcdX = 0.0, dense = 0.0;
                if (type != KX_RXN_ELEMENTARY && type != KX_RXN_PLOG) {
                    const DevAux &ax = m.aux[R.aux];
                    double X = ax.eff_default * Mc;
                    for (int e = 0; e < kInlineEff; ++e)
                        X = fma(ax.dalpha[e], sp[ax.eoff[e] / 16].C, X);
                    for (int e = 0; e < ax.ext_cnt; ++e) {
                        const DevEff f = m.eff[ax.ext_off + e];
                        X = fma(f.dalpha, sp[f.sp].C, X);
                    }
                    if (type == KX_RXN_THREEBODY) {
                        cmod = X;
                        dcdX = 1.0;
                    } else {
                        const double d0 = fma(ax.beta0, lnT, fma(-ax.ER0, invT, ax.lnA0)) - xf;
                        const double e0 = kexp(d0);
                        const double Pr = e0 * X;
                        double Fb = 1.0, g = 0.0;
                        if (type == KX_RXN_TROE || type == KX_RXN_SRI) {
                            const double lnPr =
                                fmax(d0 + kln(fmax(X, DBL_MIN)), -708.39641853226410622);
                            Fb = jblend(ax, type == KX_RXN_SRI, Ti, lnT, invT, lnPr, g);
                        }
                        const double h = krcp(1.0 + Pr);
                        if (flags & kFlagChemAct) {
                            cmod = e0 * Fb * h;
                            const double gX = g == 0.0 ? 0.0 : g * krcp(X);
                            dcdX = e0 * Fb * (gX * h - e0 * h * h);
                        } else {
                            cmod = Pr * Fb * h;
                            dcdX = e0 * Fb * (h * h + g * h);
                        }
                    }
                    dense = dcdX * (F - B) * ax.eff_default;
                }
                const double D = dcdX * (F - B);
                dense = fma(cmod * (F - B) * slope, krcp(Mc), dense);
                // species of the six slots (or of the four orders), type and flags
                // packed into one 8-byte word, so phase 3 reads no reaction table
                uint64_t pk = ((uint64_t)flags << 56) | ((uint64_t)type << 48);
                if (flags & kFlagOrders) {
                    const DevAux &ax = m.aux[R.aux];
#pragma unroll
                    for (int e = 0; e < kMaxOrd; ++e) pk |= (uint64_t)(ax.ooff[e] / 16) << (8 * e);
                } else {
#pragma unroll
                    for (int q = 0; q < kMaxSide; ++q)
                        pk |= ((uint64_t)(R.roff[q] / 16) << (8 * q)) |
                              ((uint64_t)(R.poff[q] / 16) << (8 * (q + 3)));
                }
                double *rr = rec + kRec * r;
                rr[8] = __longlong_as_double((long long)pk);
                rr[9] = __longlong_as_double((long long)R.aux);
                rr[0] = cmod * Pd[0];
                rr[1] = cmod * Pd[1];
                rr[2] = cmod * Pd[2];
                rr[3] = (flags & kFlagOrders) ? cmod * Pd[3] : cmod * Qd[0];
                rr[4] = cmod * Qd[1];
                rr[5] = cmod * Qd[2];
                rr[6] = D;
                rr[7] = dense;
            }
            __syncthreads();
            // ---- phase 3: thread = species k, its +/- entries of this chunk
            const int npos = m.gpos[c], ngrp = npos + m.gneg[c];
            for (int k = tid; k < ns; k += NT) {
                const uint4 *ge = m.gent + ((size_t)m.goff[c] * gw + k) * 2;
                double *Jk = J + k * ns;
                double rc = 0.0;
                // four groups per trip, their list loads issued together
                for (int it0 = 0; it0 < ngrp; it0 += 4) {
                    uint4 v[8];
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const size_t at = (size_t)(it0 + g < ngrp ? it0 + g : it0) * 2 * gw;
                        v[2 * g] = ge[at];
                        v[2 * g + 1] = ge[at + 1];
                    }
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const int it = it0 + g;
                        if (it >= ngrp) break;
                        const unsigned off[8] = {v[2 * g].x,     v[2 * g].y,     v[2 * g].z,
                                                 v[2 * g].w,     v[2 * g + 1].x, v[2 * g + 1].y,
                                                 v[2 * g + 1].z, v[2 * g + 1].w};
                        const double sg = it < npos ? 1.0 : -1.0;
                        for (int u = 0; u < 8; ++u) {
                            const int r = (int)(off[u] / 16);
                            if (r >= cnt) continue;  // padding entry
                            const double *rr = rec + kRec * r;
                            const uint64_t pk = (uint64_t)__double_as_longlong(rr[8]);
                            const unsigned flags = (unsigned)(pk >> 56), type = (unsigned)(pk >> 48) & 0xFFu;
                            if (flags & kFlagOrders) {
                                for (int e = 0; e < kMaxOrd; ++e) {
                                    const int jo = (int)((pk >> (8 * e)) & 0xFFu);
                                    if (jo < ns) Jk[jo] += sg * rr[e];
                                }
                            } else {
                                for (int q = 0; q < kMaxSide; ++q) {
                                    const int jr = (int)((pk >> (8 * q)) & 0xFFu);
                                    const int jp = (int)((pk >> (8 * (q + 3))) & 0xFFu);
                                    if (jr < ns) Jk[jr] += sg * rr[q];
                                    if (jp < ns) Jk[jp] -= sg * rr[3 + q];
                                }
                            }
                            if (type != KX_RXN_ELEMENTARY && type != KX_RXN_PLOG) {
                                const DevAux &ax = m.aux[(int)__double_as_longlong(rr[9])];
                                const double D = sg * rr[6];
                                for (int e = 0; e < kInlineEff; ++e)
                                    if (ax.dalpha[e] != 0.0) Jk[ax.eoff[e] / 16] += D * ax.dalpha[e];
                                for (int e = 0; e < ax.ext_cnt; ++e) {
                                    const DevEff f = m.eff[ax.ext_off + e];
                                    Jk[f.sp] += D * f.dalpha;
                                }
                            }
                            rc += sg * rr[7];
                        }
                    }
                }
                rowc[k] += rc;
            }
            __syncthreads();
        }
        // ---- phase 4: the matrix with the per-row constants, one contiguous block
        double *out = jac + (size_t)i * nsq;
        for (int e = tid; e < nsq; e += NT) out[e] = J[e] + rowc[e / ns];
        __syncthreads();
    }
}

template <class K>
kx_status set_lds(K kern, size_t lds)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute (jacobian LDS)");
    return ok();
}
}  // namespace

kx_status launch_jacobian(const kx_mech *mech, int64_t n, const double *T, const double *p,
                          const double *Y, double *jac, hipStream_t s)
{
    const MechDev &m = mech->dev;
    if (m.ns > kJacMaxSpecies)
        return fail(KX_EUNSUPPORTED, "kx_jacobian: at most 128 species are supported");
    const size_t lds = jac_lds_bytes(m);
    if (lds > 160 * 1024) return fail(KX_EUNSUPPORTED, "kx_jacobian: mechanism too large for LDS");
    // one wave when it covers both the species and the reactions of a step,
    // two otherwise
    const bool two = m.ns > kWave || m.nr > kWave;
    auto kern = two ? jacobian_kernel<2 * kWave> : jacobian_kernel<kWave>;
    kx_status st = set_lds(kern, lds);
    if (st != KX_OK) return st;
    const unsigned grid = (unsigned)std::min<int64_t>(n, 16384);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(two ? 2 * kWave : kWave), lds, s, m, n, T, p, Y,
                       jac);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "jacobian kernel launch");
    return ok();
}

}  // namespace kx
