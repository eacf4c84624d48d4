/*
 * kx_oracle.c -- plain, slow, FP64 CPU reference for the per-grid-point
 * species production rates and mixture-averaged transport properties of
 * Danciu & Frouzakis, "KinetiX" (arXiv 2411.02640), Appendix A.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library calls, links or loads
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no header, helper, table or constant with the
 * HIP path: it takes the caller's mechanism arrays as they are and evaluates
 * the textbook definitions, in the order the appendix writes them, one grid
 * point at a time (OpenMP over points; no blocking, fusion or reuse).
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *  - NASA-7 with two ranges split at t_mid: low range when T < t_mid.
 *  - log in the Troe blend is base 10; ln in Arrhenius and in the fits.
 *  - The falloff factor P_r/(1+P_r) F multiplies the whole rate of progress
 *    once, with k_f = k_inf inside r_i (eq:c_i applied once, not twice).
 *  - The third-body factor [X]_i multiplies both directions.
 *  - Wilke: (W_j/W_k)^(1/4) inside phi_kj (the form of the cited Bird et al.
 *    text); the appendix prints (W_k/W_j)^(1/4).
 *  - Binary diffusion fits are evaluated at one atmosphere and divided by
 *    p/p_atm; kind 1 tables hold fits of 1/D_kj instead.
 *  - D_km falls back to D_kk when sum_{j!=k} X_j/D_kj is exactly zero.
 *  - P_r is clamped below at the smallest normal double before log10.
 *  - SRI: log in X = 1/(1 + log^2 P_r) is base 10, like Troe.
 *  - Chemically activated falloff: c_i = F/(1+P_r) (eq:c_i) and the rate of
 *    progress r_i uses k_0 where other reactions use k_f, so that the forward
 *    rate constant is k_0 F/(1+P_r).
 *  - Pressure tables (PLOG): ln k_f linear in ln p between the two neighbouring
 *    reference pressures; outside the table the nearest end point's k_j.
 *  - Explicit forward orders (irreversible reactions): the forward product is
 *    prod_k C_k^o_k with the listed o_k, nu'_k for unlisted reactants.
 *  - QSS species (linearised QSSA of Lu & Law, 2006; the paper only plans
 *    them): C_Q from wdot_Q = 0, the mixture (W-bar, third-body sums) that of
 *    the transported species.
 *  - Units: cgs, concentrations in mol/cm^3, Ea in cal/mol.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Own copies of the physical constants (CODATA 2018 exact R; thermochemical
 * calorie; standard atmosphere). */
#define KXO_RU 8.31446261815324e7                  /* erg / (mol K) */
#define KXO_RCAL (8.31446261815324 / 4.184)        /* cal / (mol K) */
#define KXO_PATM 1013250.0                         /* dyn / cm^2 */

enum { KXO_ELEMENTARY = 0, KXO_THREEBODY = 1, KXO_LINDEMANN = 2, KXO_TROE = 3, KXO_SRI = 4,
       KXO_PLOG = 5 };

/* The oracle's own view of a mechanism: plain host arrays, row-major. */
typedef struct {
    int32_t ns, nr, ne;
    const double *elem_mass;     /* [ne] */
    const int32_t *comp;         /* [ns][ne] */
    const double *nasa_lo;       /* [ns][7] */
    const double *nasa_hi;       /* [ns][7] */
    const double *t_mid;         /* [ns] */
    const int32_t *rtype;        /* [nr] */
    const int32_t *rev;          /* [nr] */
    const int32_t *reac_ptr, *reac_sp, *reac_nu;
    const int32_t *prod_ptr, *prod_sp, *prod_nu;
    const double *A, *beta, *Ea;        /* [nr] */
    const double *A0, *beta0, *Ea0;     /* [nr] */
    const double *troe;                 /* [nr][4] */
    const int32_t *eff_ptr, *eff_sp;
    const double *eff_val, *eff_default;
    int32_t fit_order;
    double fit_L0, fit_h;
    int32_t diff_kind;
    const double *visc_fit;      /* [ns][order] */
    const double *cond_fit;      /* [ns][order] */
    const double *diff_fit;      /* [ns][ns][order] */
    const double *sri;           /* [nr][5] a, b, c, d, e (or NULL) */
    const int32_t *chem_act;     /* [nr] (or NULL) */
    const int32_t *plog_ptr;     /* [nr+1] (or NULL) */
    const double *plog_p, *plog_A, *plog_beta, *plog_Ea;
    const int32_t *ord_ptr, *ord_sp;  /* (or NULL) */
    const double *ord_val;
} kxo_mech;

static int g_threads = 0;

void kxo_set_threads(int n) { g_threads = n; }

int kxo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static double species_weight(const kxo_mech *m, int k)
{
    double w = 0.0;
    for (int e = 0; e < m->ne; ++e) w += m->comp[k * m->ne + e] * m->elem_mass[e];
    return w;
}

/* x^n for integer n by repeated multiplication (n < 0: reciprocal). */
static double int_pow(double x, int n)
{
    double r = 1.0;
    int a = n < 0 ? -n : n;
    for (int i = 0; i < a; ++i) r *= x;
    return n < 0 ? 1.0 / r : r;
}

/* ---------------------------------------------------------------- thermo */

static const double *nasa_range(const kxo_mech *m, int k, double T)
{
    return (T < m->t_mid[k]) ? m->nasa_lo + 7 * k : m->nasa_hi + 7 * k;
}

/* App. A.1: Cp/R, H/RT (eq:H_RT), S/R (eq:S_R), and G/RT written out from the
 * closed form eq:Ck.  Any output pointer may be NULL. */
void kxo_thermo(const kxo_mech *m, double T, double *cp_r, double *h_rt,
                double *s_r, double *g_rt)
{
    const double T2 = T * T, T3 = T2 * T, T4 = T3 * T, lnT = log(T);
    for (int k = 0; k < m->ns; ++k) {
        const double *a = nasa_range(m, k, T);
        if (cp_r) cp_r[k] = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
        if (h_rt)
            h_rt[k] = a[0] + a[1] / 2.0 * T + a[2] / 3.0 * T2 + a[3] / 4.0 * T3 +
                      a[4] / 5.0 * T4 + a[5] / T;
        if (s_r)
            s_r[k] = a[0] * lnT + a[1] * T + a[2] / 2.0 * T2 + a[3] / 3.0 * T3 +
                     a[4] / 4.0 * T4 + a[6];
        if (g_rt)
            g_rt[k] = a[0] * (1.0 - lnT) - a[1] / 2.0 * T - a[2] / 6.0 * T2 -
                      a[3] / 12.0 * T3 - a[4] / 20.0 * T4 + a[5] / T - a[6];
    }
}

/* Mass-specific cp_k = Cp_k / W_k, h_k = H_k / W_k and the mixture
 * cp = sum_k Y_k cp_k (App. A.1), per point; SoA layout like the rates. */
void kxo_mixture_thermo(const kxo_mech *m, int64_t n, const double *T, const double *Y,
                        double *cp_mass, double *h_mass, double *cp_mix)
{
    const int ns = m->ns;
#pragma omp parallel num_threads(g_threads > 0 ? g_threads : kxo_max_threads())
    {
        double *cp_r = malloc(sizeof(double) * ns);
        double *h_rt = malloc(sizeof(double) * ns);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            kxo_thermo(m, T[i], cp_r, h_rt, NULL, NULL);
            double cp = 0.0;
            for (int k = 0; k < ns; ++k) {
                const double W = species_weight(m, k);
                const double cpk = cp_r[k] * KXO_RU / W;
                const double hk = h_rt[k] * KXO_RU * T[i] / W;
                if (cp_mass) cp_mass[(int64_t)k * n + i] = cpk;
                if (h_mass) h_mass[(int64_t)k * n + i] = hk;
                cp += Y[(int64_t)k * n + i] * cpk;
            }
            if (cp_mix) cp_mix[i] = cp;
        }
        free(cp_r);
        free(h_rt);
    }
}

/* ---------------------------------------------------------------- kinetics */

/* eq:arrhenius with E_R = E_a / R. */
static double arrhenius(double A, double b, double Ea, double T)
{
    const double ER = Ea / KXO_RCAL;
    return A * pow(T, b) * exp(-ER / T);
}

/* [X]_i = sum_k alpha_ki [X_k] with the reaction's default efficiency for
 * species not listed (App. A.2, third-body reactions). */
static double third_body(const kxo_mech *m, int i, const double *C)
{
    double X = 0.0;
    for (int k = 0; k < m->ns; ++k) {
        double alpha = m->eff_default[i];
        for (int e = m->eff_ptr[i]; e < m->eff_ptr[i + 1]; ++e)
            if (m->eff_sp[e] == k) alpha = m->eff_val[e];
        X += alpha * C[k];
    }
    return X;
}

/* Troe blending factor F (eq:blend, base-10 logarithms). */
static double troe_F(const double *p4, double T, double Pr)
{
    const double alpha = p4[0], T3 = p4[1], T1 = p4[2], T2 = p4[3];
    double Fcent = (1.0 - alpha) * exp(-T / T3) + alpha * exp(-T / T1);
    if (!isnan(T2)) Fcent += exp(-T2 / T);
    const double lFc = log10(Fcent);
    const double c = -0.4 - 0.67 * lFc;
    const double nn = 0.75 - 1.27 * lFc;
    const double d = 0.14;
    const double lPr = log10(Pr > DBL_MIN ? Pr : DBL_MIN);
    const double f1 = (lPr + c) / (nn - d * (lPr + c));
    const double lF = lFc / (1.0 + f1 * f1);
    return pow(10.0, lF);
}

/* SRI blending factor F = d T^e [a exp(-b/T) + exp(-T/c)]^X with
 * X = 1/(1 + log10(P_r)^2) (eq:blend). */
static double sri_F(const double *p5, double T, double Pr)
{
    const double a = p5[0], b = p5[1], c = p5[2], d = p5[3], e = p5[4];
    const double lPr = log10(Pr > DBL_MIN ? Pr : DBL_MIN);
    const double X = 1.0 / (1.0 + lPr * lPr);
    return d * pow(T, e) * pow(a * exp(-b / T) + exp(-T / c), X);
}

/* Forward rate constant of a pressure-table reaction at (T, p): the
 * logarithmic interpolation of App. A.2 between the reference pressures that
 * bracket p; the end point's rate outside the table. */
static double plog_kf(const kxo_mech *m, int i, double T, double p)
{
    const int b = m->plog_ptr[i], e = m->plog_ptr[i + 1];
    const double *P = m->plog_p;
    if (p <= P[b]) return arrhenius(m->plog_A[b], m->plog_beta[b], m->plog_Ea[b], T);
    if (p >= P[e - 1])
        return arrhenius(m->plog_A[e - 1], m->plog_beta[e - 1], m->plog_Ea[e - 1], T);
    int j = b;
    while (!(p < P[j + 1])) ++j;
    const double k1 = arrhenius(m->plog_A[j], m->plog_beta[j], m->plog_Ea[j], T);
    const double k2 = arrhenius(m->plog_A[j + 1], m->plog_beta[j + 1], m->plog_Ea[j + 1], T);
    const double lk = log(k1) + (log(k2) - log(k1)) * (log(p) - log(P[j])) /
                                    (log(P[j + 1]) - log(P[j]));
    return exp(lk);
}

/* Net stoichiometric coefficient nu''_ki - nu'_ki. */
static int net_nu(const kxo_mech *m, int i, int k)
{
    int nu = 0;
    for (int e = m->reac_ptr[i]; e < m->reac_ptr[i + 1]; ++e)
        if (m->reac_sp[e] == k) nu -= m->reac_nu[e];
    for (int e = m->prod_ptr[i]; e < m->prod_ptr[i + 1]; ++e)
        if (m->prod_sp[e] == k) nu += m->prod_nu[e];
    return nu;
}

/* Neumaier's compensated summation step. */
static void neumaier_add(double *sum, double *comp, double x)
{
    const double t = *sum + x;
    if (fabs(*sum) >= fabs(x))
        *comp += (*sum - t) + x;
    else
        *comp += (x - t) + *sum;
    *sum = t;
}

/*
 * Rates for one point.  C_k from Y (W-bar = 1 / sum Y_k/W_k); then per
 * reaction: k_f (Arrhenius, or k_inf with the falloff modifier), K_c from the
 * Gibbs energies (eq:K_p, eq:Ck) and (p_atm/RT)^(sum nu), k_r = k_f/K_c, the
 * law of mass action (eq:r_i) and the modifier c_i (eq:c_i); finally
 * wdot_k = sum_i nu_ki R_i with compensated summation.
 * scale_k = sum_i |nu_ki| |c_i| (k_f prod C^nu' + k_r prod C^nu''), the size
 * of the terms whose difference the net rate is.
 */
/* The per-reaction part of the rates, from concentrations: C enters the law
 * of mass action, Cm the third-body sums [X]_i (the same array unless QSS
 * species are excluded from the collision partners, see below); g = G_k/RT.
 * ws holds 3 ns doubles. */
static void rates_conc(const kxo_mech *m, double T, double p, const double *Cm,
                       const double *C, const double *g, double *wdot, double *scale,
                       int64_t ostride, double *qf_out, double *qr_out, double *c_out,
                       double *ws)
{
    const int ns = m->ns, nr = m->nr;
    double *sum = ws, *cmp = ws + ns, *scl = ws + 2 * ns;
    for (int k = 0; k < ns; ++k) sum[k] = cmp[k] = scl[k] = 0.0;

    for (int i = 0; i < nr; ++i) {
        const int type = m->rtype[i];
        double kf = (type == KXO_PLOG) ? plog_kf(m, i, T, p)
                                       : arrhenius(m->A[i], m->beta[i], m->Ea[i], T);
        double c = 1.0;
        if (type == KXO_THREEBODY) {
            c = third_body(m, i, Cm);
        } else if (type == KXO_LINDEMANN || type == KXO_TROE || type == KXO_SRI) {
            const double k0 = arrhenius(m->A0[i], m->beta0[i], m->Ea0[i], T);
            const double Pr = k0 * third_body(m, i, Cm) / kf;
            double F = 1.0;
            if (type == KXO_TROE) F = troe_F(m->troe + 4 * i, T, Pr);
            if (type == KXO_SRI) F = sri_F(m->sri + 5 * i, T, Pr);
            if (m->chem_act && m->chem_act[i]) {
                c = F / (1.0 + Pr);
                kf = k0;
            } else {
                c = Pr / (1.0 + Pr) * F;
            }
        }
        double kr = 0.0;
        if (m->rev[i]) {
            double dG = 0.0;
            int dnu = 0;
            for (int e = m->prod_ptr[i]; e < m->prod_ptr[i + 1]; ++e) {
                dG += m->prod_nu[e] * g[m->prod_sp[e]];
                dnu += m->prod_nu[e];
            }
            for (int e = m->reac_ptr[i]; e < m->reac_ptr[i + 1]; ++e) {
                dG -= m->reac_nu[e] * g[m->reac_sp[e]];
                dnu -= m->reac_nu[e];
            }
            const double Kp = exp(-dG);
            const double Kc = Kp * int_pow(KXO_PATM / (KXO_RU * T), dnu);
            kr = kf / Kc;
        }
        double Rf = 1.0, Rr = 1.0;
        const int o0 = m->ord_ptr ? m->ord_ptr[i] : 0, o1 = m->ord_ptr ? m->ord_ptr[i + 1] : 0;
        for (int e = m->reac_ptr[i]; e < m->reac_ptr[i + 1]; ++e) {
            int listed = 0;
            for (int f = o0; f < o1; ++f)
                if (m->ord_sp[f] == m->reac_sp[e]) listed = 1;
            if (!listed) Rf *= int_pow(C[m->reac_sp[e]], m->reac_nu[e]);
        }
        for (int f = o0; f < o1; ++f) Rf *= pow(C[m->ord_sp[f]], m->ord_val[f]);
        for (int e = m->prod_ptr[i]; e < m->prod_ptr[i + 1]; ++e)
            Rr *= int_pow(C[m->prod_sp[e]], m->prod_nu[e]);
        const double qf = kf * Rf, qr = kr * Rr;
        const double R = c * (qf - qr);
        if (qf_out) qf_out[i] = qf;
        if (qr_out) qr_out[i] = qr;
        if (c_out) c_out[i] = c;
        const double mag = fabs(c) * (fabs(qf) + fabs(qr));

        /* every species touched by reaction i, each once, with its net nu */
        for (int side = 0; side < 2; ++side) {
            const int32_t *ptr = side ? m->prod_ptr : m->reac_ptr;
            const int32_t *sp = side ? m->prod_sp : m->reac_sp;
            for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
                const int k = sp[e];
                int seen = 0; /* species already handled for this reaction */
                for (int f = ptr[i]; f < e; ++f)
                    if (sp[f] == k) seen = 1;
                if (side == 1)
                    for (int f = m->reac_ptr[i]; f < m->reac_ptr[i + 1]; ++f)
                        if (m->reac_sp[f] == k) seen = 1;
                if (seen) continue;
                const int nu = net_nu(m, i, k);
                if (nu == 0) continue;
                neumaier_add(&sum[k], &cmp[k], nu * R);
                scl[k] += abs(nu) * mag;
            }
        }
    }
    for (int k = 0; k < ns; ++k) {
        wdot[k * ostride] = sum[k] + cmp[k];
        if (scale) scale[k * ostride] = scl[k];
    }
}

static void rates_point(const kxo_mech *m, double T, double p, const double *Y,
                        int64_t stride, double *wdot, double *scale, int64_t ostride,
                        double *qf_out, double *qr_out, double *c_out, double *ws)
{
    const int ns = m->ns;
    double *C = ws, *g = ws + ns;

    double inv_wbar = 0.0;
    for (int k = 0; k < ns; ++k) inv_wbar += Y[k * stride] / species_weight(m, k);
    const double wbar = 1.0 / inv_wbar;
    for (int k = 0; k < ns; ++k) {
        const double X = Y[k * stride] * wbar / species_weight(m, k);
        C[k] = X * p / (KXO_RU * T);
    }
    kxo_thermo(m, T, NULL, NULL, NULL, g);
    rates_conc(m, T, p, C, C, g, wdot, scale, ostride, qf_out, qr_out, c_out, ws + 2 * ns);
}

/* Production rates for n points.  T[n], p[n] (dyn/cm^2), Y[ns][n];
 * wdot[ns][n] (mol/cm^3/s); scale[ns][n] may be NULL. */
void kxo_production_rates(const kxo_mech *m, int64_t n, const double *T, const double *p,
                          const double *Y, double *wdot, double *scale)
{
#pragma omp parallel num_threads(g_threads > 0 ? g_threads : kxo_max_threads())
    {
        double *ws = malloc(sizeof(double) * 5 * (size_t)m->ns);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            rates_point(m, T[i], p[i], Y + i, n, wdot + i, scale ? scale + i : NULL, n,
                        NULL, NULL, NULL, ws);
        free(ws);
    }
}

/* One point with the per-reaction forward / reverse rates and modifiers
 * exposed (qf[nr], qr[nr], c[nr]); Y, wdot, scale are contiguous [ns]. */
void kxo_rates_detail(const kxo_mech *m, double T, double p, const double *Y,
                      double *wdot, double *scale, double *qf, double *qr, double *c)
{
    double *ws = malloc(sizeof(double) * 5 * (size_t)m->ns);
    rates_point(m, T, p, Y, 1, wdot, scale, 1, qf, qr, c, ws);
    free(ws);
}

/* ------------------------------------------------ quasi-steady-state species
 *
 * The paper names QSS species as planned work (§4) and gives no formulation.
 * This follows the linearised QSSA of Lu & Law (J. Phys. Chem. A 110, 2006):
 * the species flagged in qss[] are not transported; their concentrations C_Q
 * follow from the algebraic balances wdot_q = 0.  With at most one QSS
 * molecule on either side of every reaction, no QSS species among the listed
 * third-body efficiencies and none in a reaction with explicit orders (the
 * library rejects other mechanisms), every rate of progress is affine in C_Q,
 * so wdot_Q(C_Q) = A C_Q + b.
 *
 * The mixture is that of the transported species: W-bar and C_k come from the
 * non-QSS entries of Y (QSS entries are not read), and the third-body sums
 * [X]_i run over the transported species only.
 *
 * The oracle does not assemble A from the reaction lists: it evaluates the
 * plain rates above at C_Q = 0 (giving b) and at C_Q = sigma_j e_j for each j
 * (giving column j of A as the difference over sigma_j), solves A C_Q = -b by
 * Gaussian elimination with partial pivoting, and evaluates the plain rates
 * once more with the solved C_Q. */

/* Solve A x = r in place (A n x n row-major, r holds x on return) by Gaussian
 * elimination with partial pivoting.  Returns -1 for an exactly zero pivot. */
static int gepp_solve(int n, double *A, double *r)
{
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
        if (A[piv * n + k] == 0.0) return -1;
        if (piv != k) {
            for (int j = 0; j < n; ++j) {
                const double t = A[k * n + j];
                A[k * n + j] = A[piv * n + j];
                A[piv * n + j] = t;
            }
            const double t = r[k];
            r[k] = r[piv];
            r[piv] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            const double f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            r[i] -= f * r[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = r[k];
        for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * r[j];
        r[k] = s / A[k * n + k];
    }
    return 0;
}

/* One point of the QSS rates.  wdot / scale for every species (a QSS row
 * holds the residual of its balance), Cq[nq] the QSS concentrations in the
 * species order.  ws: 7 ns + nq (nq + 3) doubles. */
static void qss_point(const kxo_mech *m, const int32_t *qss, double T, double p,
                      const double *Y, int64_t stride, double *wdot, double *scale,
                      int64_t ostride, double *Cq, int64_t cstride, double *ws,
                      double *A_out, double *b_out)
{
    const int ns = m->ns;
    double *C = ws, *Cm = ws + ns, *g = ws + 2 * ns, *w = ws + 3 * ns, *rw = ws + 4 * ns;
    double *Am = ws + 7 * ns;
    int nq = 0;
    for (int k = 0; k < ns; ++k) nq += qss[k] != 0;
    double *b = Am + nq * nq;

    double inv_wbar = 0.0;
    for (int k = 0; k < ns; ++k)
        if (!qss[k]) inv_wbar += Y[k * stride] / species_weight(m, k);
    const double wbar = 1.0 / inv_wbar;
    for (int k = 0; k < ns; ++k) {
        const double X = qss[k] ? 0.0 : Y[k * stride] * wbar / species_weight(m, k);
        C[k] = X * p / (KXO_RU * T);
        Cm[k] = C[k];
    }
    kxo_thermo(m, T, NULL, NULL, NULL, g);

    /* b = wdot_Q at C_Q = 0; column j of A = (wdot_Q(sigma_j e_j) - b) / sigma_j.
     * A is the same for every sigma_j > 0, but the difference keeps its digits
     * only while the C_q-terms at sigma_j are not small next to b: the first
     * pass takes sigma_j = p/(R_u T), the later ones max(p/(R_u T), |C_q|) of
     * the pass before. */
    double *b0 = Am + nq * nq + nq, *x = b0 + nq;
    rates_conc(m, T, p, Cm, C, g, w, NULL, 1, NULL, NULL, NULL, rw);
    for (int k = 0, i = 0; k < ns; ++k)
        if (qss[k]) b0[i++] = w[k];
    const double ctot = p / (KXO_RU * T);
    for (int i = 0; i < nq; ++i) x[i] = 0.0;
    for (int pass = 0; pass < 3; ++pass) {
        for (int kj = 0, j = 0; kj < ns; ++kj) {
            if (!qss[kj]) continue;
            const double sigma = fmax(ctot, fabs(x[j]));
            C[kj] = sigma;
            rates_conc(m, T, p, Cm, C, g, w, NULL, 1, NULL, NULL, NULL, rw);
            C[kj] = 0.0;
            for (int k = 0, i = 0; k < ns; ++k)
                if (qss[k]) {
                    Am[i * nq + j] = (w[k] - b0[i]) / sigma;
                    ++i;
                }
            ++j;
        }
        for (int i = 0; i < nq; ++i) b[i] = -b0[i];
        if (pass == 2 && A_out)
            for (int i = 0; i < nq * nq; ++i) A_out[i] = Am[i];
        if (pass == 2 && b_out)
            for (int i = 0; i < nq; ++i) b_out[i] = b0[i];
        if (gepp_solve(nq, Am, b) != 0)
            for (int i = 0; i < nq; ++i) b[i] = NAN;
        for (int i = 0; i < nq; ++i) x[i] = isfinite(b[i]) ? b[i] : 0.0;
    }
    for (int k = 0, i = 0; k < ns; ++k)
        if (qss[k]) {
            C[k] = b[i];
            Cq[(int64_t)i * cstride] = b[i];
            ++i;
        }
    rates_conc(m, T, p, Cm, C, g, wdot, scale, ostride, NULL, NULL, NULL, rw);
}

/* Rates of a mechanism with QSS species for n points: wdot[ns][n] (QSS rows:
 * the residual of the balance), scale[ns][n] (may be NULL), Cq[nq][n]. */
void kxo_qss_rates(const kxo_mech *m, const int32_t *qss, int64_t n, const double *T,
                   const double *p, const double *Y, double *wdot, double *scale, double *Cq)
{
    int nq = 0;
    for (int k = 0; k < m->ns; ++k) nq += qss[k] != 0;
#pragma omp parallel num_threads(g_threads > 0 ? g_threads : kxo_max_threads())
    {
        double *ws = malloc(sizeof(double) * (7 * (size_t)m->ns + (size_t)nq * (nq + 3)));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            qss_point(m, qss, T[i], p[i], Y + i, n, wdot + i, scale ? scale + i : NULL, n,
                      Cq + i, n, ws, NULL, NULL);
        free(ws);
    }
}

/* The linear system of the QSS balances at one point, as the oracle takes it
 * (A[nq][nq] row-major and b[nq] with wdot_Q = A C_Q + b); Y is contiguous. */
void kxo_qss_system(const kxo_mech *m, const int32_t *qss, double T, double p,
                    const double *Y, double *A, double *b)
{
    int nq = 0;
    for (int k = 0; k < m->ns; ++k) nq += qss[k] != 0;
    double *ws = malloc(sizeof(double) * (7 * (size_t)m->ns + (size_t)nq * (nq + 3)));
    double *w = malloc(sizeof(double) * 2 * (size_t)m->ns), *c = malloc(sizeof(double) * (nq + 1));
    qss_point(m, qss, T, p, Y, 1, w, NULL, 1, c, 1, ws, A, b);
    free(ws);
    free(w);
    free(c);
}

/* ------------------------------------------------ Jacobian by complex step
 *
 * d wdot_k / d C_j at fixed T, the pressure following the concentrations
 * (p = R_u T sum_k C_k, so [M] = sum_k C_k and a pressure table sees p), by
 * complex-step differentiation: the rates are evaluated once more in complex
 * arithmetic at C + i h e_j and the derivative is Im(wdot) / h.  This is
 * exact to rounding (no difference of nearly equal values) and shares none of
 * the derivative algebra of an analytical Jacobian.  The complex evaluation
 * repeats the real one above step for step. */

static double complex int_pow_c(double complex x, int n)
{
    double complex r = 1.0;
    int a = n < 0 ? -n : n;
    for (int i = 0; i < a; ++i) r *= x;
    return n < 0 ? 1.0 / r : r;
}

static double complex log10_clamped_c(double complex x)
{
    return creal(x) > DBL_MIN ? clog(x) / log(10.0) : log10(DBL_MIN);
}

static double complex troe_F_c(const double *p4, double T, double complex Pr)
{
    const double alpha = p4[0], T3 = p4[1], T1 = p4[2], T2 = p4[3];
    double Fcent = (1.0 - alpha) * exp(-T / T3) + alpha * exp(-T / T1);
    if (!isnan(T2)) Fcent += exp(-T2 / T);
    const double lFc = log10(Fcent);
    const double c = -0.4 - 0.67 * lFc, nn = 0.75 - 1.27 * lFc, d = 0.14;
    const double complex lPr = log10_clamped_c(Pr);
    const double complex f1 = (lPr + c) / (nn - d * (lPr + c));
    return cexp(log(10.0) * lFc / (1.0 + f1 * f1));
}

static double complex sri_F_c(const double *p5, double T, double complex Pr)
{
    const double a = p5[0], b = p5[1], c = p5[2], d = p5[3], e = p5[4];
    const double complex lPr = log10_clamped_c(Pr);
    const double complex X = 1.0 / (1.0 + lPr * lPr);
    return d * pow(T, e) * cexp(X * log(a * exp(-b / T) + exp(-T / c)));
}

static double complex plog_kf_c(const kxo_mech *m, int i, double T, double complex p)
{
    const int b = m->plog_ptr[i], e = m->plog_ptr[i + 1];
    const double *P = m->plog_p;
    const double pr = creal(p);
    if (pr <= P[b]) return arrhenius(m->plog_A[b], m->plog_beta[b], m->plog_Ea[b], T);
    if (pr >= P[e - 1])
        return arrhenius(m->plog_A[e - 1], m->plog_beta[e - 1], m->plog_Ea[e - 1], T);
    int j = b;
    while (!(pr < P[j + 1])) ++j;
    const double k1 = arrhenius(m->plog_A[j], m->plog_beta[j], m->plog_Ea[j], T);
    const double k2 = arrhenius(m->plog_A[j + 1], m->plog_beta[j + 1], m->plog_Ea[j + 1], T);
    return cexp(log(k1) + (log(k2) - log(k1)) * (clog(p) - log(P[j])) /
                              (log(P[j + 1]) - log(P[j])));
}

/* wdot(C) at temperature T in complex arithmetic; g[ns] = G_k/RT at T. */
static void rates_conc_c(const kxo_mech *m, double T, const double complex *C, const double *g,
                         double complex *wdot)
{
    const int ns = m->ns;
    double complex Mc = 0.0;
    for (int k = 0; k < ns; ++k) {
        Mc += C[k];
        wdot[k] = 0.0;
    }
    for (int i = 0; i < m->nr; ++i) {
        const int type = m->rtype[i];
        double complex kf = (type == KXO_PLOG) ? plog_kf_c(m, i, T, Mc * KXO_RU * T)
                                               : arrhenius(m->A[i], m->beta[i], m->Ea[i], T);
        double complex c = 1.0;
        if (type != KXO_ELEMENTARY && type != KXO_PLOG) {
            double complex X = 0.0;
            for (int k = 0; k < ns; ++k) {
                double alpha = m->eff_default[i];
                for (int e = m->eff_ptr[i]; e < m->eff_ptr[i + 1]; ++e)
                    if (m->eff_sp[e] == k) alpha = m->eff_val[e];
                X += alpha * C[k];
            }
            if (type == KXO_THREEBODY) {
                c = X;
            } else {
                const double k0 = arrhenius(m->A0[i], m->beta0[i], m->Ea0[i], T);
                const double complex Pr = k0 * X / kf;
                double complex F = 1.0;
                if (type == KXO_TROE) F = troe_F_c(m->troe + 4 * i, T, Pr);
                if (type == KXO_SRI) F = sri_F_c(m->sri + 5 * i, T, Pr);
                if (m->chem_act && m->chem_act[i]) {
                    c = F / (1.0 + Pr);
                    kf = k0;
                } else {
                    c = Pr / (1.0 + Pr) * F;
                }
            }
        }
        double complex kr = 0.0;
        if (m->rev[i]) {
            double dG = 0.0;
            int dnu = 0;
            for (int e = m->prod_ptr[i]; e < m->prod_ptr[i + 1]; ++e) {
                dG += m->prod_nu[e] * g[m->prod_sp[e]];
                dnu += m->prod_nu[e];
            }
            for (int e = m->reac_ptr[i]; e < m->reac_ptr[i + 1]; ++e) {
                dG -= m->reac_nu[e] * g[m->reac_sp[e]];
                dnu -= m->reac_nu[e];
            }
            kr = kf / (exp(-dG) * int_pow(KXO_PATM / (KXO_RU * T), dnu));
        }
        double complex Rf = 1.0, Rr = 1.0;
        const int o0 = m->ord_ptr ? m->ord_ptr[i] : 0, o1 = m->ord_ptr ? m->ord_ptr[i + 1] : 0;
        for (int e = m->reac_ptr[i]; e < m->reac_ptr[i + 1]; ++e) {
            int listed = 0;
            for (int f = o0; f < o1; ++f)
                if (m->ord_sp[f] == m->reac_sp[e]) listed = 1;
            if (!listed) Rf *= int_pow_c(C[m->reac_sp[e]], m->reac_nu[e]);
        }
        for (int f = o0; f < o1; ++f)
            if (m->ord_val[f] != 0.0) Rf *= cpow(C[m->ord_sp[f]], m->ord_val[f]);
        for (int e = m->prod_ptr[i]; e < m->prod_ptr[i + 1]; ++e)
            Rr *= int_pow_c(C[m->prod_sp[e]], m->prod_nu[e]);
        const double complex R = c * (kf * Rf - kr * Rr);
        for (int k = 0; k < ns; ++k) {
            const int nu = net_nu(m, i, k);
            if (nu != 0) wdot[k] += nu * R;
        }
    }
}

/* jac[i][k][j] = d wdot_k / d C_j for n points (T, p, Y as for the rates; the
 * derivative is taken at the concentrations C_k = X_k p / (R_u T)). */
void kxo_jacobian(const kxo_mech *m, int64_t n, const double *T, const double *p,
                  const double *Y, double *jac)
{
    const int ns = m->ns;
#pragma omp parallel num_threads(g_threads > 0 ? g_threads : kxo_max_threads())
    {
        double complex *C = malloc(sizeof(double complex) * ns);
        double complex *w = malloc(sizeof(double complex) * ns);
        double *g = malloc(sizeof(double) * ns);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double inv_wbar = 0.0;
            for (int k = 0; k < ns; ++k) inv_wbar += Y[k * n + i] / species_weight(m, k);
            const double wbar = 1.0 / inv_wbar;
            kxo_thermo(m, T[i], NULL, NULL, NULL, g);
            for (int j = 0; j < ns; ++j) {
                for (int k = 0; k < ns; ++k)
                    C[k] = Y[k * n + i] * wbar / species_weight(m, k) * p[i] / (KXO_RU * T[i]);
                const double h = 1e-30;
                C[j] += h * I;
                rates_conc_c(m, T[i], C, g, w);
                for (int k = 0; k < ns; ++k)
                    jac[((size_t)i * ns + k) * ns + j] = cimag(w[k]) / h;
            }
        }
        free(C);
        free(w);
        free(g);
    }
}

/* Forward rate constants k_f (k_inf for falloff) and, for falloff reactions,
 * k_0, at temperature T (for closed-form tests). */
void kxo_rate_constants(const kxo_mech *m, double T, double p, double *kf, double *k0)
{
    for (int i = 0; i < m->nr; ++i) {
        const int t = m->rtype[i];
        kf[i] = (t == KXO_PLOG) ? plog_kf(m, i, T, p) : arrhenius(m->A[i], m->beta[i], m->Ea[i], T);
        k0[i] = (t == KXO_LINDEMANN || t == KXO_TROE || t == KXO_SRI)
                    ? arrhenius(m->A0[i], m->beta0[i], m->Ea0[i], T)
                    : 0.0;
    }
}

/* The Troe and SRI blends for parameters p4 / p5 at (T, Pr), for closed-form
 * tests. */
double kxo_troe_F(const double *p4, double T, double Pr) { return troe_F(p4, T, Pr); }
double kxo_sri_F(const double *p5, double T, double Pr) { return sri_F(p5, T, Pr); }

/* --------------------------------------------------------------- transport */

/* sum_{n=1..N} c_n x^(n-1), powers by repeated multiplication. */
static double power_series(const double *c, int N, double x)
{
    double s = 0.0, xn = 1.0;
    for (int n = 0; n < N; ++n) {
        s += c[n] * xn;
        xn *= x;
    }
    return s;
}

/* Pure-species eta_k, lambda_k and the binary D_kj at (T, p) from the ln T fits
 * (App. A.3, "Polynomial fits"; eq:Dkj at one atmosphere, divided by p/p_atm).
 * eta[ns], lam[ns], D[ns][ns] (any may be NULL). */
void kxo_pure_transport(const kxo_mech *m, double T, double p, double *eta, double *lam,
                        double *D)
{
    const int ns = m->ns, N = m->fit_order;
    const double u = (log(T) - m->fit_L0) / m->fit_h;
    for (int k = 0; k < ns; ++k) {
        if (eta) eta[k] = power_series(m->visc_fit + (size_t)k * N, N, u);
        if (lam) lam[k] = power_series(m->cond_fit + (size_t)k * N, N, u);
    }
    if (D)
        for (int k = 0; k < ns; ++k)
            for (int j = 0; j < ns; ++j) {
                const double f = power_series(m->diff_fit + ((size_t)k * ns + j) * N, N, u);
                D[(size_t)k * ns + j] = (m->diff_kind == 0) ? f * KXO_PATM / p
                                                            : 1.0 / (f * p / KXO_PATM);
            }
}

/* Wilke's phi_kj (Bird et al. form) for given pure viscosities. */
static double wilke_phi(double Wk, double Wj, double eta_k, double eta_j)
{
    const double a = 1.0 + sqrt(eta_k / eta_j) * pow(Wj / Wk, 0.25);
    return 1.0 / sqrt(8.0) * pow(1.0 + Wk / Wj, -0.5) * a * a;
}

double kxo_wilke_phi(const kxo_mech *m, double T, int k, int j)
{
    double *eta = malloc(sizeof(double) * m->ns);
    kxo_pure_transport(m, T, KXO_PATM, eta, NULL, NULL);
    const double r = wilke_phi(species_weight(m, k), species_weight(m, j), eta[k], eta[j]);
    free(eta);
    return r;
}

static void transport_point(const kxo_mech *m, double T, double p, const double *Y,
                            int64_t stride, double *mu, double *lam_out, double *Dmix,
                            int64_t ostride, double *ws)
{
    const int ns = m->ns;
    double *X = ws, *eta = ws + ns, *lam = ws + 2 * ns, *W = ws + 3 * ns,
           *D = ws + 4 * ns; /* D: ns*ns */

    double inv_wbar = 0.0;
    for (int k = 0; k < ns; ++k) {
        W[k] = species_weight(m, k);
        inv_wbar += Y[k * stride] / W[k];
    }
    for (int k = 0; k < ns; ++k) X[k] = Y[k * stride] / W[k] / inv_wbar;
    double wbar = 0.0; /* W-bar = sum_k X_k W_k */
    for (int k = 0; k < ns; ++k) wbar += X[k] * W[k];

    kxo_pure_transport(m, T, p, eta, lam, D);

    /* Wilke / Bird mixture viscosity */
    double visc = 0.0;
    for (int k = 0; k < ns; ++k) {
        double den = 0.0;
        for (int j = 0; j < ns; ++j) den += X[j] * wilke_phi(W[k], W[j], eta[k], eta[j]);
        visc += X[k] * eta[k] / den;
    }
    *mu = visc;

    /* Mathur combination averaging */
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < ns; ++k) {
        s1 += X[k] * lam[k];
        s2 += X[k] / lam[k];
    }
    *lam_out = 0.5 * (s1 + 1.0 / s2);

    /* eq:mix_diff */
    for (int k = 0; k < ns; ++k) {
        double s = 0.0;
        for (int j = 0; j < ns; ++j)
            if (j != k) s += X[j] / D[(size_t)k * ns + j];
        Dmix[k * ostride] = (s == 0.0) ? D[(size_t)k * ns + k]
                                       : (wbar - X[k] * W[k]) / wbar / s;
    }
}

/* Mixture-averaged transport for n points: mu[n] (g/cm/s), lambda[n]
 * (erg/cm/s/K), Dmix[ns][n] (cm^2/s). */
void kxo_transport(const kxo_mech *m, int64_t n, const double *T, const double *p,
                   const double *Y, double *mu, double *lam, double *Dmix)
{
    const size_t wsz = (size_t)m->ns * (4 + (size_t)m->ns);
#pragma omp parallel num_threads(g_threads > 0 ? g_threads : kxo_max_threads())
    {
        double *ws = malloc(sizeof(double) * wsz);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            transport_point(m, T[i], p[i], Y + i, n, mu + i, lam + i, Dmix + i, n, ws);
        free(ws);
    }
}
