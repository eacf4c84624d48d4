// kx_mech.cpp -- host-side mechanism table builder (kx_mech_create).
//
// Validates a kx_mech_desc, derives every table the gfx950 kernels read and
// uploads them to the device in one allocation:
//  * reactions re-ordered heaviest type first (Troe, Lindemann, three-body,
//    elementary; constant-k_f reactions last inside each type) so that the
//    falloff code runs in as few 64-lane iterations as possible and a partial
//    last iteration holds the cheapest reactions;
//  * each reaction side as a list of LDS byte offsets, one per molecule, padded
//    with a dummy species whose per-point factors are 1;
//  * ln A, E_R = E_a / R and the beta = E_R = 0 shortcut of eq:k_f;
//  * third-body efficiencies as (alpha - default) lists, falloff k_0 and Troe
//    parameters (inverse temperatures);
//  * a species-major gather list per reaction chunk for wdot_k = sum_i nu_ki R_i,
//    padded to one trip count and interleaved for coalesced loads;
//  * Gibbs coefficients of eq:Ck pre-scaled per range, raw NASA-7 for cp / h;
//  * Wilke constants c1_kj = (8 (1 + W_k/W_j))^(-1/2) and W_k^(1/4) (so that
//    (W_j/W_k)^(1/4) separates into per-species factors), and the ln T fit
//    tables in the k-blocked order of the transport kernel, in FP64 and FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "kx_internal.h"

namespace kx {
namespace {

struct Blob {
    std::vector<uint8_t> host;
    size_t add(const void *src, size_t bytes)
    {
        size_t off = (host.size() + 255) & ~size_t(255);
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, src, bytes);
        return off;
    }
};

template <class T> size_t add_vec(Blob &b, const std::vector<T> &v)
{
    return b.add(v.data(), v.size() * sizeof(T));
}

// Net stoichiometric coefficient nu''_ki - nu'_ki of species k in reaction i.
int net_nu(const kx_mech_desc *d, int i, int k)
{
    int nu = 0;
    for (int e = d->reac_ptr[i]; e < d->reac_ptr[i + 1]; ++e)
        if (d->reac_sp[e] == k) nu -= d->reac_nu[e];
    for (int e = d->prod_ptr[i]; e < d->prod_ptr[i + 1]; ++e)
        if (d->prod_sp[e] == k) nu += d->prod_nu[e];
    return nu;
}

// QSS species of one side of reaction i (the first one) and their molecule count.
int qss_side(const kx_mech_desc *d, int i, bool prod, int *count)
{
    const int32_t *ptr = prod ? d->prod_ptr : d->reac_ptr;
    const int32_t *sp = prod ? d->prod_sp : d->reac_sp;
    const int32_t *nu = prod ? d->prod_nu : d->reac_nu;
    int first = -1, c = 0;
    for (int e = ptr[i]; e < ptr[i + 1]; ++e)
        if (d->qss[sp[e]]) {
            if (first < 0) first = sp[e];
            c += nu[e];
        }
    *count = c;
    return first;
}

// The linearised QSSA needs every rate of progress affine in the QSS
// concentrations and every QSS balance to hold a sink.
kx_status validate_qss(const kx_mech_desc *d)
{
    const int ns = d->n_species, nr = d->n_reactions;
    int nq = 0;
    for (int k = 0; k < ns; ++k) {
        if (d->qss[k] != 0 && d->qss[k] != 1)
            return fail(KX_EINVAL, "kx_mech_create: qss flags must be 0 or 1");
        nq += d->qss[k];
    }
    if (nq > kMaxQss)
        return fail(KX_EUNSUPPORTED, "kx_mech_create: at most 64 QSS species are supported");
    if (nq == ns) return fail(KX_EINVAL, "kx_mech_create: every species is QSS");
    std::vector<char> consumed(ns, 0);
    for (int i = 0; i < nr; ++i) {
        const std::string ri = " (reaction " + std::to_string(i) + ")";
        int cr = 0, cp = 0;
        qss_side(d, i, false, &cr);
        qss_side(d, i, true, &cp);
        if (cr > 1 || cp > 1)
            return fail(KX_EUNSUPPORTED, "kx_mech_create: two QSS molecules on one side of a "
                                         "reaction" + ri);
        const int t = d->rxn_type[i];
        if (t != KX_RXN_ELEMENTARY && t != KX_RXN_PLOG)
            for (int e = d->eff_ptr[i]; e < d->eff_ptr[i + 1]; ++e)
                if (d->qss[d->eff_sp[e]])
                    return fail(KX_EUNSUPPORTED, "kx_mech_create: QSS species in an "
                                                 "efficiency list" + ri);
        if (d->ord_ptr && d->ord_ptr[i + 1] > d->ord_ptr[i]) {
            bool any = cr > 0 || cp > 0;
            for (int e = d->ord_ptr[i]; e < d->ord_ptr[i + 1]; ++e) any |= d->qss[d->ord_sp[e]] != 0;
            if (any)
                return fail(KX_EUNSUPPORTED, "kx_mech_create: QSS species in a reaction with "
                                             "explicit orders" + ri);
        }
        for (int k = 0; k < ns; ++k) {
            if (!d->qss[k]) continue;
            const int nu = net_nu(d, i, k);
            if (nu < 0 || (nu > 0 && d->reversible[i])) consumed[k] = 1;
        }
    }
    for (int k = 0; k < ns; ++k)
        if (d->qss[k] && !consumed[k])
            return fail(KX_EINVAL, "kx_mech_create: QSS species " + std::to_string(k) +
                                       " is consumed by no reaction");
    return KX_OK;
}

kx_status validate(const kx_mech_desc *d, std::vector<double> &W)
{
    if (!d) return fail(KX_EINVAL, "kx_mech_create: desc is NULL");
    const int ns = d->n_species, nr = d->n_reactions, ne = d->n_elements;
    if (ns <= 0 || nr < 0 || ne <= 0)
        return fail(KX_EINVAL, "kx_mech_create: n_species and n_elements must be > 0, "
                               "n_reactions >= 0");
    if (ns > kMaxSpecies)
        return fail(KX_EUNSUPPORTED, "kx_mech_create: at most 256 species are supported");
    if (!d->elem_mass || !d->composition || !d->nasa_lo || !d->nasa_hi || !d->t_mid ||
        !d->visc_fit || !d->cond_fit || !d->diff_fit)
        return fail(KX_EINVAL, "kx_mech_create: NULL species array");
    if (nr > 0 && (!d->rxn_type || !d->reversible || !d->reac_ptr || !d->reac_sp ||
                   !d->reac_nu || !d->prod_ptr || !d->prod_sp || !d->prod_nu || !d->A ||
                   !d->beta || !d->Ea || !d->A0 || !d->beta0 || !d->Ea0 || !d->troe ||
                   !d->eff_ptr || !d->eff_default))
        return fail(KX_EINVAL, "kx_mech_create: NULL reaction array");
    if (d->fit_order < 1 || d->fit_order > kMaxFitOrder)
        return fail(KX_EINVAL, "kx_mech_create: fit_order must be in 1..8");
    if (!(d->fit_h != 0.0) || !std::isfinite(d->fit_h) || !std::isfinite(d->fit_L0))
        return fail(KX_EINVAL, "kx_mech_create: fit_h must be finite and non-zero");
    if (d->diff_fit_kind != 0 && d->diff_fit_kind != 1)
        return fail(KX_EINVAL, "kx_mech_create: diff_fit_kind must be 0 or 1");
    W.assign(ns, 0.0);
    for (int k = 0; k < ns; ++k) {
        for (int e = 0; e < ne; ++e) {
            if (d->composition[k * ne + e] < 0)
                return fail(KX_EINVAL, "kx_mech_create: negative atom count");
            W[k] += d->composition[k * ne + e] * d->elem_mass[e];
        }
        if (!(W[k] > 0.0))
            return fail(KX_EINVAL, "kx_mech_create: species " + std::to_string(k) +
                                       " has non-positive molecular weight");
    }
    const int order = d->fit_order;
    for (int k = 0; k < ns; ++k)
        for (int j = 0; j < ns; ++j)
            for (int o = 0; o < order; ++o)
                if (d->diff_fit[((size_t)k * ns + j) * order + o] !=
                    d->diff_fit[((size_t)j * ns + k) * order + o])
                    return fail(KX_EINVAL, "kx_mech_create: diff_fit is not symmetric");
    for (int i = 0; i < nr; ++i) {
        const std::string ri = " (reaction " + std::to_string(i) + ")";
        const int t = d->rxn_type[i];
        if (t < KX_RXN_ELEMENTARY || t > KX_RXN_PLOG)
            return fail(KX_EINVAL, "kx_mech_create: unknown reaction type" + ri);
        const bool falloff = t == KX_RXN_LINDEMANN || t == KX_RXN_TROE || t == KX_RXN_SRI;
        if (t == KX_RXN_PLOG) {
            if (!d->plog_ptr || !d->plog_p || !d->plog_A || !d->plog_beta || !d->plog_Ea)
                return fail(KX_EINVAL, "kx_mech_create: NULL PLOG array" + ri);
            const int b = d->plog_ptr[i], e = d->plog_ptr[i + 1];
            if (b < 0 || e <= b)
                return fail(KX_EINVAL, "kx_mech_create: PLOG reaction without pressures" + ri);
            for (int j = b; j < e; ++j) {
                if (!(d->plog_p[j] > 0.0) || !std::isfinite(d->plog_p[j]) ||
                    (j > b && !(d->plog_p[j] > d->plog_p[j - 1])))
                    return fail(KX_EINVAL, "kx_mech_create: PLOG pressures must be positive "
                                           "and strictly increasing" + ri);
                if (!(d->plog_A[j] > 0.0) || !std::isfinite(d->plog_A[j]) ||
                    !std::isfinite(d->plog_beta[j]) || !std::isfinite(d->plog_Ea[j]))
                    return fail(KX_EINVAL, "kx_mech_create: PLOG A must be > 0, beta and "
                                           "Ea finite" + ri);
            }
        } else if (!(d->A[i] > 0.0) || !std::isfinite(d->A[i]) || !std::isfinite(d->beta[i]) ||
                   !std::isfinite(d->Ea[i])) {
            return fail(KX_EINVAL, "kx_mech_create: A must be > 0, beta and Ea finite" + ri);
        }
        if (d->ord_ptr && d->ord_ptr[i + 1] > d->ord_ptr[i]) {
            if (!d->ord_sp || !d->ord_val || d->ord_ptr[i] < 0)
                return fail(KX_EINVAL, "kx_mech_create: bad order arrays" + ri);
            if (d->reversible[i])
                return fail(KX_EINVAL, "kx_mech_create: explicit orders need an "
                                       "irreversible reaction" + ri);
            for (int e = d->ord_ptr[i]; e < d->ord_ptr[i + 1]; ++e) {
                if (d->ord_sp[e] < 0 || d->ord_sp[e] >= ns)
                    return fail(KX_EINVAL, "kx_mech_create: order species out of range" + ri);
                if (!(d->ord_val[e] >= 0.0) || !std::isfinite(d->ord_val[e]))
                    return fail(KX_EINVAL, "kx_mech_create: orders must be finite and >= 0" +
                                               ri);
                for (int f = d->ord_ptr[i]; f < e; ++f)
                    if (d->ord_sp[f] == d->ord_sp[e])
                        return fail(KX_EINVAL, "kx_mech_create: order listed twice" + ri);
            }
        }
        if (d->chem_act && d->chem_act[i] && !falloff)
            return fail(KX_EINVAL, "kx_mech_create: chem_act on a reaction that is not a "
                                   "falloff reaction" + ri);
        if (t == KX_RXN_SRI) {
            if (!d->sri) return fail(KX_EINVAL, "kx_mech_create: NULL sri array" + ri);
            const double *q = d->sri + 5 * i;
            for (int j = 0; j < 5; ++j)
                if (!std::isfinite(q[j]))
                    return fail(KX_EINVAL, "kx_mech_create: SRI parameters must be finite" + ri);
            if (!(q[0] >= 0.0) || !(q[2] != 0.0) || !(q[3] > 0.0))
                return fail(KX_EINVAL, "kx_mech_create: SRI needs a >= 0, c != 0, d > 0" + ri);
        }
        if (falloff &&
            (!(d->A0[i] > 0.0) || !std::isfinite(d->beta0[i]) || !std::isfinite(d->Ea0[i])))
            return fail(KX_EINVAL, "kx_mech_create: falloff A0 must be > 0" + ri);
        if (t == KX_RXN_TROE && (!(d->troe[4 * i + 1] != 0.0) || !(d->troe[4 * i + 2] != 0.0)))
            return fail(KX_EINVAL, "kx_mech_create: Troe T*** and T* must be non-zero" + ri);
        std::vector<long> bal(ne, 0);
        for (int side = 0; side < 2; ++side) {
            const int32_t *ptr = side ? d->prod_ptr : d->reac_ptr;
            const int32_t *sp = side ? d->prod_sp : d->reac_sp;
            const int32_t *nu = side ? d->prod_nu : d->reac_nu;
            if (ptr[i] < 0 || ptr[i + 1] < ptr[i])
                return fail(KX_EINVAL, "kx_mech_create: bad CSR pointer" + ri);
            long molecules = 0;
            for (int e = ptr[i]; e < ptr[i + 1]; ++e) molecules += nu[e] > 0 ? nu[e] : 0;
            if (molecules > kMaxSide)
                return fail(KX_EUNSUPPORTED,
                            "kx_mech_create: more than 3 molecules on one side" + ri);
            for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
                if (sp[e] < 0 || sp[e] >= ns)
                    return fail(KX_EINVAL, "kx_mech_create: species index out of range" + ri);
                if (nu[e] <= 0 || nu[e] > 255)
                    return fail(KX_EINVAL, "kx_mech_create: nu must be in 1..255" + ri);
                for (int f = ptr[i]; f < e; ++f)
                    if (sp[f] == sp[e])
                        return fail(KX_EINVAL,
                                    "kx_mech_create: species listed twice on one side" + ri);
                for (int el = 0; el < ne; ++el)
                    bal[el] += (side ? 1 : -1) * (long)nu[e] * d->composition[sp[e] * ne + el];
            }
        }
        for (int el = 0; el < ne; ++el)
            if (bal[el] != 0)
                return fail(KX_EINVAL, "kx_mech_create: reaction is not element-balanced" + ri);
        if (t != KX_RXN_ELEMENTARY && t != KX_RXN_PLOG) {
            if (d->eff_ptr[i] < 0 || d->eff_ptr[i + 1] < d->eff_ptr[i])
                return fail(KX_EINVAL, "kx_mech_create: bad efficiency CSR" + ri);
            for (int e = d->eff_ptr[i]; e < d->eff_ptr[i + 1]; ++e)
                if (!d->eff_sp || !d->eff_val || d->eff_sp[e] < 0 || d->eff_sp[e] >= ns)
                    return fail(KX_EINVAL, "kx_mech_create: efficiency species out of range" + ri);
        }
    }
    if (d->qss) return validate_qss(d);
    return KX_OK;
}

}  // namespace

namespace {
std::atomic<uint64_t> next_uid{0};
}  // namespace

kx_status build_mech(const kx_mech_desc *d, int device, bool host_only, kx_mech **out)
{
    if (!out) return fail(KX_EINVAL, "kx_mech_create: out is NULL");
    *out = nullptr;
    std::vector<double> W;
    kx_status st = validate(d, W);
    if (st != KX_OK) return st;
    const int ns = d->n_species, nr = d->n_reactions, order = d->fit_order;

    // ---- reaction order: heaviest type first, constant-k_f last within a type
    std::vector<int> perm(nr);
    std::iota(perm.begin(), perm.end(), 0);
    auto kfconst = [&](int i) {
        return d->rxn_type[i] != KX_RXN_PLOG && d->beta[i] == 0.0 && d->Ea[i] == 0.0;
    };
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
        if (d->rxn_type[a] != d->rxn_type[b]) return d->rxn_type[a] > d->rxn_type[b];
        return !kfconst(a) && kfconst(b);
    });

    std::vector<DevRxn> rx(nr);
    std::vector<DevAux> aux;
    std::vector<DevEff> eff;
    std::vector<DevPlog> plog;
    for (int s = 0; s < nr; ++s) {
        const int i = perm[s];
        DevRxn r;
        std::memset(&r, 0, sizeof r);
        r.lnA = std::log(d->A[i]);
        r.beta = d->beta[i];
        r.ER = d->Ea[i] / kRcal;
        r.A = d->A[i];
        const uint16_t dummy = (uint16_t)(16 * ns);
        for (int q = 0; q < kMaxSide; ++q) r.roff[q] = r.poff[q] = dummy;
        int c = 0;
        for (int e = d->reac_ptr[i]; e < d->reac_ptr[i + 1]; ++e)
            for (int v = 0; v < d->reac_nu[e]; ++v) r.roff[c++] = (uint16_t)(16 * d->reac_sp[e]);
        c = 0;
        for (int e = d->prod_ptr[i]; e < d->prod_ptr[i + 1]; ++e)
            for (int v = 0; v < d->prod_nu[e]; ++v) r.poff[c++] = (uint16_t)(16 * d->prod_sp[e]);
        r.type = (uint8_t)d->rxn_type[i];
        r.flags = (d->reversible[i] ? kFlagReversible : 0) | (kfconst(i) ? kFlagKfConst : 0) |
                  (d->chem_act && d->chem_act[i] ? kFlagChemAct : 0);
        if (r.type == KX_RXN_PLOG) {  // k_f comes from the pressure table
            r.lnA = 0.0;
            r.beta = r.ER = 0.0;
            r.A = 1.0;
        }
        // forward orders: reactants at nu' unless listed, listed species at
        // their order; zero orders dropped
        std::vector<std::pair<int, double>> ord;
        const bool has_ord = d->ord_ptr && d->ord_ptr[i + 1] > d->ord_ptr[i];
        if (has_ord) {
            for (int e = d->reac_ptr[i]; e < d->reac_ptr[i + 1]; ++e)
                ord.push_back({d->reac_sp[e], (double)d->reac_nu[e]});
            for (int e = d->ord_ptr[i]; e < d->ord_ptr[i + 1]; ++e) {
                bool found = false;
                for (auto &o : ord)
                    if (o.first == d->ord_sp[e]) {
                        o.second = d->ord_val[e];
                        found = true;
                    }
                if (!found) ord.push_back({d->ord_sp[e], d->ord_val[e]});
            }
            ord.erase(std::remove_if(ord.begin(), ord.end(),
                                     [](const std::pair<int, double> &o) { return o.second == 0.0; }),
                      ord.end());
            if ((int)ord.size() > kMaxOrd)
                return fail(KX_EUNSUPPORTED, "kx_mech_create: more than 4 species with "
                                             "explicit orders (reaction " + std::to_string(i) + ")");
            r.flags |= kFlagOrders;
        }
        r.aux = 0xFFFF;
        if (r.type != KX_RXN_ELEMENTARY || has_ord) {
            if (aux.size() >= 0xFFFF)
                return fail(KX_EUNSUPPORTED, "kx_mech_create: too many non-elementary reactions");
            DevAux a;
            std::memset(&a, 0, sizeof a);
            const bool collider = r.type != KX_RXN_PLOG && r.type != KX_RXN_ELEMENTARY;
            a.eff_default = collider ? d->eff_default[i] : 0.0;
            for (int q = 0; q < kInlineEff; ++q) {
                a.eoff[q] = (uint16_t)(16 * ns);  // dummy species, alpha - default = 0
                a.dalpha[q] = 0.0;
            }
            int q = 0;
            a.ext_off = (int32_t)eff.size();
            const int e0 = collider ? d->eff_ptr[i] : 0, e1 = collider ? d->eff_ptr[i + 1] : 0;
            for (int e = e0; e < e1; ++e) {
                const double da = d->eff_val[e] - d->eff_default[i];
                if (q < kInlineEff) {
                    a.eoff[q] = (uint16_t)(16 * d->eff_sp[e]);
                    a.dalpha[q] = da;
                    ++q;
                } else {
                    DevEff f;
                    std::memset(&f, 0, sizeof f);
                    f.sp = d->eff_sp[e];
                    f.dalpha = da;
                    eff.push_back(f);
                }
            }
            a.ext_cnt = (int32_t)eff.size() - a.ext_off;
            if (r.type == KX_RXN_LINDEMANN || r.type == KX_RXN_TROE || r.type == KX_RXN_SRI) {
                a.lnA0 = std::log(d->A0[i]);
                a.beta0 = d->beta0[i];
                a.ER0 = d->Ea0[i] / kRcal;
            }
            if (r.type == KX_RXN_TROE) {
                a.fp[0] = d->troe[4 * i + 0];
                a.fp[1] = 1.0 / d->troe[4 * i + 1];
                a.fp[2] = 1.0 / d->troe[4 * i + 2];
                a.has_T2 = std::isnan(d->troe[4 * i + 3]) ? 0 : 1;
                a.fp[3] = a.has_T2 ? d->troe[4 * i + 3] : 0.0;
            }
            if (r.type == KX_RXN_SRI) {
                const double *q = d->sri + 5 * i;
                a.fp[0] = q[0];
                a.fp[1] = q[1];
                a.fp[2] = 1.0 / q[2];
                a.fp[3] = std::log(q[3]);
                a.fp[4] = q[4];
            }
            for (int q = 0; q < kMaxOrd; ++q) {
                a.ooff[q] = (uint16_t)(16 * ns);
                a.oval[q] = 0.0;
            }
            for (size_t q = 0; q < ord.size(); ++q) {
                a.ooff[q] = (uint16_t)(16 * ord[q].first);
                a.oval[q] = ord[q].second;
            }
            if (r.type == KX_RXN_PLOG) {
                a.plog_off = (int32_t)plog.size();
                a.plog_cnt = d->plog_ptr[i + 1] - d->plog_ptr[i];
                for (int j = d->plog_ptr[i]; j < d->plog_ptr[i + 1]; ++j) {
                    DevPlog e;
                    std::memset(&e, 0, sizeof e);
                    e.lnp = std::log(d->plog_p[j]);
                    e.lnA = std::log(d->plog_A[j]);
                    e.beta = d->plog_beta[j];
                    e.ER = d->plog_Ea[j] / kRcal;
                    e.inv_dlnp = j + 1 < d->plog_ptr[i + 1]
                                     ? 1.0 / (std::log(d->plog_p[j + 1]) - e.lnp) : 0.0;
                    plog.push_back(e);
                }
            }
            r.aux = (uint16_t)aux.size();
            aux.push_back(a);
        }
        rx[s] = r;
    }
    if (eff.empty()) eff.resize(1);
    if (aux.empty()) aux.resize(1);
    if (plog.empty()) plog.resize(1);

    // ---- species-major gather lists per reaction chunk.  Each species lists
    // the chunk slots of the reactions that produce it (+q, once per unit of
    // net nu) and of those that consume it (-q); both lists are padded to a
    // whole number of eight-entry groups common to all lanes, and a group is
    // eight 32-bit LDS offsets (32 bytes per lane, so lane k reads it with a
    // pair of coalesced 16-byte loads).  The rates of progress of two points sit
    // side by side in LDS, so one offset addresses both.
    const int chunk = std::max(kWave, std::min(kChunkMax, (nr + kWave - 1) / kWave * kWave));
    const int nchunks = std::max(1, (nr + chunk - 1) / chunk);
    // species per lane of the species phases: 1, 2 or 4 (the kernels are
    // instantiated for these), so lists are laid out for 64 * gpass lanes
    const int gpass = ns <= kWave ? 1 : (ns <= 2 * kWave ? 2 : 4);
    const int gw = kWave * gpass;
    std::vector<int32_t> gpos(nchunks), gneg(nchunks), goff(nchunks);
    std::vector<uint32_t> gent;  // 8 per (group, lane)
    size_t ngroups = 0;
    std::vector<int32_t> mgrp(nchunks), moff(nchunks);
    std::vector<uint32_t> ment;  // signed lists of the rates kernel, 8 per (group, lane)
    size_t nmgroups = 0;
    for (int c = 0; c < nchunks; ++c) {
        std::vector<std::vector<uint32_t>> pos(gw), neg(gw);
        for (int s = c * chunk; s < std::min(nr, (c + 1) * chunk); ++s) {
            const int i = perm[s];
            std::vector<std::pair<int, int>> net;  // (species, nu'' - nu')
            auto addnu = [&](int k, int v) {
                for (auto &pr : net)
                    if (pr.first == k) { pr.second += v; return; }
                net.push_back({k, v});
            };
            for (int e = d->reac_ptr[i]; e < d->reac_ptr[i + 1]; ++e)
                addnu(d->reac_sp[e], -d->reac_nu[e]);
            for (int e = d->prod_ptr[i]; e < d->prod_ptr[i + 1]; ++e)
                addnu(d->prod_sp[e], d->prod_nu[e]);
            const uint32_t slot = (uint32_t)(16 * (s - c * chunk));
            for (auto &pr : net)
                for (int u = 0; u < std::abs(pr.second); ++u)
                    (pr.second > 0 ? pos : neg)[pr.first].push_back(slot);
        }
        size_t lp = 0, ln = 0;
        for (int k = 0; k < gw; ++k) {
            lp = std::max(lp, pos[k].size());
            ln = std::max(ln, neg[k].size());
        }
        gpos[c] = (int32_t)((lp + 7) / 8);
        gneg[c] = (int32_t)((ln + 7) / 8);
        goff[c] = (int32_t)ngroups;
        // the rates kernel's lists: one list per species with the sign of each
        // entry in bit 31 (+q entries first), padded to whole groups of eight
        {
            size_t lm = 0;
            for (int k = 0; k < gw; ++k) lm = std::max(lm, pos[k].size() + neg[k].size());
            mgrp[c] = (int32_t)((lm + 7) / 8);
            moff[c] = (int32_t)nmgroups;
            const uint32_t zpad = (uint32_t)(16 * chunk);
            for (int g = 0; g < mgrp[c]; ++g)
                for (int k = 0; k < gw; ++k)
                    for (int u = 0; u < 8; ++u) {
                        const size_t e = (size_t)g * 8 + u;
                        const size_t np_ = pos[k].size();
                        uint32_t v = zpad;
                        if (e < np_)
                            v = pos[k][e];
                        else if (e < np_ + neg[k].size())
                            v = neg[k][e - np_] | 0x80000000u;
                        ment.push_back(v);
                    }
            nmgroups += mgrp[c];
        }
        const uint32_t pad = (uint32_t)(16 * chunk);  // the zero slot
        for (int side = 0; side < 2; ++side) {
            const auto &lists = side ? neg : pos;
            const int groups = side ? gneg[c] : gpos[c];
            for (int g = 0; g < groups; ++g)
                for (int k = 0; k < gw; ++k)
                    for (int u = 0; u < 8; ++u) {
                        const size_t e = (size_t)g * 8 + u;
                        gent.push_back(e < lists[k].size() ? lists[k][e] : pad);
                    }
            ngroups += groups;
        }
    }
    if (gent.empty()) gent.resize(8, 0);
    if (ment.empty()) ment.resize(8, 0);

    // ---- QSS species: index per species, per reaction (kernel order) the QSS
    // species of either side, and per QSS species the reactions of its balance
    int nq = 0;
    std::vector<int32_t> qidx(ns, -1);
    if (d->qss)
        for (int k = 0; k < ns; ++k)
            if (d->qss[k]) qidx[k] = nq++;
    std::vector<int2> qrx(std::max(nr, 1), int2{-1, -1});
    std::vector<int32_t> qrow_ptr(nq + 1, 0);
    std::vector<int4> qrow_ent;
    if (nq > 0) {
        for (int s = 0; s < nr; ++s) {
            int c = 0;
            const int a = qss_side(d, perm[s], false, &c), b = qss_side(d, perm[s], true, &c);
            qrx[s] = int2{a >= 0 ? qidx[a] : -1, b >= 0 ? qidx[b] : -1};
        }
        for (int k = 0; k < ns; ++k) {
            if (qidx[k] < 0) continue;
            for (int s = 0; s < nr; ++s) {
                const int nu = net_nu(d, perm[s], k);
                // x: the reaction's LDS slot in the QSS kernel (a zero slot
                // follows each chunk, so reaction s sits at s + s / chunk)
                if (nu != 0) qrow_ent.push_back(int4{s + s / chunk, nu, qrx[s].x, qrx[s].y});
            }
            qrow_ptr[qidx[k] + 1] = (int32_t)qrow_ent.size();
        }
    }
    if (qrow_ent.empty()) qrow_ent.push_back(int4{0, 0, -1, -1});

    // ---- species thermo
    std::vector<DevSpecies> spv(ns);
    for (int k = 0; k < ns; ++k) {
        DevSpecies s;
        std::memset(&s, 0, sizeof s);
        for (int r = 0; r < 2; ++r) {
            const double *a = (r ? d->nasa_hi : d->nasa_lo) + 7 * k;
            double *g = r ? s.g_hi : s.g_lo;
            g[0] = a[0];
            g[1] = -a[1] / 2.0;
            g[2] = -a[2] / 6.0;
            g[3] = -a[3] / 12.0;
            g[4] = -a[4] / 20.0;
            g[5] = a[5];
            g[6] = -a[6];
            std::memcpy(r ? s.nasa_hi : s.nasa_lo, a, 7 * sizeof(double));
        }
        s.t_mid = d->t_mid[k];
        s.inv_W = 1.0 / W[k];
        spv[k] = s;
    }
    std::vector<double> gsoa((size_t)((ns + kWave - 1) / kWave) * 16 * kWave, 0.0);
    for (int k = 0; k < ns; ++k) {
        double *g = gsoa.data() + (size_t)(k / kWave) * 16 * kWave + k % kWave;
        for (int e = 0; e < 7; ++e) {
            g[e * kWave] = spv[k].g_lo[e];
            g[(7 + e) * kWave] = spv[k].g_hi[e];
        }
        g[14 * kWave] = spv[k].t_mid;
        g[15 * kWave] = spv[k].inv_W;
    }

    // ---- transport tables
    const int nkb = (ns + kKB - 1) / kKB;
    std::vector<double> visc((size_t)ns * order), cond((size_t)ns * order);
    std::memcpy(visc.data(), d->visc_fit, visc.size() * sizeof(double));
    std::memcpy(cond.data(), d->cond_fit, cond.size() * sizeof(double));
    std::vector<double> wilke((size_t)nkb * ns * kKB, 0.0), wq(ns);
    for (int k = 0; k < ns; ++k) wq[k] = std::pow(W[k], 0.25);
    std::vector<double> dfit((size_t)nkb * ns * kKB * order, 0.0);
    std::vector<double> ddiag((size_t)ns * order);
    for (int kb = 0; kb < nkb; ++kb)
        for (int j = 0; j < ns; ++j)
            for (int kk = 0; kk < kKB; ++kk) {
                const int k = kb * kKB + kk;
                if (k >= ns) {
                    // padding rows of the last block: a fit identically 1 keeps
                    // the branch-free pair loop finite (their sums are unused)
                    dfit[(((size_t)kb * ns + j) * kKB + kk) * order] = 1.0;
                    continue;
                }
                // phi_kj = c1_kj (1 + sigma_k rho_j)^2 with c2_kj = (W_j/W_k)^(1/4)
                // = wq_j / wq_k folded into the per-species factors
                wilke[((size_t)kb * ns + j) * kKB + kk] = 1.0 / std::sqrt(8.0 * (1.0 + W[k] / W[j]));
                std::memcpy(&dfit[(((size_t)kb * ns + j) * kKB + kk) * order],
                            d->diff_fit + ((size_t)k * ns + j) * order, order * sizeof(double));
            }
    for (int k = 0; k < ns; ++k)
        std::memcpy(&ddiag[(size_t)k * order], d->diff_fit + ((size_t)k * ns + k) * order,
                    order * sizeof(double));
    auto to32 = [](const std::vector<double> &v) {
        return std::vector<float>(v.begin(), v.end());
    };

    // ---- MFMA fragments of the quadratic sums (fits of 1/D_kj only)
    const int mblk = (ns + 15) / 16, kstep = (ns + 3) / 4;
    const bool mfma = d->diff_fit_kind == 1;
    std::vector<double> gfrag, c1frag;
    if (mfma) {
        gfrag.assign((size_t)order * mblk * kstep * 64, 0.0);
        c1frag.assign((size_t)mblk * kstep * 64, 0.0);
        for (int mb = 0; mb < mblk; ++mb)
            for (int ks = 0; ks < kstep; ++ks)
                for (int l = 0; l < 64; ++l) {
                    const int k = 16 * mb + l % 16, j = 4 * ks + l / 16;
                    if (k >= ns || j >= ns) continue;
                    c1frag[((size_t)mb * kstep + ks) * 64 + l] =
                        1.0 / std::sqrt(8.0 * (1.0 + W[k] / W[j]));
                    if (j == k) continue;
                    for (int o = 0; o < order; ++o)
                        gfrag[(((size_t)o * mblk + mb) * kstep + ks) * 64 + l] =
                            d->diff_fit[((size_t)k * ns + j) * order + o];
                }
    } else {
        gfrag.resize(1);
        c1frag.resize(1);
    }

    Blob b;
    const size_t o_rxn = add_vec(b, rx), o_aux = add_vec(b, aux), o_eff = add_vec(b, eff);
    const size_t o_plog = add_vec(b, plog);
    const size_t o_sp = add_vec(b, spv), o_gpos = add_vec(b, gpos), o_gneg = add_vec(b, gneg);
    const size_t o_gsoa = add_vec(b, gsoa);
    const size_t o_goff = add_vec(b, goff);
    const size_t o_gent = add_vec(b, gent);
    const size_t o_mgrp = add_vec(b, mgrp), o_moff = add_vec(b, moff), o_ment = add_vec(b, ment);
    const size_t o_W = add_vec(b, W), o_visc = add_vec(b, visc), o_cond = add_vec(b, cond);
    const size_t o_wil = add_vec(b, wilke), o_df = add_vec(b, dfit), o_dd = add_vec(b, ddiag);
    const size_t o_wq = add_vec(b, wq), o_wq32 = add_vec(b, to32(wq));
    const size_t o_visc32 = add_vec(b, to32(visc)), o_cond32 = add_vec(b, to32(cond));
    const size_t o_wil32 = add_vec(b, to32(wilke)), o_df32 = add_vec(b, to32(dfit));
    const size_t o_dd32 = add_vec(b, to32(ddiag));
    const size_t o_gf = add_vec(b, gfrag), o_c1f = add_vec(b, c1frag);
    const size_t o_gf32 = add_vec(b, to32(gfrag)), o_c1f32 = add_vec(b, to32(c1frag));
    const size_t o_qidx = add_vec(b, qidx), o_qrx = add_vec(b, qrx);
    const size_t o_qptr = add_vec(b, qrow_ptr), o_qent = add_vec(b, qrow_ent);

    void *blob = nullptr;
    if (!host_only) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        e = hipSetDevice(device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        e = hipMalloc(&blob, b.host.size());
        if (e != hipSuccess) {
            hipSetDevice(prev);
            return fail(KX_ENOMEM, "kx_mech_create: hipMalloc of " +
                                       std::to_string(b.host.size()) + " bytes failed");
        }
        e = hipMemcpy(blob, b.host.data(), b.host.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            hipFree(blob);
            hipSetDevice(prev);
            return hip_fail(e, "hipMemcpy (mechanism upload)");
        }
        hipSetDevice(prev);
    }

    kx_mech *m = new kx_mech;
    m->device = host_only ? -1 : device;
    m->blob = blob;
    m->bytes = (int64_t)b.host.size();
    m->n_species = ns;
    m->uid = next_uid.fetch_add(1) + 1;
    m->n_reactions = nr;
    MechDev &v = m->dev;
    // device addresses of the tables (null for a host-only handle)
    auto at = [&](size_t off) {
        return blob ? (const void *)((const uint8_t *)blob + off) : (const void *)nullptr;
    };
    v.ns = ns;
    v.nr = nr;
    v.chunk = chunk;
    v.nchunks = nchunks;
    v.gpass = gpass;
    v.fit_order = order;
    v.diff_kind = d->diff_fit_kind;
    v.fit_L0 = d->fit_L0;
    v.inv_fit_h = 1.0 / d->fit_h;
    v.rxn = (const DevRxn *)at(o_rxn);
    v.aux = (const DevAux *)at(o_aux);
    v.eff = (const DevEff *)at(o_eff);
    v.plog = (const DevPlog *)at(o_plog);
    v.sp = (const DevSpecies *)at(o_sp);
    v.gsoa = (const double *)at(o_gsoa);
    v.gpos = (const int32_t *)at(o_gpos);
    v.gneg = (const int32_t *)at(o_gneg);
    v.goff = (const int32_t *)at(o_goff);
    v.gent = (const uint4 *)at(o_gent);
    v.gmgrp = (const int32_t *)at(o_mgrp);
    v.gmoff = (const int32_t *)at(o_moff);
    v.gment = (const uint4 *)at(o_ment);
    v.W = (const double *)at(o_W);
    v.visc = (const double *)at(o_visc);
    v.cond = (const double *)at(o_cond);
    v.wilke = (const double *)at(o_wil);
    v.wq = (const double *)at(o_wq);
    v.wq32 = (const float *)at(o_wq32);
    v.dfit = (const double *)at(o_df);
    v.ddiag = (const double *)at(o_dd);
    v.visc32 = (const float *)at(o_visc32);
    v.cond32 = (const float *)at(o_cond32);
    v.wilke32 = (const float *)at(o_wil32);
    v.dfit32 = (const float *)at(o_df32);
    v.ddiag32 = (const float *)at(o_dd32);
    v.mblk = mblk;
    v.kstep = kstep;
    v.gfrag = mfma ? (const double *)at(o_gf) : nullptr;
    v.c1frag = mfma ? (const double *)at(o_c1f) : nullptr;
    v.gfrag32 = mfma ? (const float *)at(o_gf32) : nullptr;
    v.c1frag32 = mfma ? (const float *)at(o_c1f32) : nullptr;
    v.nq = nq;
    v.nqent = nq > 0 ? qrow_ptr[nq] : 0;
    v.qidx = (const int32_t *)at(o_qidx);
    v.qrx = (const int2 *)at(o_qrx);
    v.qrow_ptr = (const int32_t *)at(o_qptr);
    v.qrow_ent = (const int4 *)at(o_qent);
    *out = m;
    return ok();
}

bool rebase_tables(const kx_mech *m, const void *base, MechDev *out)
{
    MechDev v = m->dev;
    const char *old = static_cast<const char *>(m->blob);
    const char *nb = static_cast<const char *>(base);
#define KX_REBASE(f) \
    v.f = m->dev.f ? reinterpret_cast<decltype(v.f)>(nb + (reinterpret_cast<const char *>(m->dev.f) - old)) \
                   : nullptr
    KX_REBASE(rxn); KX_REBASE(aux); KX_REBASE(eff); KX_REBASE(plog); KX_REBASE(sp);
    KX_REBASE(gsoa);
    KX_REBASE(gpos); KX_REBASE(gneg); KX_REBASE(goff); KX_REBASE(gent);
    KX_REBASE(gmgrp); KX_REBASE(gmoff); KX_REBASE(gment);
    KX_REBASE(W); KX_REBASE(visc); KX_REBASE(cond); KX_REBASE(wq); KX_REBASE(wilke);
    KX_REBASE(dfit); KX_REBASE(ddiag);
    KX_REBASE(visc32); KX_REBASE(cond32); KX_REBASE(wq32); KX_REBASE(wilke32);
    KX_REBASE(dfit32); KX_REBASE(ddiag32);
    KX_REBASE(gfrag); KX_REBASE(c1frag); KX_REBASE(gfrag32); KX_REBASE(c1frag32);
    KX_REBASE(qidx); KX_REBASE(qrow_ptr); KX_REBASE(qrow_ent); KX_REBASE(qrx);
#undef KX_REBASE
    // every table pointer must have moved: no 8-byte word of the result may
    // still address the original tables
    uintptr_t words[sizeof(MechDev) / sizeof(uintptr_t)];
    std::memcpy(words, &v, sizeof words);
    const uintptr_t lo = reinterpret_cast<uintptr_t>(old), hi = lo + (uintptr_t)m->bytes;
    for (uintptr_t w : words)
        if (w >= lo && w < hi) return false;
    *out = v;
    return true;
}

}  // namespace kx
