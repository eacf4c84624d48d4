/*
 * kx.h -- C ABI of the MI355X (gfx950) per-grid-point chemistry library.
 *
 * The library evaluates, independently for every grid point of a reacting-flow
 * field, the quantities of Danciu & Frouzakis, "KinetiX: A performance
 * portable code generator for chemical kinetics and transport properties"
 * (arXiv 2411.02640), Appendix A:
 *   - species net production rates wdot_k = sum_i nu_ki R_i (App. A.2) from
 *     modified-Arrhenius forward rates (eq:arrhenius), equilibrium constants
 *     from NASA-7 Gibbs energies (eq:K_p, eq:Ck), third-body and
 *     Lindemann / Troe falloff modifiers (eq:c_i, eq:blend) and the law of mass
 *     action (eq:r_i);
 *   - mixture-averaged transport (App. A.3): Wilke / Bird viscosity, Mathur
 *     conductivity and mixture-averaged diffusion coefficients (eq:mix_diff)
 *     from ln T polynomial fits of the pure-species viscosity, conductivity and
 *     binary diffusion coefficients (eq:Dkj);
 *   - mixture thermodynamics cp_k, h_k and cp (App. A.1).
 *
 * Conventions shared by every entry point
 *   Units      cgs: T in K, p in dyn/cm^2 (1 atm = 1013250), concentrations in
 *              mol/cm^3, wdot in mol/(cm^3 s), mu in g/(cm s), lambda in
 *              erg/(cm s K), D in cm^2/s, cp in erg/(g K), h in erg/g; Arrhenius
 *              A in (cm^3/mol)^(order-1)/s and E_a in cal/mol.
 *   Layout     structure of arrays.  Point arrays T[n], p[n]; per-species
 *              arrays are species-major, element (k, i) at k*n + i (Y, wdot,
 *              Dmix, cp_k, h_k).  Every point array is a DEVICE pointer on the
 *              handle's device, 8-byte aligned, contiguous; outputs must not
 *              alias inputs or each other.
 *   Asynchrony Compute calls only enqueue work on `stream` (0 = the legacy
 *              default stream).  KX_OK means "enqueued"; results are ready once
 *              the stream is synchronised.  Device faults surface at that sync.
 *   Arguments  Validated on the host: a NULL handle or pointer, n < 0, or an
 *              unknown precision return KX_EINVAL; n == 0 is a no-op
 *              returning KX_OK.  Point values are not checked on the device;
 *              preconditions are 200 <= T <= 3500, p > 0, Y_k >= 0, sum Y = 1.
 *   Threads    A handle is immutable after creation and may be used from any
 *              host thread and on any stream of its device concurrently.
 *              kx_last_error() is per host thread.
 *   Errors     Every entry point returns a kx_status; on failure nothing is
 *              enqueued and kx_last_error() describes the cause.
 */
#ifndef KX_H
#define KX_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kx_status;
enum {
    KX_OK = 0,
    KX_EINVAL = -1,        /* bad argument or inconsistent descriptor */
    KX_ENOMEM = -2,        /* device or host allocation failed, or over budget */
    KX_EDEVICE = -3,       /* HIP runtime error (launch, copy, device select) */
    KX_EUNSUPPORTED = -4,  /* valid input outside what the kernels implement */
    KX_EAGAIN = -5         /* serving: not complete yet / queue full */
};

/* Precision flag of the _ex entry points. */
enum {
    KX_FP64 = 0,   /* every operation in IEEE double precision */
    KX_MIXED = 1   /* FP32 for the exponentials' reduced arguments, the falloff
                      blend and the transport fits and pair sums; FP64 for the
                      rest (see kx_production_rates_ex and kx_transport_ex) */
};

/* Option of kx_transport_ex, OR-ed into its precision argument: for tables of
 * D_kj fits (diff_fit_kind 0) evaluate each unordered pair's fit once and let
 * its 1/D_kj enter both S_k and S_j (D_kj = D_jk; §2.2.2, §2.3.2), keeping the
 * sums of every species per point in LDS: one wave per 64 points, ns * 64
 * values of LDS (KX_EUNSUPPORTED beyond 160 KB, i.e. more than 320 species in
 * FP64).  Ignored for tables of 1/D_kj fits, whose sums run on the matrix
 * cores (or, below 24 species, on the vector units without a reciprocal per
 * pair). */
enum { KX_DKJ_SYMMETRIC = 0x100 };

/* Reaction types (App. A.2). */
enum {
    KX_RXN_ELEMENTARY = 0, /* c_i = 1 */
    KX_RXN_THREEBODY = 1,  /* c_i = [X]_i */
    KX_RXN_LINDEMANN = 2,  /* c_i = P_r/(1+P_r), F = 1 */
    KX_RXN_TROE = 3,       /* c_i = P_r/(1+P_r) F_Troe (eq:blend) */
    KX_RXN_SRI = 4,        /* c_i = P_r/(1+P_r) F_SRI (eq:blend, SRI form) */
    KX_RXN_PLOG = 5        /* c_i = 1, k_f interpolated in ln p between reference
                              pressures (App. A.2, pressure-dependent reactions) */
};

/* Mechanism descriptor.  Every array is HOST memory owned by the caller and
 * only read during kx_mech_create (it may be freed afterwards).  Row-major.
 * Ns = n_species, Nr = n_reactions, Ne = n_elements. */
typedef struct {
    int32_t n_species, n_reactions, n_elements;
    const double *elem_mass;      /* [Ne] g/mol; W_k = sum_e composition[k][e] elem_mass[e] */
    const int32_t *composition;   /* [Ns][Ne] atom counts */
    const double *nasa_lo;        /* [Ns][7] a0..a6 used when T <  t_mid[k] (App. A.1) */
    const double *nasa_hi;        /* [Ns][7] a0..a6 used when T >= t_mid[k] */
    const double *t_mid;          /* [Ns] K */
    const int32_t *rxn_type;      /* [Nr] KX_RXN_* */
    const int32_t *reversible;    /* [Nr] 0: k_r = 0; else k_r = k_f / K_c */
    const int32_t *reac_ptr;      /* [Nr+1] CSR of reactants; distinct species per reaction */
    const int32_t *reac_sp;       /*   species index */
    const int32_t *reac_nu;       /*   integer stoichiometric coefficient nu' > 0 */
    const int32_t *prod_ptr;      /* [Nr+1] CSR of products, same rules (nu'' > 0) */
    const int32_t *prod_sp;
    const int32_t *prod_nu;
    const double *A, *beta, *Ea;     /* [Nr] Arrhenius (k_inf for falloff) */
    const double *A0, *beta0, *Ea0;  /* [Nr] low-pressure limit k_0 (falloff only) */
    const double *troe;           /* [Nr][4] alpha, T***, T*, T** (T** = NaN: term omitted) */
    const int32_t *eff_ptr;       /* [Nr+1] CSR of third-body efficiencies that differ */
    const int32_t *eff_sp;        /*   from eff_default (third-body and falloff only) */
    const double *eff_val;        /*   alpha_ki */
    const double *eff_default;    /* [Nr] efficiency of unlisted species (1 = [M]; 0 with
                                     one listed species m of efficiency 1 = [X_m]) */
    int32_t fit_order;            /* coefficients per fit, 1..8 (5 in the paper) */
    double fit_L0, fit_h;         /* fits are polynomials in u = (ln T - fit_L0) / fit_h;
                                     (0, 1) is the paper's literal ln T basis */
    int32_t diff_fit_kind;        /* 0: diff_fit holds D_kj(T, 1 atm) (eq:Dkj);
                                     1: diff_fit holds 1 / D_kj(T, 1 atm) */
    const double *visc_fit;       /* [Ns][order] eta_k(u), constant term first */
    const double *cond_fit;       /* [Ns][order] lambda_k(u) */
    const double *diff_fit;       /* [Ns][Ns][order], symmetric in (k, j); the diagonal
                                     is used only when sum_{j!=k} X_j/D_kj == 0 */
    /* Further reaction forms (App. A.2).  Each pointer may be NULL when no
     * reaction uses it. */
    const double *sri;            /* [Nr][5] a, b, c, d, e of KX_RXN_SRI reactions:
                                     F = d T^e [a exp(-b/T) + exp(-T/c)]^X with
                                     X = 1 / (1 + log10(P_r)^2); a >= 0, c != 0,
                                     d > 0 (d = 1, e = 0 when a mechanism gives three) */
    const int32_t *chem_act;      /* [Nr] nonzero marks a chemically activated falloff
                                     reaction (types LINDEMANN, TROE, SRI): c_i =
                                     F/(1+P_r) (eq:c_i) and r_i uses k_0 in place of
                                     k_inf, i.e. k_f = k_0 F/(1+P_r) */
    const int32_t *plog_ptr;      /* [Nr+1] CSR of the reference pressures of KX_RXN_PLOG
                                     reactions (at least one each; empty for the other
                                     types, whose entries are not read) */
    const double *plog_p;         /*   reference pressure p_j > 0, dyn/cm^2, strictly
                                     increasing within a reaction */
    const double *plog_A, *plog_beta, *plog_Ea;  /* Arrhenius k_j(T) at p_j.  ln k_f is
                                     linear in ln p between neighbouring p_j; below the
                                     first (above the last) pressure k_f is that point's
                                     k_j.  A, beta, Ea of a PLOG reaction are not read. */
    const int32_t *ord_ptr;       /* [Nr+1] CSR of explicit forward reaction orders (may be
                                     NULL): the forward rate of progress is
                                     k_f prod_k [X_k]^o_k with o_k the listed order, or
                                     nu'_k for a reactant not listed; only for
                                     irreversible reactions, at most 4 species with a
                                     non-zero order per reaction */
    const int32_t *ord_sp;        /*   species index */
    const double *ord_val;        /*   order o_k >= 0 (need not be an integer) */
    /* Quasi-steady-state species (the paper plans them, §4; linearised QSSA of
     * Lu & Law 2006).  May be NULL.  qss[k] = 1 marks species k as quasi-steady:
     * it is not transported, and its concentration follows at every point from
     * its balance wdot_k = 0.  Requirements (checked at create): at most 64 QSS
     * species and at least one other; at most one QSS molecule on either side
     * of every reaction (so the balances are linear in the QSS
     * concentrations); no QSS species in an efficiency list or in a reaction
     * with explicit orders; every QSS species consumed by some reaction (a
     * reactant, or a product of a reversible reaction, with non-zero net nu).
     * The flags change kx_production_rates only: kx_transport and kx_thermo
     * treat QSS species like the others, with their Y entries as given. */
    const int32_t *qss;           /* [Ns] 0 or 1 */
} kx_mech_desc;

typedef struct kx_mech kx_mech; /* opaque device-resident mechanism */

/* Validate `desc`, derive the device tables (reaction order, scaled Gibbs
 * coefficients, stoichiometry and efficiency lists, Wilke constants, fit
 * tables) and upload them to `device`.  Rejects (KX_EINVAL) negative or zero
 * sizes, out-of-range species indices, non-positive W_k or A, a species listed
 * twice on one side of a reaction, unbalanced element counts, an unknown
 * reaction type, a non-symmetric diff_fit, fit_order outside 1..8,
 * fit_h == 0, SRI parameters outside their ranges, chem_act set on a reaction
 * that is not a falloff reaction, PLOG tables that are empty, not
 * increasing in pressure or with A <= 0, and explicit orders on a reversible
 * reaction or with a negative order, qss flags other than 0 / 1, a QSS
 * species that no reaction consumes, or no transported species.
 * KX_EUNSUPPORTED: more than 3 molecules (sum of nu) on one side
 * of a reaction, more than 4 species with a non-zero explicit order, more
 * than 256 species, more than 64 QSS species, two QSS molecules on one side
 * of a reaction, or a QSS species in an efficiency list or in a reaction with
 * explicit orders.  On success *out owns the tables until
 * kx_mech_destroy.  Allocates device memory (hipMalloc); blocks until the
 * upload is complete. */
kx_status kx_mech_create(const kx_mech_desc *desc, int device, kx_mech **out);

/* Validate `desc` and build the tables exactly as kx_mech_create does, without
 * a device: the handle reports kx_mech_info and can be used with a server
 * created with KX_SERVER_SIMULATE, but every compute call rejects it
 * (KX_EINVAL).  For checking descriptors and serving logic on a host. */
kx_status kx_mech_create_host(const kx_mech_desc *desc, kx_mech **out);

/* Free the device tables.  The caller must have synchronised every stream on
 * which work using `mech` was enqueued.  NULL is a no-op. */
kx_status kx_mech_destroy(kx_mech *mech);

/* Sizes of a created mechanism and the bytes of device memory its tables use
 * (any output may be NULL). */
kx_status kx_mech_info(const kx_mech *mech, int32_t *n_species, int32_t *n_reactions,
                       int64_t *device_bytes);

/* Net production rates wdot[Ns][n] (App. A.2: wdot_k = sum_i nu_ki c_i r_i with
 * eq:arrhenius, eq:K_p / eq:Ck for K_c, eq:c_i, eq:blend and eq:r_i) for n points
 * with temperature T[n], pressure p[n] and mass fractions Y[Ns][n].  Plain FP64.
 * For a mechanism with QSS species the concentrations of those species are
 * solved first (see kx_qss_concentrations) and enter the rates of progress;
 * the mixture is that of the transported species (W-bar from their mass
 * fractions, third-body sums over them), the QSS entries of Y are not read and
 * the QSS rows of wdot are written as 0 (their balance). */
kx_status kx_production_rates(const kx_mech *mech, int64_t n, const double *T,
                              const double *p, const double *Y, double *wdot,
                              hipStream_t stream);

/* As kx_production_rates with a precision flag.  KX_MIXED changes three steps
 * to FP32: the exponentials of the forward rate constants (eq:arrhenius) and of
 * the falloff ratio k_0/k_inf, whose arguments are formed and reduced by n ln 2
 * in FP64 so that only e^r, |r| <= ln2/2, is evaluated in FP32 (about 1e-7
 * relative); and the Troe / SRI blending factor F (eq:blend).  Everything else
 * stays FP64: the species Gibbs energies and K_c factors, the third-body sums,
 * the products of concentrations, the bracket of forward minus reverse terms,
 * and the wdot sum (Neumaier-compensated across groups of eight terms).  The
 * result is within 1e-5 of the FP64 value relative to s_k = sum_i |nu_ki|
 * |R_i| (the magnitude of the terms that cancel into wdot_k); where s_k >>
 * |wdot_k| the plain relative error can exceed 1e-5.  Inputs and outputs are
 * FP64 either way.  KX_MIXED on a mechanism with QSS species returns
 * KX_EUNSUPPORTED. */
kx_status kx_production_rates_ex(const kx_mech *mech, int64_t n, const double *T,
                                 const double *p, const double *Y, double *wdot,
                                 int32_t precision, hipStream_t stream);

/* Mixture-averaged transport for n points (App. A.3): mu[n] by Wilke / Bird,
 * lambda[n] by Mathur's combination averaging, Dmix[Ns][n] by eq:mix_diff
 * (falling back to D_kk where sum_{j!=k} X_j/D_kj is zero).  Pure-species
 * properties come from the ln T fits; D_kj = fit_kj * p_atm / p.  Plain FP64. */
kx_status kx_transport(const kx_mech *mech, int64_t n, const double *T, const double *p,
                       const double *Y, double *mu, double *lambda, double *Dmix,
                       hipStream_t stream);

/* As kx_transport with a precision flag (optionally | KX_DKJ_SYMMETRIC).
 * KX_MIXED evaluates the pure-species
 * fits, the Wilke factors and the pair sums (sum_j X_j phi_kj, sum_j X_j/D_kj)
 * in FP32 with FP32 accumulation; the mole fractions, W-bar, Mathur's two sums
 * over species, the final sum over species of mu and the D_km numerator
 * (W-bar - X_k W_k)/W-bar stay FP64.  Each output is within 1e-5 relative of
 * the FP64 value. */
kx_status kx_transport_ex(const kx_mech *mech, int64_t n, const double *T, const double *p,
                          const double *Y, double *mu, double *lambda, double *Dmix,
                          int32_t precision, hipStream_t stream);

/* Mixture thermodynamics (App. A.1) for n points: cp_k[Ns][n] = Cp_k/W_k,
 * h_k[Ns][n] = H_k/W_k and cp_mix[n] = sum_k Y_k cp_k.  Any of the three
 * outputs may be NULL.  Plain FP64. */
kx_status kx_thermo(const kx_mech *mech, int64_t n, const double *T, const double *Y,
                    double *cp_k, double *h_k, double *cp_mix, hipStream_t stream);

/* Analytical Jacobian of the production rates (App. A.2 differentiated; the
 * paper names it as the input of implicit BDF integrators, §1, §4):
 * jac[(i * Ns + k) * Ns + j] = d wdot_k / d C_j in 1/s at point i, at fixed
 * temperature T[i], the derivative taken at C_k = X_k p / (R_u T) with the
 * pressure following the concentrations (p = R_u T sum_k C_k, so [M] = sum C
 * and a pressure-table rate constant sees the change of p).  One dense
 * row-major Ns x Ns matrix per point, contiguous (the layout batched linear
 * solvers take); jac holds n * Ns * Ns doubles (device memory).  Plain FP64.
 * KX_EUNSUPPORTED for mechanisms of more than 128 species or with QSS
 * species.  Where an explicit
 * order below one meets an absent species the derivative is +inf. */
kx_status kx_jacobian(const kx_mech *mech, int64_t n, const double *T, const double *p,
                      const double *Y, double *jac, hipStream_t stream);

/* Concentrations of the QSS species (mol/cm^3) for n points: Cq[j][n] for the
 * j-th QSS species in species order.  At each point they solve the balances
 * wdot_q = 0 of the linearised QSSA (Lu & Law 2006; the paper plans QSS
 * species, §4): with the rates of progress affine in the QSS concentrations
 * (at most one QSS molecule per reaction side), the balances are a linear
 * system A C_Q = -b of order n_qss, assembled from the forward and reverse
 * terms of the reactions and solved by elimination.  The mixture is that of
 * the transported species; QSS entries of Y are not read.  A QSS species whose
 * every sink vanishes at a point (a zero consumption rate) makes the system
 * singular there and its concentration is then not finite.  Cq is device
 * memory of n_qss * n doubles.  KX_EINVAL if the mechanism has no QSS species.
 * Plain FP64. */
kx_status kx_qss_concentrations(const kx_mech *mech, int64_t n, const double *T,
                                const double *p, const double *Y, double *Cq,
                                hipStream_t stream);

/* ------------------------------------------------------------------------
 * Serving: a continuous-batching request server (project addition; the paper
 * notes that GPUs reach their throughput only with >~1e5 points, so small
 * requests are batched).  A server owns an HBM arena of `hbm_budget` bytes that
 * holds the tables of its resident mechanisms (kx_server_add_mech) and the
 * outputs of admitted requests; a scheduler thread admits queued requests in
 * arrival order whenever a slot and arena space are free, groups admitted
 * requests by (mechanism, precision) into batches of up to 64, and runs each
 * batch over a device work list on one of several streams -- batches of
 * different groups overlap on the device.  A batch of fewer than 2^17 points
 * replays a captured HIP graph of work-stealing kernels; a bigger one is
 * launched directly with one rates workgroup per tile.  Every request is cut
 * into the same tiles as a direct call, so its outputs are bit-identical alone
 * and in a batch.
 * ------------------------------------------------------------------------ */
typedef struct kx_server kx_server;
typedef int64_t kx_ticket;

enum { KX_OP_RATES = 1, KX_OP_TRANSPORT = 2 };          /* request ops (bit set) */
enum { KX_SERVER_SIMULATE = 1 };                         /* kx_server_create flags */
enum {                                                   /* kx_result.state */
    KX_REQ_QUEUED = 0, KX_REQ_ADMITTED = 1, KX_REQ_RUNNING = 2,
    KX_REQ_DONE = 3, KX_REQ_CANCELLED = 4, KX_REQ_FAILED = 5
};

typedef struct {
    const kx_mech *mech;      /* created on the server's device; must outlive the request */
    int32_t ops;              /* KX_OP_RATES, optionally | KX_OP_TRANSPORT */
    int32_t precision;        /* KX_FP64 or KX_MIXED */
    int64_t n;                /* points */
    const double *T, *p, *Y;  /* DEVICE inputs (layout as kx_production_rates); they
                                 must stay valid and unchanged until the request is
                                 DONE, CANCELLED or FAILED */
    double arrival_s;         /* arrival time on kx_server_clock() for latency
                                 accounting; < 0 means "now" */
    hipEvent_t inputs_ready;  /* NULL: the inputs are complete when kx_submit is
                                 called (the stream that wrote them synchronised).
                                 Otherwise an event recorded after the work that
                                 writes them: the server's streams wait for it
                                 before reading them.  It must stay valid until the
                                 request is DONE, CANCELLED or FAILED. */
} kx_request;

typedef struct {
    int32_t state;                      /* KX_REQ_* */
    int32_t pad;
    double *wdot, *mu, *lambda, *Dmix;  /* server-owned DEVICE outputs, valid from DONE
                                           until kx_release (NULL where not requested) */
    double t_arrival, t_admit, t_launch, t_done;  /* kx_server_clock() seconds */
} kx_result;

typedef struct {
    int64_t submitted, completed, cancelled, failed;
    int64_t queued, in_flight;          /* now */
    int64_t batches, graph_launches;   /* graph_launches: batches replayed from a graph */
    int64_t arena_in_use, arena_capacity;  /* bytes; in use includes resident tables */
    int64_t resident_mechs, resident_bytes;
} kx_server_stats;

/* Monotonic clock (seconds) used for all server time stamps. */
double kx_server_clock(void);

/* Create a server on `device` with an output arena of `hbm_budget` bytes and
 * at most `max_slots` requests admitted at once.  KX_SERVER_SIMULATE runs the
 * scheduler without a GPU (no memory, no kernels; a batch "completes" after
 * 5 ns per point), for testing admission and queueing logic on a host.
 * Allocates device memory, streams and pinned host buffers. */
kx_status kx_server_create(int device, int64_t hbm_budget, int32_t max_slots, int32_t flags,
                           kx_server **out);

/* Stop the scheduler: queued and admitted requests are cancelled, batches
 * already on the device are waited for, then every resource is freed.
 * Pointers from kx_result become invalid. */
kx_status kx_server_destroy(kx_server *srv);

/* Make `mech` resident on the server: its device tables (kx_mech_info's
 * device_bytes, rounded up to 256) are copied into the server's arena, where
 * they stay until kx_server_destroy and count against the HBM budget, and the
 * launch graphs of its batches (both precisions, both op sets, every stream)
 * are captured now rather than by its first requests.  Requests may name only
 * resident mechanisms.  Adding a mechanism twice is a no-op.  KX_ENOMEM if the
 * tables do not fit in the arena's free space; KX_EINVAL for a NULL argument
 * or a mechanism without tables on the server's device (a host-only handle is
 * accepted by a KX_SERVER_SIMULATE server, which charges its bytes without a
 * copy); KX_EUNSUPPORTED for a mechanism with QSS species.  Blocks until the
 * copy and the captures are done.  `mech` must outlive the server (it keys the
 * requests that name it). */
kx_status kx_server_add_mech(kx_server *srv, const kx_mech *mech);

/* Queue a request.  KX_EINVAL for a bad request or a mechanism that is not
 * resident (kx_server_add_mech); KX_ENOMEM if its output footprint
 * n * 8 * (Ns [wdot] + (Ns + 2) [transport]) exceeds the budget left after the
 * resident tables; KX_EUNSUPPORTED for a mechanism with QSS species (call
 * kx_production_rates for those).  n == 0 completes immediately. */
kx_status kx_submit(kx_server *srv, const kx_request *req, kx_ticket *ticket);

/* Current state and outputs of a request (non-blocking). */
kx_status kx_poll(kx_server *srv, kx_ticket ticket, kx_result *res);

/* Block until the request is DONE, CANCELLED or FAILED, or `timeout_s`
 * seconds pass (KX_EAGAIN; timeout_s < 0 waits forever). */
kx_status kx_wait(kx_server *srv, kx_ticket ticket, double timeout_s, kx_result *res);

/* Cancel a request that has not been launched (QUEUED or ADMITTED); KX_EAGAIN
 * if it is already running or finished. */
kx_status kx_cancel(kx_server *srv, kx_ticket ticket);

/* Enqueue copies of a DONE request's outputs into caller buffers (any may be
 * NULL) on `stream`; each buffer is device memory or pinned host memory
 * (hipHostMalloc), in which case the copy goes over the host link.  The copies
 * must have completed before the ticket is released (its arena space is reused
 * at once), and a ticket must not be copied and released from two threads at
 * the same time. */
kx_status kx_result_copy(kx_server *srv, kx_ticket ticket, double *wdot, double *mu,
                         double *lambda, double *Dmix, hipStream_t stream);

/* Forget a finished request and return its arena space; KX_EAGAIN if it is
 * still queued or running.  A DONE request keeps its outputs (and arena
 * space) until released, so a client that holds finished requests while it
 * waits for queued ones can stall admission once the arena is full. */
kx_status kx_release(kx_server *srv, kx_ticket ticket);

kx_status kx_server_stats_get(kx_server *srv, kx_server_stats *stats);

/* ------------------------------------------------------------------------
 * Batched evaluation without allocation.  For callers that cannot allocate
 * device or pinned memory while they run: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  It runs the request
 * server's batch kernels for big batches (one workgroup per tile, the same
 * tiles, so every item's outputs are bit-identical to kx_production_rates /
 * kx_transport and to a served request on the same inputs) over up to
 * KX_BATCH_MAX_ITEMS point sets of one mechanism, without a server: the work
 * list lives in a fixed device array of the library (about 5 KB per device,
 * held until the process ends), written by a setup kernel on `stream` (no
 * memset, no host-to-device copy).  Calls that overlap on one device race for that
 * array: issue them on one stream, or order them.
 * ------------------------------------------------------------------------ */
#define KX_BATCH_MAX_ITEMS 32

typedef struct {
    int64_t n;                        /* points of this item (0: skipped) */
    const double *T, *p, *Y;          /* DEVICE inputs, layout as kx_production_rates */
    double *wdot;                     /* DEVICE output [Ns][n] */
    double *mu, *lambda, *Dmix;       /* DEVICE outputs [n], [n], [Ns][n]; read only with
                                         KX_OP_TRANSPORT */
} kx_batch_item;

/* Evaluate `ops` (KX_OP_RATES, optionally | KX_OP_TRANSPORT) in `precision` for
 * `nitems` items of `mech`, enqueued on `stream`.  Allocates nothing: no
 * hipMalloc, hipFree or allocating library routine is called.  KX_EINVAL for
 * nitems outside 0..KX_BATCH_MAX_ITEMS, an item with n < 0 or a NULL array it
 * needs, bad ops or precision, or more than 2^31 - 1 tiles in one call;
 * KX_EUNSUPPORTED for a mechanism with QSS species. */
kx_status kx_batch_noalloc(const kx_mech *mech, int32_t ops, int32_t precision, int32_t nitems,
                           const kx_batch_item *items, hipStream_t stream);

/* Human-readable description of the calling thread's most recent failure
 * ("" if none).  The pointer stays valid until the thread's next kx_* call. */
const char *kx_last_error(void);

/* Library version string, e.g. "kx 0.1 gfx950". */
const char *kx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KX_H */
