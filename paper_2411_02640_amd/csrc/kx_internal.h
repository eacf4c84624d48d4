// kx_internal.h -- device-resident mechanism tables and launch helpers shared
// by the host table builder (kx_mech.cpp) and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/kx.h"

namespace kx {

// Physical constants (cgs; CODATA 2018 exact R, thermochemical calorie).
constexpr double kRu = 8.31446261815324e7;            // erg / (mol K)
constexpr double kRcal = 8.31446261815324 / 4.184;    // cal / (mol K)
constexpr double kPatm = 1013250.0;                   // dyn / cm^2

constexpr int kMaxSide = 3;          // molecules per reaction side (sum of nu)
constexpr int kMaxSpecies = 256;     // species per mechanism (4 per lane)
constexpr int kMaxFitOrder = 8;
constexpr int kWave = 64;
constexpr int kMaxQss = 64;          // QSS species per mechanism (one wave of rows)
constexpr int kChunkMax = 192;       // reactions per chunk of the gather lists, at most

// Reaction flags.
enum : uint8_t {
    kFlagReversible = 1,
    kFlagKfConst = 2,    // beta = E_R = 0: k_f = A without an exponential
    kFlagChemAct = 4,    // chemically activated falloff: c = F / (1 + P_r) with k_0 in r_i
    kFlagOrders = 8,     // explicit forward orders (irreversible): prod C^o from DevAux
};

// One reaction slot in kernel order.  Reactions are sorted heaviest type
// first (Troe, Lindemann, three-body, elementary, constant-k_f elementary) so
// that the expensive falloff code runs in as few 64-lane iterations as
// possible.  Each side lists one LDS byte offset per molecule (a species
// with nu = 2 appears twice); unused entries point at a dummy species whose
// per-point factors are 1.  48 bytes.
struct alignas(16) DevRxn {
    double lnA;              // ln A
    double beta;             // temperature exponent
    double ER;               // activation temperature E_a / R
    double A;                // A itself (k_f when kFlagKfConst)
    uint16_t roff[kMaxSide]; // reactant molecules: 16 * species
    uint16_t poff[kMaxSide]; // product molecules
    uint8_t type;            // KX_RXN_*
    uint8_t flags;
    uint16_t aux;            // index into DevAux for types 1..3
};
static_assert(sizeof(DevRxn) == 48, "DevRxn layout");

// Third-body, falloff and pressure-table data of one reaction.  Up to
// kInlineEff explicit efficiencies are stored inline (LDS byte offset of the
// species and alpha - default; unused entries point at the dummy species with
// 0); any further ones are in DevEff[ext_off .. ext_off + ext_cnt).  A PLOG
// reaction's reference pressures are DevPlog[plog_off .. plog_off + plog_cnt).
// 224 bytes.
constexpr int kInlineEff = 8;
constexpr int kMaxOrd = 4;            // species with explicit orders per reaction
struct alignas(16) DevAux {
    double eff_default;      // efficiency of unlisted species
    double lnA0, beta0, ER0; // k_0 (falloff)
    // Falloff blend parameters (eq:blend):
    //   Troe: alpha, 1/T***, 1/T*, T** (used when has_T2), 0
    //   SRI:  a, b, 1/c, ln d, e
    double fp[5];
    double dalpha[kInlineEff];
    uint16_t eoff[kInlineEff];
    int32_t has_T2, ext_off, ext_cnt;
    int32_t plog_off, plog_cnt, pad;
    // explicit forward orders: LDS byte offset of the species pair and the
    // order (unused entries have order 0)
    double oval[kMaxOrd];
    uint16_t ooff[kMaxOrd];
};
static_assert(sizeof(DevAux) == 224, "DevAux layout");

// One reference pressure of a PLOG reaction: ln p_j, the Arrhenius exponent
// ln k_j = lnA + beta ln T - ER / T, and 1 / (ln p_(j+1) - ln p_j) (0 for the
// last).  48 bytes.
struct alignas(16) DevPlog {
    double lnp, lnA, beta, ER, inv_dlnp, pad;
};

struct alignas(16) DevEff {
    double dalpha;           // alpha_ki - eff_default
    int32_t sp;
    int32_t pad;
};

// Per-species thermo: Gibbs coefficients g/RT = c0 (1 - ln T) + c1 T + c2 T^2 +
// c3 T^3 + c4 T^4 + c5 / T + c6 for both ranges (eq:Ck pre-scaled), the raw
// NASA coefficients for cp and h, T_mid and 1/W.  Each species: 32 doubles.
struct alignas(16) DevSpecies {
    double g_lo[8];   // c0..c6 + pad
    double g_hi[8];
    double nasa_lo[7];
    double t_mid;
    double nasa_hi[7];
    double inv_W;
};
static_assert(sizeof(DevSpecies) == 256, "DevSpecies layout");

// Transport tables are blocked by kKB species k so that the coefficients of
// one (k-block, j) step are contiguous for scalar loads.
constexpr int kKB = 8;

struct MechDev {
    int32_t ns, nr, nchunks;   // species, reactions, reaction chunks for the gather
    int32_t chunk;             // reactions per chunk (multiple of 64)
    int32_t gpass;             // species per lane in the species phases (1, 2 or 4)
    int32_t fit_order, diff_kind;
    double fit_L0, inv_fit_h;
    const DevRxn *rxn;         // [nr] kernel order
    const DevAux *aux;         // [naux]
    const DevEff *eff;         // [neff]
    const DevPlog *plog;       // [nplog]
    const DevSpecies *sp;      // [ns]
    const double *gsoa;        // [ceil(ns/64)][16][64] the rates kernel's species data by
                               // field in blocks of 64 species, so that the lanes of a
                               // wave read one contiguous 512-byte row: field 0..6 g_lo,
                               // 7..13 g_hi, 14 T_mid, 15 1/W of species 64 blk + lane
    const int32_t *gpos;       // [nchunks] groups of eight +q entries of the gather
    const int32_t *gneg;       // [nchunks] groups of eight -q entries
    const int32_t *goff;       // [nchunks] first group of each chunk
    const uint4 *gent;         // [group][64 * gpass][2]: eight 32-bit LDS byte offsets
                               // 16 * slot_in_chunk per lane and group (a species with
                               // |nu''-nu'| = 2 or 3 lists the slot that many times);
                               // padding entries read the zero slot after the chunk
    const int32_t *gmgrp;      // [nchunks] the rates kernel's lists: groups per chunk
    const int32_t *gmoff;      // [nchunks] first group of each chunk
    const uint4 *gment;        // [group][64 * gpass][2]: as gent, one list per species
                               // with the +q and -q entries together, the sign of an
                               // entry in bit 31 (set: -q) above its LDS byte offset
    // transport (FP64)
    const double *W;           // [ns]
    const double *visc;        // [ns][order]
    const double *cond;        // [ns][order]
    const double *wq;          // [ns] W_k^(1/4)
    const double *wilke;       // [nkb][ns][kKB] c1_kj = (8 (1 + W_k/W_j))^(-1/2)
    const double *dfit;        // [nkb][ns][kKB][order]  fit of (k = kb*KB+kk, j)
    const double *ddiag;       // [ns][order] diagonal fits for the fallback
    // transport (FP32 copies for the mixed path)
    const float *visc32, *cond32, *wq32, *wilke32, *dfit32, *ddiag32;
    // Matrix-core form of the quadratic transport sums (tables holding fits of
    // 1/D_kj only; null otherwise).  mblk = ceil(ns / 16) row blocks of 16
    // species k, kstep = ceil(ns / 4) steps of 4 species j.  Fragments are
    // stored in the lane order of a 16x16x4 MFMA A operand: lane l holds row
    // k = 16 mb + l % 16, column j = 4 ks + l / 16, so each is one coalesced
    // 64-element load.
    //   gfrag  [fit_order][mblk][kstep][64]: d_kjn, the n-th coefficient of the
    //          fit of 1/D_kj (zero on the diagonal j = k and in the padding)
    //   c1frag [mblk][kstep][64]: Wilke c1_kj (zero in the padding)
    int32_t mblk, kstep;
    const double *gfrag, *c1frag;
    const float *gfrag32, *c1frag32;
    // Quasi-steady-state species (nq = 0 when there are none).  QSS index j
    // numbers them in species order.
    int32_t nq, nqent;         // QSS species, entries of their balance rows
    const int32_t *qidx;       // [ns] QSS index of species k, -1 if transported
    const int32_t *qrow_ptr;   // [nq + 1] entries of the balance of QSS species j
    const int4 *qrow_ent;      // {LDS slot of the reaction (kernel order s, at s + s /
                               //  chunk), net nu of j, QSS index among the reaction's
                               //  reactants, among its products}
    const int2 *qrx;           // [nr] kernel order: QSS index among the reactants,
                               // among the products (-1: none)
};

// Work list of one batch of served requests (device memory, written by the
// host before the batch launches).  start[op][r] is the first tile of item r
// for op 0 (rates) and op 1 (transport); start[op][nitems] = ntiles[op].
constexpr int kMaxBatch = 64;
struct WorkItem {
    const double *T, *p, *Y;
    double *wdot, *mu, *lam, *Dmix;
    int64_t n;
};
struct WorkList {
    int32_t nitems;
    int32_t ntiles[2];
    int32_t pad;
    int32_t start[2][kMaxBatch + 1];
    WorkItem items[kMaxBatch];
};

// The item that holds tile t of op: the last item whose first tile is <= t.
// A batch kernel takes its tiles in increasing order (within an XCD range), so
// the search starts from the previous tile's item r -- amortised O(1) instead of
// a walk over the items per tile (each step a dependent scalar load) -- and
// restarts from item 0 when t lies before item r.
__device__ __forceinline__ int work_item_of(const WorkList *wl, int op, int t, int r)
{
    if (wl->start[op][r] > t) r = 0;
    while (r + 1 < wl->nitems && wl->start[op][r + 1] <= t) ++r;
    return r;
}

// The same in one step for a kernel that runs one tile per workgroup: lane l
// of each wave reads the first tile of item l + 1 and the wave counts the
// items after the first whose first tile is <= t (a work list holds at most
// kMaxBatch = 64 items).  Wave-uniform result.
__device__ __forceinline__ int work_item_ballot(const WorkList *wl, int op, int t)
{
    const int l = (int)(threadIdx.x & 63);
    const bool below = l + 1 < wl->nitems && wl->start[op][l + 1] <= t;
    return __builtin_amdgcn_readfirstlane(__popcll(__builtin_amdgcn_ballot_w64(below)));
}
static_assert(kMaxBatch <= 64, "work_item_ballot covers the items with one wave");

}  // namespace kx

struct kx_mech {
    int device;
    kx::MechDev dev;
    void *blob;          // single device allocation holding every table
    int64_t bytes;
    int32_t n_species, n_reactions;
    uint64_t uid;        // never reused within a process (keys cached launch graphs)
};

namespace kx {
// Error reporting shared by all entry points (thread-local message).
kx_status fail(kx_status code, const std::string &msg);
kx_status ok();
kx_status hip_fail(hipError_t e, const char *what);

// Launchers (defined in the kernel translation units).
kx_status launch_rates(const kx_mech *m, int64_t n, const double *T, const double *p,
                       const double *Y, double *wdot, int precision, hipStream_t s);
kx_status launch_transport(const kx_mech *m, int64_t n, const double *T, const double *p,
                           const double *Y, double *mu, double *lam, double *Dmix,
                           int precision, hipStream_t s);
kx_status launch_thermo(const kx_mech *m, int64_t n, const double *T, const double *Y,
                        double *cpk, double *hk, double *cpmix, hipStream_t s);
kx_status launch_jacobian(const kx_mech *m, int64_t n, const double *T, const double *p,
                          const double *Y, double *jac, hipStream_t s);
// Rates of a mechanism with QSS species; either output may be null.
kx_status launch_qss(const kx_mech *m, int64_t n, const double *T, const double *p,
                     const double *Y, double *wdot, double *Cq, hipStream_t s);

// Points per tile of the two kernels for a mechanism and precision (the
// serving work lists are cut in the same tiles as a direct call, so a request
// gives bit-identical results alone and in a batch).
int rates_tile_points(const MechDev &m);
int transport_tile_points(const MechDev &m, int precision);
// Batched (work-list) launches; `counter` must be zero at launch.
// prepare_rates_batch sets the kernel's dynamic-LDS limit (call it before
// capturing a launch into a graph).
kx_status prepare_rates_batch(const MechDev &m, int precision);
// One workgroup per tile of the work list (`ntiles` = wl->ntiles[0] for rates,
// wl->ntiles[1] for transport, known to the host that wrote the list); no
// counters.
kx_status launch_rates_items(const MechDev &m, const WorkList *wl, int64_t ntiles, int precision,
                             hipStream_t s);
kx_status launch_transport_items(const MechDev &m, const WorkList *wl, int64_t ntiles,
                                 int precision, hipStream_t s);
kx_status launch_rates_batch(const MechDev &m, const WorkList *wl, int *counter, int precision,
                             int grid, hipStream_t s);
kx_status launch_transport_batch(const MechDev &m, const WorkList *wl, int *counter,
                                 int precision, int grid, hipStream_t s);
// Sets the transport batch kernel's dynamic-LDS limit (before graph capture).
kx_status prepare_transport_batch(const MechDev &m, int precision);
kx_status launch_zero(int *p, int count, hipStream_t s);
// Persistent grids of the batch kernels: one-wave workgroups of the rates batch
// kernel (16 per CU, at least as many as fit) and 256-lane workgroups of the
// transport batch kernel.
constexpr int kRatesBatchGrid = 4096;
constexpr int kTransportBatchGrid = 1024;
// Counters a batch uses: one per XCD for the rates tiles, one for transport.
constexpr int kXcds = 8;
constexpr int kBatchCounters = kXcds + 1;
// The device tables of `m` as they read from a byte-identical copy placed at
// `base`: every table pointer moved from m->blob to base.  False if some
// pointer still addresses the original tables (a field this function misses).
bool rebase_tables(const kx_mech *m, const void *base, MechDev *out);
}  // namespace kx
