// kx_batch.hip -- production rates (and transport) of several point sets of
// one mechanism in one launch sequence, with no allocation.
//
// The batch kernels the request server runs for big batches (one workgroup
// per tile) take their work list from device memory.  Here that memory is a
// file-scope device array, `scratch`, of fixed size: a setup kernel writes the
// work list (from its by-value argument), then the rates kernel and, if asked
// for, the transport kernel run over it with grids of the host's tile counts.
// No device or pinned memory is allocated and no host-to-device copy is made,
// so the call can be captured into a HIP graph or issued from a loop that must
// not allocate.
// Every call on a device uses that device's one copy of the array.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "kx_internal.h"

namespace kx {
namespace {

// The work list, 256-byte aligned.
constexpr size_t kScratchBytes = (sizeof(WorkList) + 255) & ~size_t(255);

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, taken once per device.
constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// The kernel argument: the items of one call (the work list's items without
// the tile bookkeeping, which the setup kernel derives).
struct BatchArgs {
    int32_t nitems;
    int32_t rates_tp, transport_tp;  // points per tile of the two kernels
    int32_t transport;               // the transport kernel runs
    WorkItem items[KX_BATCH_MAX_ITEMS];
};

// Writes the work list (tile ranges of every item, in item order, as the
// server cuts them).  One thread.
__global__ void batch_setup_kernel(BatchArgs a, WorkList *wl)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    wl->nitems = a.nitems;
    int tr = 0, tt = 0;
    for (int r = 0; r < a.nitems; ++r) {
        wl->items[r] = a.items[r];
        wl->start[0][r] = tr;
        wl->start[1][r] = tt;
        tr += (int)((a.items[r].n + a.rates_tp - 1) / a.rates_tp);
        if (a.transport) tt += (int)((a.items[r].n + a.transport_tp - 1) / a.transport_tp);
    }
    wl->start[0][a.nitems] = wl->ntiles[0] = tr;
    wl->start[1][a.nitems] = wl->ntiles[1] = tt;
}

kx_status scratch_address(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(KX_EINVAL, "kx_batch_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "kx_batch_noalloc: hipGetSymbolAddress");
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return KX_OK;
}

}  // namespace
}  // namespace kx

using namespace kx;

extern "C" kx_status kx_batch_noalloc(const kx_mech *mech, int32_t ops, int32_t precision,
                                      int32_t nitems, const kx_batch_item *items,
                                      hipStream_t stream)
{
    if (!mech) return fail(KX_EINVAL, "kx_batch_noalloc: mech is NULL");
    if (!mech->blob) return fail(KX_EINVAL, "kx_batch_noalloc: mechanism has no device tables");
    if (mech->dev.nq > 0)
        return fail(KX_EUNSUPPORTED, "kx_batch_noalloc: mechanisms with QSS species are not "
                                     "supported (call kx_production_rates)");
    if (!(ops & KX_OP_RATES) || (ops & ~(KX_OP_RATES | KX_OP_TRANSPORT)))
        return fail(KX_EINVAL, "kx_batch_noalloc: ops must be KX_OP_RATES [| KX_OP_TRANSPORT]");
    if (precision != KX_FP64 && precision != KX_MIXED)
        return fail(KX_EINVAL, "kx_batch_noalloc: unknown precision");
    if (nitems < 0 || nitems > KX_BATCH_MAX_ITEMS)
        return fail(KX_EINVAL, "kx_batch_noalloc: nitems must be 0.." +
                                   std::to_string(KX_BATCH_MAX_ITEMS));
    if (nitems > 0 && !items) return fail(KX_EINVAL, "kx_batch_noalloc: items is NULL");
    const bool tr = (ops & KX_OP_TRANSPORT) != 0;
    const int rtp = rates_tile_points(mech->dev);
    const int ttp = transport_tile_points(mech->dev, precision);
    BatchArgs a;
    std::memset(&a, 0, sizeof a);
    int64_t tiles_r = 0, tiles_t = 0;
    for (int r = 0; r < nitems; ++r) {
        const kx_batch_item &it = items[r];
        if (it.n < 0) return fail(KX_EINVAL, "kx_batch_noalloc: an item has n < 0");
        if (it.n > 0 && (!it.T || !it.p || !it.Y || !it.wdot))
            return fail(KX_EINVAL, "kx_batch_noalloc: NULL input or wdot array");
        if (it.n > 0 && tr && (!it.mu || !it.lambda || !it.Dmix))
            return fail(KX_EINVAL, "kx_batch_noalloc: NULL transport output array");
        tiles_r += (it.n + rtp - 1) / rtp;
        tiles_t += tr ? (it.n + ttp - 1) / ttp : 0;
        WorkItem &w = a.items[a.nitems++];
        w.T = it.T;
        w.p = it.p;
        w.Y = it.Y;
        w.wdot = it.wdot;
        w.mu = tr ? it.mu : nullptr;
        w.lam = tr ? it.lambda : nullptr;
        w.Dmix = tr ? it.Dmix : nullptr;
        w.n = it.n;
    }
    if (tiles_r > 0x7fffffff || tiles_t > 0x7fffffff)
        return fail(KX_EINVAL, "kx_batch_noalloc: too many points in one call");
    if (tiles_r == 0) return ok();
    a.rates_tp = rtp;
    a.transport_tp = ttp;
    a.transport = tr;

    // the mechanism's device is current for the calls below (the scratch address
    // is that device's), the caller's device again on return
    struct Guard {
        int prev = -1;
        hipError_t err = hipSuccess;
        explicit Guard(int dev)
        {
            err = hipGetDevice(&prev);
            if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
        }
        ~Guard()
        {
            int cur = -1;
            if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
                (void)hipSetDevice(prev);
        }
    } g(mech->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "kx_batch_noalloc: hipSetDevice");
    void *base = nullptr;
    kx_status st = scratch_address(mech->device, &base);
    if (st != KX_OK) return st;
    WorkList *wl = static_cast<WorkList *>(base);
    hipLaunchKernelGGL(batch_setup_kernel, dim3(1), dim3(64), 0, stream, a, wl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kx_batch_noalloc: setup kernel launch");
    st = launch_rates_items(mech->dev, wl, tiles_r, precision, stream);
    if (st == KX_OK && tr) st = launch_transport_items(mech->dev, wl, tiles_t, precision, stream);
    if (st != KX_OK) return st;
    return ok();
}
