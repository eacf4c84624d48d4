// kx_api.cpp -- the C ABI entry points: argument checks, device selection,
// error reporting, and dispatch to the kernel launchers.
#include <hip/hip_runtime.h>

#include <string>

#include "kx_internal.h"

namespace kx {

static thread_local std::string t_last_error;

kx_status fail(kx_status code, const std::string &msg)
{
    t_last_error = msg;
    return code;
}

kx_status ok()
{
    t_last_error.clear();
    return KX_OK;
}

kx_status hip_fail(hipError_t e, const char *what)
{
    return fail(KX_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

kx_status build_mech(const kx_mech_desc *d, int device, bool host_only, kx_mech **out);

namespace {

// Makes the handle's device current for the duration of a launch.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

kx_status check_common(const kx_mech *m, int64_t n, const char *who)
{
    if (!m) return fail(KX_EINVAL, std::string(who) + ": mech is NULL");
    if (!m->blob) return fail(KX_EINVAL, std::string(who) + ": mechanism has no device tables");
    if (n < 0) return fail(KX_EINVAL, std::string(who) + ": n < 0");
    return KX_OK;
}

}  // namespace
}  // namespace kx

using namespace kx;

extern "C" {

kx_status kx_mech_create(const kx_mech_desc *desc, int device, kx_mech **out)
{
    return build_mech(desc, device, false, out);
}

kx_status kx_mech_create_host(const kx_mech_desc *desc, kx_mech **out)
{
    return build_mech(desc, -1, true, out);
}

kx_status kx_mech_destroy(kx_mech *mech)
{
    if (!mech) return ok();
    if (!mech->blob) {
        delete mech;
        return ok();
    }
    DeviceGuard g(mech->device);
    hipError_t e = hipFree(mech->blob);
    delete mech;
    if (e != hipSuccess) return hip_fail(e, "hipFree (mechanism)");
    return ok();
}

kx_status kx_mech_info(const kx_mech *mech, int32_t *n_species, int32_t *n_reactions,
                       int64_t *device_bytes)
{
    if (!mech) return fail(KX_EINVAL, "kx_mech_info: mech is NULL");
    if (n_species) *n_species = mech->n_species;
    if (n_reactions) *n_reactions = mech->n_reactions;
    if (device_bytes) *device_bytes = mech->bytes;
    return ok();
}

kx_status kx_production_rates_ex(const kx_mech *mech, int64_t n, const double *T,
                                 const double *p, const double *Y, double *wdot,
                                 int32_t precision, hipStream_t stream)
{
    kx_status st = check_common(mech, n, "kx_production_rates");
    if (st != KX_OK) return st;
    if (precision != KX_FP64 && precision != KX_MIXED)
        return fail(KX_EINVAL, "kx_production_rates: unknown precision");
    if (mech->dev.nq > 0 && precision != KX_FP64)
        return fail(KX_EUNSUPPORTED, "kx_production_rates: mechanisms with QSS species are "
                                     "evaluated in FP64 only");
    if (n == 0) return ok();
    if (!T || !p || !Y || !wdot) return fail(KX_EINVAL, "kx_production_rates: NULL array");
    DeviceGuard g(mech->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    if (mech->dev.nq > 0) return launch_qss(mech, n, T, p, Y, wdot, nullptr, stream);
    return launch_rates(mech, n, T, p, Y, wdot, precision, stream);
}

kx_status kx_production_rates(const kx_mech *mech, int64_t n, const double *T,
                              const double *p, const double *Y, double *wdot,
                              hipStream_t stream)
{
    return kx_production_rates_ex(mech, n, T, p, Y, wdot, KX_FP64, stream);
}

kx_status kx_transport_ex(const kx_mech *mech, int64_t n, const double *T, const double *p,
                          const double *Y, double *mu, double *lambda, double *Dmix,
                          int32_t precision, hipStream_t stream)
{
    kx_status st = check_common(mech, n, "kx_transport");
    if (st != KX_OK) return st;
    const int32_t prec = precision & ~KX_DKJ_SYMMETRIC;
    if (prec != KX_FP64 && prec != KX_MIXED)
        return fail(KX_EINVAL, "kx_transport: unknown precision");
    if (n == 0) return ok();
    if (!T || !p || !Y || !mu || !lambda || !Dmix)
        return fail(KX_EINVAL, "kx_transport: NULL array");
    DeviceGuard g(mech->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return launch_transport(mech, n, T, p, Y, mu, lambda, Dmix, precision, stream);
}

kx_status kx_transport(const kx_mech *mech, int64_t n, const double *T, const double *p,
                       const double *Y, double *mu, double *lambda, double *Dmix,
                       hipStream_t stream)
{
    return kx_transport_ex(mech, n, T, p, Y, mu, lambda, Dmix, KX_FP64, stream);
}

kx_status kx_thermo(const kx_mech *mech, int64_t n, const double *T, const double *Y,
                    double *cp_k, double *h_k, double *cp_mix, hipStream_t stream)
{
    kx_status st = check_common(mech, n, "kx_thermo");
    if (st != KX_OK) return st;
    if (n == 0) return ok();
    if (!T || !Y) return fail(KX_EINVAL, "kx_thermo: NULL input array");
    if (!cp_k && !h_k && !cp_mix) return ok();
    DeviceGuard g(mech->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return launch_thermo(mech, n, T, Y, cp_k, h_k, cp_mix, stream);
}

kx_status kx_jacobian(const kx_mech *mech, int64_t n, const double *T, const double *p,
                      const double *Y, double *jac, hipStream_t stream)
{
    kx_status st = check_common(mech, n, "kx_jacobian");
    if (st != KX_OK) return st;
    if (mech->dev.nq > 0)
        return fail(KX_EUNSUPPORTED, "kx_jacobian: mechanisms with QSS species are not supported");
    if (n == 0) return ok();
    if (!T || !p || !Y || !jac) return fail(KX_EINVAL, "kx_jacobian: NULL array");
    DeviceGuard g(mech->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return launch_jacobian(mech, n, T, p, Y, jac, stream);
}

kx_status kx_qss_concentrations(const kx_mech *mech, int64_t n, const double *T,
                                const double *p, const double *Y, double *Cq,
                                hipStream_t stream)
{
    kx_status st = check_common(mech, n, "kx_qss_concentrations");
    if (st != KX_OK) return st;
    if (mech->dev.nq == 0)
        return fail(KX_EINVAL, "kx_qss_concentrations: the mechanism has no QSS species");
    if (n == 0) return ok();
    if (!T || !p || !Y || !Cq) return fail(KX_EINVAL, "kx_qss_concentrations: NULL array");
    DeviceGuard g(mech->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    return launch_qss(mech, n, T, p, Y, nullptr, Cq, stream);
}

const char *kx_last_error(void) { return t_last_error.c_str(); }

const char *kx_version(void) { return "kx 0.1 gfx950"; }

}  // extern "C"
