// kx_micro.hip -- throughput of the elementary functions the kernels use, on
// gfx950, in units of the FP64 fused multiply-add.
//
// gfx950 has no FP64 exponential, logarithm, division or square root
// instruction, so the price of each in a roofline must be measured on the
// library's own sequences (kx_math.h).  Each probe kernel runs a loop in which
// every lane advances eight independent values through one operation (enough
// independent work that the VALU, not latency, sets the rate), on a grid that
// fills every SIMD.  A loop that applies only the bookkeeping add is timed
// too, and the price of an operation is
//     2 * (t_op - t_add) / t_fma               flops,
// i.e. the issue time of the operation in FP64 FMAs (2 flops each); an FP64
// add issues like an FMA, so the add probe removes the bookkeeping and the FMA
// probe (one FMA per step) is the unit.
//
// The matrix-core probes (ops 10..13) issue one MFMA per step into each of
// eight independent accumulators per wave, on the same grid; they measure the
// rate each instruction sustains on this GPU, against which the transport
// kernel's matrix-core throughput is read.
//
// This file is a measuring tool: it is built into its own library, which the
// benchmark loads; the chemistry library does not contain it.
#include <hip/hip_runtime.h>

#include "kx_math.h"

namespace {

using namespace kx;

constexpr int kValues = 8;

enum Op {
    kOpAdd = 0,      // v = v - 2 (bookkeeping only)
    kOpFma = 1,      // v = v * c + d
    kOpExp = 2,      // v = kexp(v) - 2
    kOpLog = 3,      // v = kln(v) + 2
    kOpRcp = 4,      // v = krcp(v) + 1/2 (reciprocal, two Newton steps)
    kOpRsqrt = 5,    // v = krsqrt(v) + 1/2
    kOpExpMixed = 6, // v = e^v - 2 with the FP64 argument reduced and e^r in FP32
    kOpExp32 = 7,    // FP32: v = __expf(v) - 2
    kOpRcp32 = 8,    // FP32: v = 1 / v + 1/2 (correctly rounded division)
    kOpFma32 = 9,    // FP32: v = v * c + d (also the bookkeeping of the FP32 probes)
    kOpMfma64x16 = 10,  // v_mfma_f64_16x16x4_f64 (2048 flops)
    kOpMfma64x4 = 11,   // v_mfma_f64_4x4x4_4b_f64 (512 flops)
    kOpMfma32x16 = 12,  // v_mfma_f32_16x16x4_f32 (2048 flops)
    kOpMfma32x32 = 13,  // v_mfma_f32_32x32x2_f32 (4096 flops)
};

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Eight accumulators per wave, each advanced by one MFMA per step.
template <int OP>
__device__ __forceinline__ double mfma_probe(int iters, double seed)
{
    const double a = seed + threadIdx.x * 1e-3, b = seed - threadIdx.x * 1e-3;
    const float af = (float)a, bf = (float)b;
    double r = 0.0;
    if (OP == kOpMfma64x16) {
        v4d c[8];
        for (int q = 0; q < 8; ++q) c[q] = v4d{seed, 0.0, 0.0, 0.0};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[q], 0, 0, 0);
        }
        for (int q = 0; q < 8; ++q) r += c[q][q & 3];
    } else if (OP == kOpMfma64x4) {
        double c[8];
        for (int q = 0; q < 8; ++q) c[q] = seed;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c[q], 0, 0, 0);
        }
        for (int q = 0; q < 8; ++q) r += c[q];
    } else if (OP == kOpMfma32x16) {
        v4f c[8];
        for (int q = 0; q < 8; ++q) c[q] = v4f{(float)seed, 0.0f, 0.0f, 0.0f};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf, c[q], 0, 0, 0);
        }
        for (int q = 0; q < 8; ++q) r += c[q][q & 3];
    } else {
        v16f c[8];
        for (int q = 0; q < 8; ++q) {
            c[q] = v16f{};
            c[q][0] = (float)seed;
        }
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(af, bf, c[q], 0, 0, 0);
        }
        for (int q = 0; q < 8; ++q) r += c[q][q];
    }
    return r;
}

__device__ __forceinline__ double exp_mixed_probe(double x)
{
    const double nd = rint(x * 1.4426950408889634);
    const double r = fma(-nd, 6.93147180559945286e-01, x);
    const float er = __expf((float)r);
    return ldexp((double)er, (int)nd);
}

template <int OP>
__global__ __launch_bounds__(256) void probe_kernel(int iters, double seed, double *out)
{
    if (OP >= kOpMfma64x16) {
        out[blockIdx.x * blockDim.x + threadIdx.x] = mfma_probe<OP>(iters, seed);
        return;
    }
    if (OP >= kOpExp32) {
        float v[kValues];
#pragma unroll
        for (int j = 0; j < kValues; ++j) v[j] = (float)seed + 0.01f * (float)(threadIdx.x % 7 + j);
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int j = 0; j < kValues; ++j) {
                if (OP == kOpExp32) v[j] = __expf(v[j]) - 2.0f;
                if (OP == kOpRcp32) v[j] = 1.0f / v[j] + 0.5f;
                if (OP == kOpFma32) v[j] = fmaf(v[j], 0.999f, 0.001f);
            }
        }
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < kValues; ++j) s += v[j];
        out[blockIdx.x * blockDim.x + threadIdx.x] = (double)s;
        return;
    }
    double v[kValues];
#pragma unroll
    for (int j = 0; j < kValues; ++j) v[j] = seed + 0.01 * (double)(threadIdx.x % 7 + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kValues; ++j) {
            if (OP == kOpAdd) v[j] = v[j] - 2.0;
            if (OP == kOpFma) v[j] = fma(v[j], 0.999, 0.001);
            if (OP == kOpExp) v[j] = kexp(v[j]) - 2.0;
            if (OP == kOpLog) v[j] = kln(v[j]) + 2.0;
            if (OP == kOpRcp) v[j] = krcp(v[j]) + 0.5;
            if (OP == kOpRsqrt) v[j] = krsqrt(v[j]) + 0.5;
            if (OP == kOpExpMixed) v[j] = exp_mixed_probe(v[j]) - 2.0;
        }
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kValues; ++j) s += v[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Start values inside each operation's stable range (the iteration maps stay
// bounded and away from special values).
double seed_of(int op)
{
    switch (op) {
        case kOpExp: case kOpExpMixed: case kOpExp32: return -1.8;
        case kOpLog: return 3.1;
        case kOpRcp: case kOpRcp32: return 1.3;
        case kOpRsqrt: return 1.2;
        case kOpAdd: return 1e9;
        default: return 0.5;
    }
}

}  // namespace

extern "C" {

// Time `reps` launches of the probe for operation `op` (0..13, see Op) with
// `iters` loop trips on a grid of `blocks` workgroups of 256 threads; `out`
// is device scratch of blocks * 256 doubles.  Writes the mean milliseconds per
// launch to *ms.  Returns 0, or -1 for a bad argument, -3 for a HIP error.
int kx_micro_time(int op, int iters, int blocks, int reps, double *out, double *ms)
{
    if (op < 0 || op > 13 || iters <= 0 || blocks <= 0 || reps <= 0 || !out || !ms) return -1;
    void (*k)(int, double, double *) = nullptr;
    switch (op) {
        case 0: k = probe_kernel<0>; break;
        case 1: k = probe_kernel<1>; break;
        case 2: k = probe_kernel<2>; break;
        case 3: k = probe_kernel<3>; break;
        case 4: k = probe_kernel<4>; break;
        case 5: k = probe_kernel<5>; break;
        case 6: k = probe_kernel<6>; break;
        case 7: k = probe_kernel<7>; break;
        case 8: k = probe_kernel<8>; break;
        case 9: k = probe_kernel<9>; break;
        case 10: k = probe_kernel<10>; break;
        case 11: k = probe_kernel<11>; break;
        case 12: k = probe_kernel<12>; break;
        default: k = probe_kernel<13>; break;
    }
    const double seed = seed_of(op);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -3;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return -3;
    }
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, 0, iters, seed, out);  // warm-up
    hipEventRecord(e0, 0);
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, 0, iters, seed, out);
    hipEventRecord(e1, 0);
    hipError_t e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess) e = hipGetLastError();
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return -3;
    *ms = (double)t / reps;
    return 0;
}

}  // extern "C"
