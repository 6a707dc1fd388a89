// Measured FP64 issue rates of the device: register-only loops of the 16x16x4
// and the four-block 4x4x4 FP64 MFMA and of the FP64 vector FMA, each with
// independent accumulator chains. A calibration for the roofline figures of
// the FP64 kernels (which instruction form a kernel is written in); not part
// of the method.
#include <hip/hip_runtime.h>

#include "../../include/ccham.h"

namespace {

typedef double dx4p __attribute__((ext_vector_type(4)));
constexpr int PROBE_WG = 2048, PROBE_ITERS = 2000;

// MODE 0: 4 chains of 16x16x4 per iteration (4 x 2048 flops a wave);
// MODE 1: 16 four-block 4x4x4 on 8 chains (16 x 512); MODE 2: 64 FMAs on 8
// chains (64 x 64 lanes x 2). The sums are written so nothing is dead code.
template <int MODE>
__global__ __launch_bounds__(256) void k_probe(double *__restrict__ out, int iters, double s)
{
    dx4p acc[4];
    double c[8];
    for (int j = 0; j < 4; ++j) acc[j] = (dx4p){0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < 8; ++j) c[j] = s * j;
    const double a = s * (threadIdx.x + 1), b = s + threadIdx.x;
    for (int i = 0; i < iters; ++i) {
        if (MODE == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        } else if (MODE == 1) {
#pragma unroll
            for (int j = 0; j < 16; ++j) c[j & 7] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c[j & 7], 0, 0, 0);
        } else {
#pragma unroll
            for (int j = 0; j < 64; ++j) c[j & 7] = __builtin_fma(c[j & 7], a, b);
        }
    }
    double t = 0.0;
    for (int j = 0; j < 4; ++j) t += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    for (int j = 0; j < 8; ++j) t += c[j];
    out[blockIdx.x * 256 + threadIdx.x] = t;
}

// flops of one launch: waves x iterations x flops per wave-iteration
constexpr double probe_flops(int mode)
{
    return (double)PROBE_WG * 4 * PROBE_ITERS * (mode == 0 ? 4 * 2048.0 : (mode == 1 ? 16 * 512.0 : 64 * 64 * 2.0));
}

}  // namespace

extern "C" cch_status cch_probe_fp64(int32_t device, void *hip_stream, double *rates)
{
    if (!rates) return CCH_E_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return CCH_E_HIP;
    hipStream_t st = (hipStream_t)hip_stream;
    double *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    cch_status rc = CCH_OK;
    if (hipMalloc((void **)&out, sizeof(double) * PROBE_WG * 256) != hipSuccess) return CCH_E_OOM;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = CCH_E_HIP;
    for (int mode = 0; mode < 3 && rc == CCH_OK; ++mode) {
        float best = 0.0f;
        for (int rep = 0; rep < 3 && rc == CCH_OK; ++rep) {   // the first launch warms up
            if (hipEventRecord(e0, st) != hipSuccess) rc = CCH_E_HIP;
            if (mode == 0) hipLaunchKernelGGL(k_probe<0>, dim3(PROBE_WG), dim3(256), 0, st, out, PROBE_ITERS, 1e-9);
            else if (mode == 1) hipLaunchKernelGGL(k_probe<1>, dim3(PROBE_WG), dim3(256), 0, st, out, PROBE_ITERS, 1e-9);
            else hipLaunchKernelGGL(k_probe<2>, dim3(PROBE_WG), dim3(256), 0, st, out, PROBE_ITERS, 1e-9);
            float ms = 0.0f;
            if (rc == CCH_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
                                 hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = CCH_E_HIP;
            if (rep > 0 && (best == 0.0f || ms < best)) best = ms;
        }
        rates[mode] = rc == CCH_OK && best > 0.0f ? probe_flops(mode) / (best * 1e-3) / 1e12 : 0.0;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}
