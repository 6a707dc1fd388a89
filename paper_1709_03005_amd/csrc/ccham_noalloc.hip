// cch_subspace_eig_noalloc: the Rayleigh-Ritz eigenproblem of the Davidson
// solver (every eigenpair of a small symmetric matrix, FP64) without any
// device allocation. Its staging buffers and fallback counter live in one
// file-scope device array per GPU; host code reaches that array only through
// the address hipGetSymbolAddress returns on each device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ccham.h"
#include "ccham_internal.h"

namespace cch {
hipError_t launch_rr_eig(const double *G, int ldg, int m, double *theta, double *Y, int ldy, int32_t *nfallback,
                         hipStream_t st);
hipError_t launch_jacobi_eig(const double *G, int ldg, int m, double *theta, double *Y, int ldy, hipStream_t st);
}  // namespace cch

// context fields this entry point needs (device, stream, error text)
int32_t cch_ctx_device(const cch_ctx *c);
hipStream_t cch_ctx_stream(const cch_ctx *c);
cch_status cch_ctx_fail(cch_ctx *c, cch_status code, const char *msg);

namespace {
constexpr int NA_MMAX = 96;                                   // largest m accepted
constexpr size_t NA_MAT = (size_t)NA_MMAX * NA_MMAX;          // doubles per staged matrix
// layout (doubles): [0] fallback counter (8 bytes), [32, 32 + NA_MAT) G,
// then Y (NA_MAT), then theta (NA_MMAX); every part 256-byte aligned
constexpr size_t NA_OFF_G = 32, NA_OFF_Y = NA_OFF_G + NA_MAT, NA_OFF_T = NA_OFF_Y + NA_MAT;
constexpr size_t NA_DOUBLES = NA_OFF_T + NA_MMAX;             // 148 480 bytes in all
constexpr int NA_MAX_DEV = 64;
}  // namespace

// one copy per GPU, held until the process ends
static __device__ __align__(256) double scratch[NA_DOUBLES];

namespace {
std::mutex na_mu;
double *na_ptr[NA_MAX_DEV] = {};   // device address of `scratch` on each device (nullptr: not resolved)

// the device address of this device's array; resolved once per device with
// the device current (the caller has made it current)
hipError_t na_scratch(int dev, double **out)
{
    if (dev < 0 || dev >= NA_MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(na_mu);
    if (!na_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        na_ptr[dev] = static_cast<double *>(p);
    }
    *out = na_ptr[dev];
    return hipSuccess;
}
}  // namespace

cch_status cch_subspace_eig_noalloc(cch_ctx *c, const double *G, int32_t ldg, int32_t m, double *theta, double *Y,
                                    int32_t ldy, int32_t method, int32_t *fallback, int32_t flags)
{
    if (!c || !G || !theta || !Y) return CCH_E_INVALID_ARG;
    if (m < 1 || m > NA_MMAX)
        return cch_ctx_fail(c, CCH_E_INVALID_ARG, "cch_subspace_eig_noalloc: m must lie in [1, 96] (scratch limit)");
    if (ldg < m || ldy < m) return cch_ctx_fail(c, CCH_E_INVALID_ARG, "leading dimension below m");
    if (method != CCH_EIG_AUTO && method != CCH_EIG_JACOBI)
        return cch_ctx_fail(c, CCH_E_INVALID_ARG, "unknown method");
    const bool dev = flags & CCH_MEM_DEVICE;
    // host arrays are staged with the scratch's own leading dimension m; their
    // extents must fit it (device arrays are used in place)
    const int dev_id = cch_ctx_device(c);
    hipStream_t st = cch_ctx_stream(c);
    hipError_t e = hipSetDevice(dev_id);
    double *base = nullptr;
    if (e == hipSuccess) e = na_scratch(dev_id, &base);
    if (e != hipSuccess) return cch_ctx_fail(c, CCH_E_HIP, hipGetErrorString(e));
    int32_t *d_fb = reinterpret_cast<int32_t *>(base);
    const double *dG = G;
    double *dT = theta, *dY = Y;
    int lg = ldg, ly = ldy;
    // every call shares this device's array: the counter starts at zero
    e = cch::launch_fill_i64(reinterpret_cast<int64_t *>(base), 0, 1, st);
    if (e == hipSuccess && !dev) {
        // G is read row by row into the scratch with leading dimension m
        e = hipMemcpy2DAsync(base + NA_OFF_G, 8 * (size_t)m, G, 8 * (size_t)ldg, 8 * (size_t)m, m,
                             hipMemcpyHostToDevice, st);
        dG = base + NA_OFF_G;
        dY = base + NA_OFF_Y;
        dT = base + NA_OFF_T;
        lg = ly = m;
    }
    if (e == hipSuccess) {
        if (method == CCH_EIG_JACOBI) e = cch::launch_jacobi_eig(dG, lg, m, dT, dY, ly, st);
        else e = cch::launch_rr_eig(dG, lg, m, dT, dY, ly, d_fb, st);
    }
    int32_t hf = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hf, d_fb, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && !dev) {
        e = hipMemcpyAsync(theta, dT, 8 * (size_t)m, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(Y, 8 * (size_t)ldy, dY, 8 * (size_t)m, 8 * (size_t)m, m, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return cch_ctx_fail(c, CCH_E_HIP, hipGetErrorString(e));
    if (fallback) *fallback = hf;
    return CCH_OK;
}
