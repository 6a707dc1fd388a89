// Matrix bookkeeping kernels: mirror of the lower triangle (the matrix is
// real symmetric and only the lower triangle is evaluated, Sec. 2.2),
// diagonal extraction, and fills that replace memsets on the stream.
#include <algorithm>

#include "ccham_internal.h"

namespace cch {

// H[c][r] = H[r][c] for r > c, over 64 x 64 tiles of the lower triangle;
// off-diagonal tiles go through LDS so both reads and writes are coalesced.
__global__ __launch_bounds__(256) void k_mirror(double *__restrict__ H, int64_t ld, int D)
{
    __shared__ double tile[64][65];
    const int64_t b = blockIdx.x;
    int64_t ti = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > b) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    const int64_t tj = b - ti * (ti + 1) / 2;
    const int r0 = (int)(ti * 64), c0 = (int)(tj * 64);
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int R = r0 + r, C = c0 + tx;
        tile[r][tx] = (R < D && C < D) ? H[(int64_t)R * ld + C] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        // destination row c0 + r, column r0 + tx  <-  source (r0 + tx, c0 + r)
        const int R = c0 + r, C = r0 + tx;
        if (R < D && C < D && C > R) H[(int64_t)R * ld + C] = tile[tx][r];
    }
}

hipError_t launch_mirror(double *H, int64_t ld, int D, hipStream_t st)
{
    if (D <= 0) return hipSuccess;
    const int64_t T = (D + 63) / 64;
    hipLaunchKernelGGL(k_mirror, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, st, H, ld, D);
    return hipGetLastError();
}

__global__ void k_diag(const double *__restrict__ H, int64_t ld, int D, double *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < D) out[i] = H[(int64_t)i * ld + i];
}

hipError_t launch_diag(const double *H, int64_t ld, int D, double *out, hipStream_t st)
{
    if (D <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag, dim3((D + 255) / 256), dim3(256), 0, st, H, ld, D, out);
    return hipGetLastError();
}

// out[r * ldo + c] = H[(row0 + r) * ldh + col0 + c] where the element belongs to
// the selected class, else 0. mode: 0 every element; 1 / 3 same / different
// target state (r / nca vs c / ncb); 5 / 6 same / different continuum orbital
// (r % nca vs c % ncb); 2 / 8 diagonal / off-diagonal (r vs c)
__global__ void k_get_block(const double *__restrict__ H, int64_t ldh, int64_t row0, int nrows, int64_t col0,
                            int ncols, int mode, int nca, int ncb, double *__restrict__ out, int64_t ldo)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= ncols || r >= nrows) return;
    bool keep = true;
    if (mode == 1) keep = r / nca == c / ncb;
    else if (mode == 3) keep = r / nca != c / ncb;
    else if (mode == 5) keep = r % nca == c % ncb;
    else if (mode == 6) keep = r % nca != c % ncb;
    else if (mode == 2) keep = r == c;
    else if (mode == 8) keep = r != c;
    out[(int64_t)r * ldo + c] = keep ? H[(row0 + r) * ldh + col0 + c] : 0.0;
}

hipError_t launch_get_block(const double *H, int64_t ldh, int64_t row0, int nrows, int64_t col0, int ncols, int mode,
                            int nca, int ncb, double *out, int64_t ldo, hipStream_t st)
{
    if (nrows <= 0 || ncols <= 0) return hipSuccess;
    if ((mode == 1 || mode == 3 || mode == 5 || mode == 6) && (nca <= 0 || ncb <= 0)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_get_block, dim3((ncols + 255) / 256, nrows), dim3(256), 0, st, H, ldh, row0, nrows, col0,
                       ncols, mode, nca, ncb, out, ldo);
    return hipGetLastError();
}

// out[i] = H[rows[i]][cols[i]], indices checked by the caller
__global__ void k_gather_elements(const double *__restrict__ H, int64_t ldh, const int64_t *__restrict__ rows,
                                  const int64_t *__restrict__ cols, int64_t n, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = H[rows[i] * ldh + cols[i]];
}

hipError_t launch_gather_elements(const double *H, int64_t ldh, const int64_t *rows, const int64_t *cols, int64_t n,
                                  double *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_elements, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, H, ldh, rows, cols, n,
                       out);
    return hipGetLastError();
}

__global__ void k_fill_i64(int64_t *__restrict__ p, int64_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

__global__ void k_fill_f64(double *__restrict__ p, double v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// census of a pair list for the work counts: out[0] degree-0 pairs, out[1]
// degree-1 pairs whose excitation is alpha, out[2] degree-1 beta, out[3]
// degree-2 pairs (integer atomics: the counts do not depend on the order)
__global__ __launch_bounds__(256) void k_pair_census(const int8_t *__restrict__ deg,
                                                     const uint64_t *__restrict__ label, int64_t n,
                                                     unsigned long long *__restrict__ out)
{
    unsigned long long c[4] = {0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int d = deg[i];
        if (d == 0) ++c[0];
        else if (d == 1) ++c[(label[i] & 1u) ? 2 : 1];   // field 0 = particle spin-orbital, bit 0 = spin
        else ++c[3];
    }
    __shared__ unsigned long long red[4][256];
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = c[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) atomicAdd(&out[threadIdx.x], red[threadIdx.x][0]);
}

hipError_t launch_pair_census(const int8_t *deg, const uint64_t *label, int64_t n, unsigned long long *out,
                              hipStream_t st)
{
    hipError_t e = launch_fill_i64(reinterpret_cast<int64_t *>(out), 0, 4, st);
    if (e != hipSuccess || n <= 0) return e;
    const int grid = (int)std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_pair_census, dim3(grid), dim3(256), 0, st, deg, label, n, out);
    return hipGetLastError();
}

// out[x][y] (or out[y][x] when transposed) = value of pair i of a pair list
__global__ void k_scatter_pairs(const int32_t *__restrict__ px, const int32_t *__restrict__ py,
                                const double *__restrict__ v, int64_t n, int transpose, double *__restrict__ out,
                                int64_t ldo)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t x = px[i], y = py[i];
    out[transpose ? y * ldo + x : x * ldo + y] = v[i];
}

hipError_t launch_scatter_pairs(const int32_t *px, const int32_t *py, const double *v, int64_t n, int transpose,
                                double *out, int64_t ldo, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, px, py, v, n, transpose,
                       out, ldo);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

}  // namespace cch
