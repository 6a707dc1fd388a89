// Classes 2 and 8: the pure L2 block <chi_l | H | chi_l'> with no
// contraction (Sec. 2.2), evaluated by Slater's rules on bitstrings for the
// lower triangle (Sec. 3.1 collapses the triangular double loop into one
// loop; here each workgroup takes one 64 x 64 tile of the flattened lower
// triangle). The scan and the element evaluation are fused: every tile
// element is written (zero when more than a double substitution apart).
#include <algorithm>

#include "ccham_internal.h"

namespace cch {

struct L2Args {
    const uint64_t *dets;   // [n_l2][W]
    int n_l2;
    TgtInts I;
    double *H;
    int64_t ld;
    int64_t row0;           // first L2 row / column of the matrix
};

__device__ __forceinline__ void tri_decode(int64_t b, int64_t *ti, int64_t *tj)
{
    // flattened lower-triangular tile index -> (ti >= tj)
    int64_t i = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > b) --i;
    while ((i + 1) * (i + 2) / 2 <= b) ++i;
    *ti = i;
    *tj = b - i * (i + 1) / 2;
}

template <int W>
__device__ __forceinline__ void l2_tile(const L2Args &a, int64_t b, uint64_t (*bra)[W], uint64_t (*ket)[W])
{
    int64_t ti, tj;
    tri_decode(b, &ti, &tj);
    const int l0 = (int)(ti * 64), k0 = (int)(tj * 64);
    __syncthreads();   // the LDS dets are reused by the next tile of a persistent loop
    for (int t = threadIdx.x; t < 64 * W; t += 256) {
        const int r = t / W, w = t % W;
        bra[r][w] = (l0 + r < a.n_l2) ? a.dets[(size_t)(l0 + r) * W + w] : 0ull;
        ket[r][w] = (k0 + r < a.n_l2) ? a.dets[(size_t)(k0 + r) * W + w] : 0ull;
    }
    __syncthreads();
    const int c = threadIdx.x & 63;
    const int lc = k0 + c;
    uint64_t B[W];
#pragma unroll
    for (int w = 0; w < W; ++w) B[w] = ket[c][w];
    for (int r = threadIdx.x >> 6; r < 64; r += 4) {
        const int lr = l0 + r;
        if (lr >= a.n_l2 || lc >= a.n_l2 || lc > lr) continue;
        uint64_t A[W];
#pragma unroll
        for (int w = 0; w < W; ++w) A[w] = bra[r][w];
        int h[2], p[2], s;
        const int deg = excite<W>(A, B, h, p, &s);
        double v = 0.0;
        if (deg <= 2) v = sc_value<W>(a.I, A, B, deg, h, p, s);
        a.H[(a.row0 + lr) * a.ld + a.row0 + lc] = v;
    }
}

template <int W>
__global__ __launch_bounds__(256) void k_l2_block(L2Args a)
{
    __shared__ uint64_t bra[64][W], ket[64][W];
    l2_tile<W>(a, blockIdx.x, bra, ket);
}

hipError_t launch_l2_block(int W, const L2Args &a, hipStream_t st)
{
    if (a.n_l2 <= 0) return hipSuccess;
    const int64_t T = (a.n_l2 + 63) / 64;
    const int64_t nb = T * (T + 1) / 2;
    const dim3 g((unsigned)nb), bl(256);
    switch (W) {
    case 1: hipLaunchKernelGGL((k_l2_block<1>), g, bl, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_l2_block<2>), g, bl, 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_l2_block<3>), g, bl, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_l2_block<4>), g, bl, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// L2 functions given as CSFs, chi_l = sum_t coef_t |det_t> (Eq. 1's second
// sum over configuration state functions): the lower triangle of the matrix
// over the CSFs from the lower triangle of the one built over the distinct L2
// determinants (Hd, not mirrored): continuum rows are copied, a class-4 row
// is sum_t coef_t Hd[det_t][c], an L2 x L2 element sum_t sum_u coef_t coef_u
// Hd[det_t][det_u] (read from the lower triangle), terms in input order. One
// workgroup per row.
__global__ __launch_bounds__(256) void k_l2csf_gather(const double *__restrict__ Hd, int64_t ldd, int Dc,
                                                      const int32_t *__restrict__ start,
                                                      const int32_t *__restrict__ det,
                                                      const double *__restrict__ coef, double *__restrict__ H,
                                                      int64_t ld)
{
    const int64_t r = blockIdx.x;
    double *out = H + r * ld;
    if (r < Dc) {
        const double *in = Hd + r * ldd;
        for (int64_t c = threadIdx.x; c <= r; c += blockDim.x) out[c] = in[c];
        return;
    }
    const int a = (int)(r - Dc);
    const int t0 = start[a], t1 = start[a + 1];
    for (int64_t c = threadIdx.x; c <= r; c += blockDim.x) {
        double v = 0.0;
        if (c < Dc) {
            for (int t = t0; t < t1; ++t) v += coef[t] * Hd[(Dc + (int64_t)det[t]) * ldd + c];
        } else {
            const int b = (int)(c - Dc), u0 = start[b], u1 = start[b + 1];
            for (int t = t0; t < t1; ++t) {
                const int64_t x = Dc + (int64_t)det[t];
                double s = 0.0;
                for (int u = u0; u < u1; ++u) {
                    const int64_t y = Dc + (int64_t)det[u];
                    s += coef[u] * (x >= y ? Hd[x * ldd + y] : Hd[y * ldd + x]);
                }
                v += coef[t] * s;
            }
        }
        out[c] = v;
    }
}

hipError_t launch_l2csf_gather(const double *Hd, int64_t ldd, int Dc, int ncsf, const int32_t *start,
                               const int32_t *det, const double *coef, double *H, int64_t ld, hipStream_t st)
{
    const int64_t D = (int64_t)Dc + ncsf;
    if (D <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_l2csf_gather, dim3((unsigned)D), dim3(256), 0, st, Hd, ldd, Dc, start, det, coef, H, ld);
    return hipGetLastError();
}

// persistent form over many instances with the same word count
struct L2Task {
    L2Args a;
    int64_t first;   // first global tile of this instance
};

int64_t l2_tiles(int n_l2)
{
    const int64_t T = (n_l2 + 63) / 64;
    return T * (T + 1) / 2;
}

template <int W>
__global__ __launch_bounds__(256) void k_l2_batched(const L2Task *__restrict__ tasks, int ntask, int64_t total)
{
    __shared__ uint64_t bra[64][W], ket[64][W];
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = ntask - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tasks[mid].first <= t) lo = mid;
            else hi = mid - 1;
        }
        l2_tile<W>(tasks[lo].a, t - tasks[lo].first, bra, ket);
    }
}

hipError_t launch_l2_batched(int W, const L2Task *tasks, int ntask, int64_t total, int grid, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    const dim3 g((unsigned)std::min<int64_t>(total, grid)), bl(256);
    switch (W) {
    case 1: hipLaunchKernelGGL((k_l2_batched<1>), g, bl, 0, st, tasks, ntask, total); break;
    case 2: hipLaunchKernelGGL((k_l2_batched<2>), g, bl, 0, st, tasks, ntask, total); break;
    case 3: hipLaunchKernelGGL((k_l2_batched<3>), g, bl, 0, st, tasks, ntask, total); break;
    case 4: hipLaunchKernelGGL((k_l2_batched<4>), g, bl, 0, st, tasks, ntask, total); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace cch
