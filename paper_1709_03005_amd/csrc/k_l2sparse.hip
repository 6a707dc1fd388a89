// Classes 2 and 8 built sparse (Sec. 2.2: the off-diagonal pure-L2 class is
// the sparse one; Sec. 4 builds an L2-heavy matrix): the L2 block is stored
// as CSR of its structural non-zeros, the L2 determinant pairs within a
// double substitution, and never as a dense block. The structure comes from
// the excitation scan over all pairs (count pass, then the ascending column
// list of each row); the values of the lower triangle are Slater's rules on
// the bitstrings (the same evaluation the dense L2 block uses), each written
// to its own entry and to its mirror in the row of its column, so the stored
// block is exactly symmetric. Beside it, the matrix keeps two dense panels:
// the continuum columns of every row (continuum block and class 4) and the
// transpose of class 4 (the L2 columns of the continuum rows).
#include <algorithm>

#include "ccham_internal.h"

namespace cch {

constexpr int LS_THREADS = 256;

// row x of the L2 block: count (EMIT = false) or list (EMIT = true) the
// columns y in [0, n) with the pair (x, y) within a double substitution,
// ascending, from off[x]
template <int W, bool EMIT>
__global__ __launch_bounds__(LS_THREADS) void k_l2s_struct(const uint64_t *__restrict__ dets, int n,
                                                           const int64_t *__restrict__ off,
                                                           int64_t *__restrict__ cnt, int32_t *__restrict__ col)
{
    const int x = blockIdx.x;
    if (x >= n) return;
    uint64_t a[W];
#pragma unroll
    for (int w = 0; w < W; ++w) a[w] = dets[(size_t)x * W + w];
    __shared__ int wave_tot[LS_THREADS / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t base = EMIT ? off[x] : 0;
    int64_t c = 0;
    for (int y0 = 0; y0 < n; y0 += LS_THREADS) {
        const int y = y0 + threadIdx.x;
        bool conn = false;
        if (y < n) {
            int d = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) d += __popcll(a[w] ^ dets[(size_t)y * W + w]);
            conn = d <= 4;
        }
        if (!EMIT) {
            c += conn;
            continue;
        }
        const uint64_t bal = __ballot(conn);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wave_tot[wv] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < LS_THREADS / 64; ++k) {
            woff += (k < wv) ? wave_tot[k] : 0;
            tot += wave_tot[k];
        }
        if (conn) col[base + woff + before] = y;
        base += tot;
        __syncthreads();   // wave_tot is written again by the next tile
    }
    if (!EMIT) {
        __shared__ int64_t red[LS_THREADS];
        red[threadIdx.x] = c;
        __syncthreads();
        for (int o = LS_THREADS / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) cnt[x] = red[0];
    }
}

// position of column y in row x (the row's columns ascend), -1 if absent
__device__ __forceinline__ int64_t csr_find(const int64_t *__restrict__ off, const int32_t *__restrict__ col, int x,
                                            int y)
{
    int64_t lo = off[x], hi = off[x + 1] - 1;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int c = col[mid];
        if (c == y) return mid;
        if (c < y) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// values: one wave per row x; entry (x, y) with y <= x gets <chi_x|H|chi_y>
// by Slater's rules (bra = row, ket = column, as in the dense L2 block), and
// the same value goes to entry (y, x) of row y
template <int W>
__global__ __launch_bounds__(LS_THREADS) void k_l2s_values(const uint64_t *__restrict__ dets, int n, TgtInts I,
                                                           const int64_t *__restrict__ off,
                                                           const int32_t *__restrict__ col, double *__restrict__ val)
{
    const int lane = threadIdx.x & 63;
    const int x = blockIdx.x * (LS_THREADS / 64) + (threadIdx.x >> 6);
    if (x >= n) return;   // the whole wave
    uint64_t A[W];
#pragma unroll
    for (int w = 0; w < W; ++w) A[w] = dets[(size_t)x * W + w];
    const int64_t e1 = off[x + 1];
    for (int64_t e = off[x] + lane; e < e1; e += 64) {
        const int y = col[e];
        if (y > x) break;   // the columns ascend: the rest of this lane's entries are above the diagonal
        uint64_t B[W];
#pragma unroll
        for (int w = 0; w < W; ++w) B[w] = dets[(size_t)y * W + w];
        int h[2], p[2], s;
        const int deg = excite<W>(A, B, h, p, &s);
        const double v = deg <= 2 ? sc_value<W>(I, A, B, deg, h, p, s) : 0.0;
        val[e] = v;
        if (y < x) {
            const int64_t m = csr_find(off, col, y, x);
            if (m >= 0) val[m] = v;
        }
    }
}

// the diagonal of the L2 block (every row holds its own column)
__global__ void k_l2s_diag(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                           const double *__restrict__ val, int n, double *__restrict__ out)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t m = csr_find(off, col, x, x);
    out[x] = m >= 0 ? val[m] : 0.0;
}

template <int W>
static hipError_t struct_w(bool emit, const uint64_t *dets, int n, const int64_t *off, int64_t *cnt, int32_t *col,
                           hipStream_t st)
{
    if (emit)
        hipLaunchKernelGGL((k_l2s_struct<W, true>), dim3(n), dim3(LS_THREADS), 0, st, dets, n, off, cnt, col);
    else
        hipLaunchKernelGGL((k_l2s_struct<W, false>), dim3(n), dim3(LS_THREADS), 0, st, dets, n, off, cnt, col);
    return hipGetLastError();
}

// count pass (off == nullptr: counts per row into cnt) or column lists
hipError_t launch_l2s_struct(int W, const uint64_t *dets, int n, const int64_t *off, int64_t *cnt, int32_t *col,
                             hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const bool emit = off != nullptr;
    switch (W) {
    case 1: return struct_w<1>(emit, dets, n, off, cnt, col, st);
    case 2: return struct_w<2>(emit, dets, n, off, cnt, col, st);
    case 3: return struct_w<3>(emit, dets, n, off, cnt, col, st);
    case 4: return struct_w<4>(emit, dets, n, off, cnt, col, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_l2s_values(int W, const uint64_t *dets, int n, const TgtInts &I, const int64_t *off,
                             const int32_t *col, double *val, double *diag, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const dim3 g((n + 3) / 4), b(LS_THREADS);
    switch (W) {
    case 1: hipLaunchKernelGGL((k_l2s_values<1>), g, b, 0, st, dets, n, I, off, col, val); break;
    case 2: hipLaunchKernelGGL((k_l2s_values<2>), g, b, 0, st, dets, n, I, off, col, val); break;
    case 3: hipLaunchKernelGGL((k_l2s_values<3>), g, b, 0, st, dets, n, I, off, col, val); break;
    case 4: hipLaunchKernelGGL((k_l2s_values<4>), g, b, 0, st, dets, n, I, off, col, val); break;
    default: return hipErrorInvalidValue;
    }
    if (diag) hipLaunchKernelGGL(k_l2s_diag, dim3((n + 255) / 256), dim3(256), 0, st, off, col, val, n, diag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the dense panels of a sparse-L2 matrix
//   P [D][ldp]: columns < Dc of every row (continuum block, class 4)
//   R [Dc][ldr]: R[r][l] = H[r][Dc + l], the transpose of class 4
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_transpose_c4(const double *__restrict__ P, int64_t ldp, int Dc, int nl2,
                                                      double *__restrict__ R, int64_t ldr)
{
    __shared__ double t[32][33];
    const int l0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int i = ty; i < 32; i += 8) {
        const int l = l0 + i, r = r0 + tx;
        t[i][tx] = (l < nl2 && r < Dc) ? P[(int64_t)(Dc + l) * ldp + r] : 0.0;
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int r = r0 + i, l = l0 + tx;
        if (r < Dc && l < nl2) R[(int64_t)r * ldr + l] = t[tx][i];
    }
}

hipError_t launch_transpose_c4(const double *P, int64_t ldp, int Dc, int nl2, double *R, int64_t ldr, hipStream_t st)
{
    if (Dc <= 0 || nl2 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose_c4, dim3((nl2 + 31) / 32, (Dc + 31) / 32), dim3(256), 0, st, P, ldp, Dc, nl2, R,
                       ldr);
    return hipGetLastError();
}

// H[r][c] of the sparse-L2 matrix
__device__ __forceinline__ double sparse_elem(const SparseMat &S, int64_t r, int64_t c)
{
    if (c < S.Dc) return S.P[r * S.ldp + c];
    if (r < S.Dc) return S.R[r * S.ldr + (c - S.Dc)];
    const int64_t m = csr_find(S.off, S.col, (int)(r - S.Dc), (int)(c - S.Dc));
    return m >= 0 ? S.val[m] : 0.0;
}

__global__ void k_sparse_gather(SparseMat S, const int64_t *__restrict__ rows, const int64_t *__restrict__ cols,
                                int64_t n, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = sparse_elem(S, rows[i], cols[i]);
}

hipError_t launch_sparse_gather(const SparseMat &S, const int64_t *rows, const int64_t *cols, int64_t n, double *out,
                                hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sparse_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, S, rows, cols, n, out);
    return hipGetLastError();
}

// G[a][b] = H[idx[a]][idx[b]], a, b < ns (the seed block of the Davidson start)
__global__ void k_sparse_principal(SparseMat S, const int32_t *__restrict__ idx, int ns, double *__restrict__ G,
                                   int ldg)
{
    const int a = blockIdx.y, b = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < ns && b < ns) G[(int64_t)a * ldg + b] = sparse_elem(S, idx[a], idx[b]);
}

hipError_t launch_sparse_principal(const SparseMat &S, const int32_t *idx, int ns, double *G, int ldg, hipStream_t st)
{
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sparse_principal, dim3((ns + 63) / 64, ns), dim3(64), 0, st, S, idx, ns, G, ldg);
    return hipGetLastError();
}

// rows [r0, r0 + nr) of the matrix written densely into out (leading
// dimension ldo >= D): the read-out of a sparse-L2 matrix, one row block at a
// time. mode 0: every element; mode 2 / 8: only the L2 block's diagonal /
// off-diagonal elements, columns from Dc on (the class blocks of the L2 part)
__global__ __launch_bounds__(256) void k_sparse_rows(SparseMat S, int64_t r0, int nr, int64_t c0, int ncols, int mode,
                                                     double *__restrict__ out, int64_t ldo)
{
    const int i = blockIdx.x;
    if (i >= nr) return;
    const int64_t r = r0 + i;
    double *o = out + (int64_t)i * ldo;
    const bool l2row = r >= S.Dc;
    for (int j = threadIdx.x; j < ncols; j += 256) {
        const int64_t c = c0 + j;
        double v = 0.0;
        if (!l2row || c < S.Dc) v = mode == 0 ? (c < S.Dc ? S.P[r * S.ldp + c] : S.R[r * S.ldr + (c - S.Dc)]) : 0.0;
        o[j] = v;
    }
    if (!l2row) return;
    __syncthreads();   // the zero fill of this row is complete before the scatter
    const int x = (int)(r - S.Dc);
    for (int64_t e = S.off[x] + threadIdx.x; e < S.off[x + 1]; e += 256) {
        const int64_t c = S.Dc + S.col[e];
        if (c < c0 || c >= c0 + ncols) continue;
        const bool diag = S.col[e] == x;
        if (mode == 0 || (mode == 2 && diag) || (mode == 8 && !diag)) o[c - c0] = S.val[e];
    }
}

hipError_t launch_sparse_rows(const SparseMat &S, int64_t r0, int nr, int64_t c0, int ncols, int mode, double *out,
                              int64_t ldo, hipStream_t st)
{
    if (nr <= 0 || ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sparse_rows, dim3(nr), dim3(256), 0, st, S, r0, nr, c0, ncols, mode, out, ldo);
    return hipGetLastError();
}

// off-diagonal row norms rho[r] = sqrt(sum_{c != r} H[r][c]^2) of the
// sparse-L2 matrix (features of the learned correction); one workgroup per row
__global__ __launch_bounds__(256) void k_sparse_row_norms(SparseMat S, int D, double *__restrict__ rho)
{
    const int r = blockIdx.x;
    if (r >= D) return;
    double s = 0.0;
    for (int c = threadIdx.x; c < S.Dc; c += 256)
        if (c != r) {
            const double v = S.P[(int64_t)r * S.ldp + c];
            s += v * v;
        }
    if (r < S.Dc) {
        for (int l = threadIdx.x; l < D - S.Dc; l += 256) {
            const double v = S.R[(int64_t)r * S.ldr + l];
            s += v * v;
        }
    } else {
        const int x = r - S.Dc;
        for (int64_t e = S.off[x] + threadIdx.x; e < S.off[x + 1]; e += 256)
            if (S.col[e] != x) s += S.val[e] * S.val[e];
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) rho[r] = sqrt(red[0]);
}

hipError_t launch_sparse_row_norms(const SparseMat &S, int D, double *rho, hipStream_t st)
{
    if (D <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sparse_row_norms, dim3(D), dim3(256), 0, st, S, D, rho);
    return hipGetLastError();
}

}  // namespace cch
