// Every eigenpair of a dense real symmetric matrix in FP64 on one GPU (the
// paper's Sec. 3.2 notes that often all eigenvectors are wanted and a dense
// diagonaliser is used then):
//   1. Householder tridiagonalisation Q^T A Q = T, one reflector per column,
//      blocked in panels of TRD_NB columns with lazy updates: per column
//      the corrected column with its partial sums, then the product of the
//      trailing block with the reflector (the HBM-bound part: from the lower
//      triangle in tiles, plus a kernel that adds the tiles' partial sums,
//      while the block has at least TRD_TILE_MIN rows; by whole rows below
//      that), and one rank-2 TRD_NB FP64 MFMA update of the trailing block
//      per panel.
//   2. Eigenvalues of T by multisection on Sturm counts, 8 lanes each.
//   3. Eigenvectors of T by twisted factorisations, one thread each, with
//      modified Gram-Schmidt (and inverse iteration for vectors that
//      collapse) inside clusters of close eigenvalues, one workgroup each.
//   4. Back-transformation Z = Q Z_T in blocks of 128 reflectors, each as
//      I - V T V^T (compact WY) by three FP64 MFMA products.
#include <algorithm>
#include <cmath>

#include "ccham_internal.h"

namespace cch {

// ---------------------------------------------------------------------------
// general FP64 MFMA product C = alpha A B + beta C (row-major C)
//   A(i, k) = A[i * sai + k * sak], B(k, j) = B[k * sbk + j * sbj]
// 64 x 64 tile per workgroup (4 waves of 32 x 32, on the 4x4x4 form: it
// issues faster per flop than 16x16x4 on this chip), K staged through LDS in
// slices of 16 (the next slice loaded into registers during the products);
// loads follow whichever index of an operand has stride 1; C, when the
// product adds to it, is loaded at entry
// ---------------------------------------------------------------------------
constexpr int EG_T = 64, EG_K = 16;

// With P != nullptr the K range is split over blockIdx.z (kc each) and each
// split writes its unscaled partial product to P[z][M][N]; k_eig_gemm_sum adds
// the splits in order and applies alpha and beta (deterministic).
__global__ __launch_bounds__(256) void k_eig_gemm(int M, int N, int K, double alpha, const double *__restrict__ A,
                                                  int64_t sai, int64_t sak, const double *__restrict__ B, int64_t sbk,
                                                  int64_t sbj, double beta, double *__restrict__ C, int64_t ldc,
                                                  int kc, double *__restrict__ P, int lowq)
{
    // lowq >= 0: only the tiles on and below the diagonal, and every tile of
    // the square of tile rows and columns >= lowq
    if (lowq >= 0 && (int)blockIdx.x > (int)blockIdx.y && ((int)blockIdx.x < lowq || (int)blockIdx.y < lowq)) return;
    __shared__ double As[EG_K][EG_T + 1], Bs[EG_K][EG_T + 1];
    const int i0 = blockIdx.y * EG_T, j0 = blockIdx.x * EG_T;
    const int kb0 = P ? (int)blockIdx.z * kc : 0, kb1 = P ? min(K, kb0 + kc) : K;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    const bool a_kfast = sak == 1, b_jfast = sbj == 1;
    // C of this thread's outputs, loaded at entry when the product adds to it
    const bool addc = P == nullptr && beta != 0.0;
    // 4x4x4 FP64 MFMA, four blocks with the same A: an instruction multiplies
    // 4 rows (A at lane i + 16 k, any block) by 16 columns (B at lane
    // j + 16 k), the result D[i][j] at lane j + 16 i. A wave's 32 x 32 tile is
    // 8 row quads x 2 column groups.
    double cin[8][2];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int i = i0 + wm * 32 + 4 * a + (lane >> 4);
            const int j = j0 + wn * 32 + 16 * b + (lane & 15);
            cin[a][b] = addc && i < M && j < N ? C[(int64_t)i * ldc + j] : 0.0;
        }
    double acc[8][2];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = 0.0;
    // the K slices pass through registers: the next one is loaded while the
    // current one is multiplied from LDS
    double ra[4], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int ii, kk;
            if (a_kfast) { kk = t & 15; ii = (t >> 4) + 16 * u; }
            else { ii = t & 63; kk = (t >> 6) + 4 * u; }
            const int i = i0 + ii, k = k0 + kk;
            ra[u] = (i < M && k < kb1) ? A[(int64_t)i * sai + (int64_t)k * sak] : 0.0;
            int jj, kb;
            if (b_jfast) { jj = t & 63; kb = (t >> 6) + 4 * u; }
            else { kb = t & 15; jj = (t >> 4) + 16 * u; }
            const int j = j0 + jj, kq = k0 + kb;
            rb[u] = (j < N && kq < kb1) ? B[(int64_t)kq * sbk + (int64_t)j * sbj] : 0.0;
        }
    };
    if (kb0 < kb1) load(kb0);
    for (int k0 = kb0; k0 < kb1; k0 += EG_K) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int ii, kk;
            if (a_kfast) { kk = t & 15; ii = (t >> 4) + 16 * u; }
            else { ii = t & 63; kk = (t >> 6) + 4 * u; }
            As[kk][ii] = ra[u];
            int jj, kb;
            if (b_jfast) { jj = t & 63; kb = (t >> 6) + 4 * u; }
            else { kb = t & 15; jj = (t >> 4) + 16 * u; }
            Bs[kb][jj] = rb[u];
        }
        __syncthreads();
        if (k0 + EG_K < kb1) load(k0 + EG_K);
#pragma unroll
        for (int ks = 0; ks < EG_K; ks += 4) {
            const int kk = ks + (lane >> 4);
            double af[8], bf[2];
#pragma unroll
            for (int a = 0; a < 8; ++a) af[a] = As[kk][wm * 32 + 4 * a + (lane & 3)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bf[b] = Bs[kk][wn * 32 + 16 * b + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int i = i0 + wm * 32 + 4 * a + (lane >> 4);
        if (i >= M) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int j = j0 + wn * 32 + 16 * b + (lane & 15);
            if (j >= N) continue;
            if (P) P[((int64_t)blockIdx.z * M + i) * N + j] = acc[a][b];
            else C[(int64_t)i * ldc + j] = alpha * acc[a][b] + (beta == 0.0 ? 0.0 : beta * cin[a][b]);
        }
    }
}

__global__ void k_eig_gemm_sum(int M, int N, int ns, const double *__restrict__ P, double alpha, double beta,
                               double *__restrict__ C, int64_t ldc)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * N) return;
    double s = 0.0;
    for (int z = 0; z < ns; ++z) s += P[(int64_t)z * M * N + e];
    double *c = C + (e / N) * ldc + e % N;
    *c = alpha * s + (beta == 0.0 ? 0.0 : beta * *c);
}

// P (optional, p_cap doubles): split-K scratch for products with few output
// tiles and a long K (the Gram and projection products of the
// back-transformation)
hipError_t launch_eig_gemm(int M, int N, int K, double alpha, const double *A, int64_t sai, int64_t sak,
                           const double *B, int64_t sbk, int64_t sbj, double beta, double *C, int64_t ldc,
                           hipStream_t st, double *P, int64_t p_cap, int lowq)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    const dim3 g((N + EG_T - 1) / EG_T, (M + EG_T - 1) / EG_T);
    const int64_t tiles = (int64_t)g.x * g.y;
    int ns = 1;
    if (P && lowq < 0 && tiles < 512 && K >= 1024) {
        ns = (int)std::min<int64_t>({(K + 255) / 256, std::max<int64_t>(1, 1024 / tiles), 64});
        ns = (int)std::min<int64_t>(ns, p_cap / ((int64_t)M * N));
    }
    if (ns <= 1) {
        hipLaunchKernelGGL(k_eig_gemm, g, dim3(256), 0, st, M, N, K, alpha, A, sai, sak, B, sbk, sbj, beta, C, ldc,
                           K, (double *)nullptr, lowq);
        return hipGetLastError();
    }
    const int kc = ((K + ns - 1) / ns + EG_K - 1) / EG_K * EG_K;
    ns = (K + kc - 1) / kc;
    hipLaunchKernelGGL(k_eig_gemm, dim3(g.x, g.y, ns), dim3(256), 0, st, M, N, K, alpha, A, sai, sak, B, sbk, sbj,
                       beta, C, ldc, kc, P, -1);
    const int64_t e = (int64_t)M * N;
    hipLaunchKernelGGL(k_eig_gemm_sum, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, M, N, ns, P, alpha, beta,
                       C, ldc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 1. tridiagonalisation (lower triangle convention: reflector j annihilates
//    A[j+2:, j]; v_j[j+1] = 1 is stored explicitly in A[j+1][j] and below),
//    blocked with lazy updates: in a panel of TRD_NB columns the trailing
//    matrix A_0 is only read. The matrix after the panel's reflectors k < i is
//    A_0 - sum_k (v_k w_k^T + w_k v_k^T), so column j is read from A_0 and
//    corrected, and its product A_j v_j = A_0 v_j - sum_k (v_k (w_k . v_j) +
//    w_k (v_k . v_j)); one rank-2 TRD_NB product (FP64 MFMA) updates the
//    trailing block at the end of the panel. w_j = p - (tau_j / 2)(p . v_j) v_j
//    with p = tau_j A_j v_j.
// Per column a column kernel and a pass, each spread over the rows; a
// workgroup never waits for another one. The column kernel adds the pass's
// partial sums of p . v (the scalar of the previous w), finishes that w,
// corrects column j and stores, per workgroup, the partial sums of sigma =
// |x|^2 over the part to annihilate and of the panel's vectors times it.
// Every workgroup of the pass adds those partial sums in workgroup order (so
// all get the same reflector) and forms v_j = x / (alpha - beta) as it reads
// it; the pass leaves p and the partial sums of p . v_j. For trailing blocks
// of at least TRD_TILE_MIN rows the pass reads only the lower triangle, in
// tiles, and a second kernel adds each row's tile sums.
// panel buffers (ldp doubles a row): PV rows 2k, 2k + 1 = v_k, w_k; PW rows
// 2k, 2k + 1 = w_k, v_k (the update is A -= PV^T PW over 2 nb rows); PVt the
// same values by matrix row (PVt[r][d] = PV[d][r]: a row's panel entries are
// contiguous for the kernels that read them per row); z[2k] = v_k . v_j,
// z[2k + 1] = w_k . v_j. Entries below the reflector's first row are never
// read.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double blk_sum(double x, double *red)
{
    // sum over the 256 threads of a workgroup (red: 256 doubles of LDS)
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// x[b stride] summed for b = b0, b0 + step, ... < b1 in that order; the
// loads go out in batches of 8
__device__ __forceinline__ double ordered_sum(const double *__restrict__ x, int64_t stride, int b0, int b1, int step)
{
    double y = 0.0;
    for (int b = b0; b < b1; b += 8 * step) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int c = b + u * step;
            v[u] = c < b1 ? x[(int64_t)c * stride] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) y += v[u];
    }
    return y;
}

// rows j + TRD_CR blockIdx.x + threadIdx.x. With i > 0, w of the panel's
// reflector i - 1 (column j - 1) into PV row 2i - 1 and PW row 2i - 2 for
// rows >= j. With col: column j of the current matrix into wp, d[j], and the
// partial sums [sigma, PV[0] . x, ..., PV[2i - 1] . x] of this workgroup's
// rows >= j + 2 into part1.
__global__ __launch_bounds__(256) void k_trd_col(const double *__restrict__ A, int64_t lda, int n, int j, int i,
                                                 int col, TrdVec V, TrdPanel P)
{
    __shared__ double vw[2 * TRD_NB];   // v_k[j], w_k[j], k < i
    __shared__ double xs[TRD_CR], ws[TRD_CR];
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int r0 = j + (int)blockIdx.x * TRD_CR, r = r0 + t;
    const bool in = r < n;
    double wr = 0.0;
    if (i > 0) {
        // p of reflector j - 1 (rows >= j) and the scalar -(tau / 2)(p . v) of its w
        const double *vq = P.PVt + (2 * i - 2);   // v of reflector i - 1, stride 2 TRD_NB
        // (the row pass leaves one partial sum of p . v per 4 rows, the sum
        // kernel of the tiled pass one per TRD_SR rows)
        const int g2 = n - j < TRD_TILE_MIN ? (n - j + 3) / 4 : (n - j + TRD_SR - 1) / TRD_SR;
        const double al = -0.5 * V.tau[j - 1] * blk_sum(ordered_sum(P.part2, 1, t, g2, 256), red);
        const double pr = in ? V.p[r] : 0.0, pj = t == 0 ? V.p[j] : 0.0;
        if (in) {
            wr = pr + al * vq[(int64_t)r * TRD_PT];
            P.PV[(int64_t)(2 * i - 1) * P.ldp + r] = wr;
            P.PW[(int64_t)(2 * i - 2) * P.ldp + r] = wr;
            P.PVt[(int64_t)r * TRD_PT + 2 * i - 1] = wr;
        }
        if (col && t == 0) {
            vw[2 * i - 2] = vq[(int64_t)j * TRD_PT];
            vw[2 * i - 1] = pj + al * vq[(int64_t)j * TRD_PT];
        }
    }
    if (!col) return;
    for (int e = t; e < 2 * i - 2; e += 256) vw[e] = P.PVt[(int64_t)j * TRD_PT + e];
    __syncthreads();
    double x = 0.0;
    if (in) {
        x = A[(int64_t)r * lda + j];
#pragma unroll 4
        for (int k = 0; k < i - 1; ++k)
            x -= P.PVt[(int64_t)r * TRD_PT + 2 * k] * vw[2 * k + 1] + P.PVt[(int64_t)r * TRD_PT + 2 * k + 1] * vw[2 * k];
        if (i > 0) x -= P.PVt[(int64_t)r * TRD_PT + 2 * i - 2] * vw[2 * i - 1] + wr * vw[2 * i - 2];
        V.wp[r] = x;
        if (r == j) V.d[j] = x;
    }
    if (j >= n - 1) return;   // the last column has no reflector (one workgroup)
    const bool below = in && r >= j + 2;
    xs[t] = below ? x : 0.0;
    ws[t] = below ? wr : 0.0;
    const double sig = blk_sum(below ? x * x : 0.0, red);   // (its barriers publish xs, ws)
    // PV[q] . x over this workgroup's rows: thread (q = t mod 64, g = t / 64)
    // over the 64 rows 64 g .. 64 g + 63, then the four groups in order
    const int q = t & 63, g = t >> 6;
    double y = 0.0;
    if (q < 2 * i - 1) {
        // (the 64 lanes read 64 consecutive entries of one row of PVt)
        const double *pr = P.PVt + (int64_t)(r0 + 64 * g) * TRD_PT + q;
        const int lo = max(0, j + 2 - r0 - 64 * g), hi = min(64, n - r0 - 64 * g);
#pragma unroll 16
        for (int k = lo; k < hi; ++k) y += pr[(int64_t)k * TRD_PT] * xs[64 * g + k];
    } else if (q == 2 * i - 1) {   // w_{i-1}, kept in ws
#pragma unroll 16
        for (int k = 0; k < 64; ++k) y += ws[64 * g + k] * xs[64 * g + k];
    }
    __syncthreads();
    red[t] = y;
    __syncthreads();
    double *out = P.part1 + (int64_t)blockIdx.x * TRD_PS;
    if (t == 0) out[0] = sig;
    if (t < 2 * i) out[1 + t] = red[t] + red[64 + t] + red[128 + t] + red[192 + t];
}

// rows r of the trailing block (j, n), one wave per row, lanes over the
// columns, fixed-order reductions: v_j[r] into column j of A and the panel
// buffers, p[r] = tau_j (A_0[r][j+1:] . v_j - sum_k (v_k[r] (w_k . v_j) +
// w_k[r] (v_k . v_j))), and this workgroup's partial sum of p . v_j into
// part2. The row is streamed first as A_0[r][j+1] + scale (A_0[r][j+2:] . x)
// (v_j = 1 at row j + 1 and scale x below), while every workgroup forms the
// reflector of column j from the column kernel's partial sums (workgroup 0
// stores e[j] and tau[j]) and z.
__global__ __launch_bounds__(256) void k_trd_pass(double *__restrict__ A, int64_t lda, int n, int j, int i, TrdVec V,
                                                  TrdPanel P)
{
    __shared__ double red[TRD_PS];
    __shared__ double zs[2 * TRD_NB];
    __shared__ double sc[2];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int g1 = (n - j + TRD_CR - 1) / TRD_CR;
    const int r = j + 1 + (int)blockIdx.x * 4 + wv;
    const bool in = r < n;
    // loads first: the partial sums, z's panel entries at row j + 1, alpha,
    // this row's panel entries and x at this row
    double ps = 0.0;
    if (t < 2 * i + 1) {
        double u[32];
#pragma unroll
        for (int b = 0; b < 32; ++b) u[b] = b < g1 ? P.part1[(int64_t)b * TRD_PS + t] : 0.0;
#pragma unroll
        for (int b = 0; b < 32; ++b) ps += u[b];
        for (int b = 32; b < g1; ++b) ps += P.part1[(int64_t)b * TRD_PS + t];
    }
    const double pz = t < 2 * i ? P.PVt[(int64_t)(j + 1) * TRD_PT + t] : 0.0;
    const double alpha = t == 0 ? V.wp[j + 1] : 0.0;
    double k0 = 0.0, k1 = 0.0, xr = 0.0;
    if (in && lane < i) {
        k0 = P.PVt[(int64_t)r * TRD_PT + 2 * lane];
        k1 = P.PVt[(int64_t)r * TRD_PT + 2 * lane + 1];
    }
    if (in) xr = V.wp[r];
    // the row: A_0[r][j+1] and A_0[r][j+2:] . x
    double s1 = 0.0, s2 = 0.0;
    if (in) {
        const double *row = A + (int64_t)r * lda;
        if (lane == 0) s1 = row[j + 1];
#pragma unroll 8
        for (int c = j + 2 + lane; c < n; c += 64) s2 += row[c] * V.wp[c];
        for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
    }
    if (t < 2 * i + 1) red[t] = ps;
    __syncthreads();
    if (t == 0) {
        const double sig = red[0];
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (sig > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + sig), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        sc[0] = scale;
        sc[1] = tau;
        if (blockIdx.x == 0) {
            V.e[j] = beta;
            V.tau[j] = tau;
        }
    }
    __syncthreads();
    const double scale = sc[0], tau = sc[1];
    // z[d] = PV[d] . v_j with v_j[j + 1] = 1 and v_j = scale x below
    if (t < 2 * i) zs[t] = pz + scale * red[t + 1];
    __syncthreads();
    double pv = 0.0;
    if (in) {
        double q = lane < i ? k0 * zs[2 * lane + 1] + k1 * zs[2 * lane] : 0.0;
        for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
        const double sr = __shfl(s1, 0, 64) + scale * s2;
        const double vr = r == j + 1 ? 1.0 : xr * scale;
        const double p = tau * (sr - q);
        if (lane == 0) {
            V.p[r] = p;
            A[(int64_t)r * lda + j] = vr;   // kept for the back-transformation
            P.PV[(int64_t)(2 * i) * P.ldp + r] = vr;
            P.PW[(int64_t)(2 * i + 1) * P.ldp + r] = vr;
            P.PVt[(int64_t)r * TRD_PT + 2 * i] = vr;
        }
        pv = p * vr;
    }
    __syncthreads();
    if (lane == 0) red[wv] = pv;
    __syncthreads();
    if (t == 0) P.part2[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// the product of the trailing block (j, n) with v_j from its lower triangle
// only, for trailing blocks of at least TRD_TILE_MIN rows: one workgroup per
// TRD_TT x TRD_TT tile (rt, ct), ct <= rt, of the block (tile rows and columns
// counted from row j + 1). A tile stores the row sums of its rows (columns up
// to the diagonal) into rowp[ct], the column sums of its columns (rows below
// the diagonal) into colp[rt]; k_trd_tile_sum adds them per row in a fixed
// order. As in the row
// pass every workgroup first forms the reflector of column j; workgroup 0
// stores e[j], tau[j] and z, and the tiles of column 0 store v_j for
// their rows.
__global__ __launch_bounds__(256, 4) void k_trd_tiles(double *__restrict__ A, int64_t lda, int n, int j, int i, TrdVec V,
                                                   TrdPanel P)
{
    __shared__ double red[TRD_PS];
    __shared__ double sc[2];
    __shared__ double vr[TRD_TT], vc[TRD_TT], rsum[TRD_TT];
    __shared__ double cs[4][TRD_TT];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int b = blockIdx.x;
    int rt = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((rt + 1) * (rt + 2) / 2 <= b) ++rt;
    while (rt * (rt + 1) / 2 > b) --rt;
    const int ct = b - rt * (rt + 1) / 2;
    const int R0 = j + 1 + TRD_TT * rt, C0 = j + 1 + TRD_TT * ct;
    // the reflector of column j (as in the row pass)
    const int g1 = (n - j + TRD_CR - 1) / TRD_CR;
    const double ps = t < 2 * i + 1 ? ordered_sum(P.part1 + t, TRD_PS, 0, g1, 1) : 0.0;
    const double pz = t < 2 * i ? P.PVt[(int64_t)(j + 1) * TRD_PT + t] : 0.0;
    const double alpha = t == 0 ? V.wp[j + 1] : 0.0;
    const int e = t < TRD_TT ? R0 + t : C0 + t - TRD_TT;   // this thread's row (t < TT) or column of x
    const double xe = e < n ? V.wp[e] : 0.0;
    if (t < 2 * i + 1) red[t] = ps;
    __syncthreads();
    if (t == 0) {
        const double sig = red[0];
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (sig > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + sig), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        sc[0] = scale;
        if (b == 0) {
            V.e[j] = beta;
            V.tau[j] = tau;
        }
    }
    __syncthreads();
    const double scale = sc[0];
    const double ve = e < n ? (e == j + 1 ? 1.0 : xe * scale) : 0.0;
    if (t < TRD_TT) vr[t] = ve;
    else vc[t - TRD_TT] = ve;
    if (b == 0 && t < 2 * i) P.z[t] = pz + scale * red[t + 1];
    if (ct == 0 && t < TRD_TT && e < n) {
        A[(int64_t)e * lda + j] = ve;   // kept for the back-transformation
        P.PV[(int64_t)(2 * i) * P.ldp + e] = ve;
        P.PW[(int64_t)(2 * i + 1) * P.ldp + e] = ve;
        P.PVt[(int64_t)e * TRD_PT + 2 * i] = ve;
    }
    __syncthreads();
    // wave wv: tile rows 32 wv .. 32 wv + 31 in four groups of 8, lanes over
    // 64 columns at a time; row sums per lane, then over the lanes
    const bool diag = ct == rt;
    double colacc[2] = {0.0, 0.0};
#pragma unroll 1
    for (int g = 0; g < 4; ++g) {
        const int rl0 = 32 * wv + 8 * g;
        double racc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) racc[u] = 0.0;
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) {
            const int cl = 64 * ch + lane, c = C0 + cl;
            const double vcl = vc[cl];
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int r = R0 + rl0 + u;
                a[u] = (r < n && c < n && (!diag || cl <= rl0 + u)) ? A[(int64_t)r * lda + c] : 0.0;
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                racc[u] += a[u] * vcl;   // row part: c <= r
                colacc[ch] += ((!diag || cl < rl0 + u) ? a[u] : 0.0) * vr[rl0 + u];   // column part: r > c
            }
        }
        // the 8 row sums over the 64 lanes (halving exchanges in a fixed pattern)
        const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
        double h4[4], h2[2];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            h4[k] = (b5 ? racc[4 + k] : racc[k]) + __shfl_xor(b5 ? racc[k] : racc[4 + k], 32, 64);
#pragma unroll
        for (int k = 0; k < 2; ++k) h2[k] = (b4 ? h4[2 + k] : h4[k]) + __shfl_xor(b4 ? h4[k] : h4[2 + k], 16, 64);
        double h1 = (b3 ? h2[1] : h2[0]) + __shfl_xor(b3 ? h2[0] : h2[1], 8, 64);
        h1 += __shfl_xor(h1, 4, 64);
        h1 += __shfl_xor(h1, 2, 64);
        h1 += __shfl_xor(h1, 1, 64);
        if ((lane & 7) == 0) rsum[rl0 + 4 * b5 + 2 * b4 + (b3 ? 1 : 0)] = h1;
    }
    cs[wv][lane] = colacc[0];
    cs[wv][64 + lane] = colacc[1];
    __syncthreads();
    if (t < TRD_TT) {
        const int r = R0 + t, c = C0 + t;
        if (r < n) P.rowp[(int64_t)ct * n + r] = rsum[t];
        if (c < n) P.colp[(int64_t)rt * n + c] = cs[0][t] + cs[1][t] + cs[2][t] + cs[3][t];
    }
}

// p[r] = tau_j (A_0 v_j - sum_k (v_k (w_k . v_j) + w_k (v_k . v_j)))[r] for the
// rows r of the tiled pass of column j: eight lanes per row add its row sums
// (tile columns up to its own) and column sums (tile rows from its own down),
// lane l taking items l, l + 8, ..., then the eight lanes in a fixed pattern;
// p into V.p and this workgroup's partial sum of p . v_j into part2 (as the
// row pass leaves them)
__global__ __launch_bounds__(256) void k_trd_tile_sum(int n, int j, int i, TrdVec V, TrdPanel P)
{
    __shared__ double red[256];
    const int t = threadIdx.x, l = t & 7;
    const int r = j + 1 + (int)blockIdx.x * TRD_SR + (t >> 3);
    const int T = trd_tiles(n - j - 1);
    double s = 0.0, q = 0.0;
    if (r < n) {
        const int rt = (r - j - 1) / TRD_TT;
        // item b <= rt: rowp[b][r]; item b > rt: colp[b - 1][r]
        for (int b0 = l; b0 <= T; b0 += 32) {
            double u[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int b = b0 + 8 * k;
                u[k] = b > T ? 0.0 : (b <= rt ? P.rowp[(int64_t)b * n + r] : P.colp[(int64_t)(b - 1) * n + r]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) s += u[k];
        }
        for (int k = l; k < i; k += 8)
            q += P.PVt[(int64_t)r * TRD_PT + 2 * k] * P.z[2 * k + 1] + P.PVt[(int64_t)r * TRD_PT + 2 * k + 1] * P.z[2 * k];
    }
    for (int o = 4; o > 0; o >>= 1) {
        s += __shfl_xor(s, o, 8);
        q += __shfl_xor(q, o, 8);
    }
    double pv = 0.0;
    if (r < n && l == 0) {
        const double p = V.tau[j] * (s - q);
        V.p[r] = p;
        pv = p * P.PVt[(int64_t)r * TRD_PT + 2 * i];
    }
    pv = blk_sum(pv, red);   // (rows in order of their first lane; the others add 0)
    if (t == 0) P.part2[blockIdx.x] = pv;
}

// columns j0 .. j0 + nbp - 1 of the reduction, then the update of the
// trailing block [j0 + nbp, n)^2
hipError_t launch_trd_panel(double *A, int64_t lda, int n, int j0, int nbp, const TrdVec &V, const TrdPanel &P,
                            hipStream_t st)
{
    for (int i = 0; i < nbp; ++i) {
        const int j = j0 + i;
        hipLaunchKernelGGL(k_trd_col, dim3((n - j + TRD_CR - 1) / TRD_CR), dim3(256), 0, st, A, lda, n, j, i, 1, V,
                           P);
        if (j < n - 1) {
            const int m = n - j - 1;
            if (m >= TRD_TILE_MIN) {
                const int T = trd_tiles(m);
                hipLaunchKernelGGL(k_trd_tiles, dim3(T * (T + 1) / 2), dim3(256), 0, st, A, lda, n, j, i, V, P);
                hipLaunchKernelGGL(k_trd_tile_sum, dim3((m + TRD_SR - 1) / TRD_SR), dim3(256), 0, st, n, j, i, V, P);
            } else {
                hipLaunchKernelGGL(k_trd_pass, dim3((m + 3) / 4), dim3(256), 0, st, A, lda, n, j, i, V, P);
            }
        }
    }
    const int t = j0 + nbp;
    if (t < n) {
        // w of the panel's last reflector, then A -= PV^T PW on the trailing block
        hipLaunchKernelGGL(k_trd_col, dim3((n - t + TRD_CR - 1) / TRD_CR), dim3(256), 0, st, A, lda, n, t, nbp, 0, V,
                           P);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // while the trailing block has TRD_TILE_MIN rows or more it is read
        // only below the diagonal (tiled product, column kernel, reflectors);
        // the row pass reads whole rows of the last TRD_TILE_MIN, so the
        // square from a tile row at or before n - TRD_TILE_MIN is updated whole
        const int lowq = n - TRD_TILE_MIN - t > 0 ? (n - TRD_TILE_MIN - t) / EG_T : 0;
        return launch_eig_gemm(n - t, n - t, 2 * nbp, -1.0, P.PV + t, 1, P.ldp, P.PW + t, P.ldp, 1, 1.0,
                               A + (int64_t)t * lda + t, lda, st, nullptr, 0, lowq);
    }
    return hipGetLastError();
}

// W = (W + W^T) / 2 in place (the operation is defined on a symmetric matrix)
__global__ void k_symmetrize(double *__restrict__ W, int64_t ld, int n)
{
    const int64_t i = blockIdx.y, j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= i) return;
    const double a = 0.5 * (W[i * ld + j] + W[j * ld + i]);
    W[i * ld + j] = a;
    W[j * ld + i] = a;
}

hipError_t launch_symmetrize(double *W, int64_t ld, int n, hipStream_t st)
{
    if (n <= 1) return hipSuccess;
    hipLaunchKernelGGL(k_symmetrize, dim3((n + 255) / 256, n), dim3(256), 0, st, W, ld, n);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// 2. eigenvalues of the tridiagonal T (diagonal d[0..n), off-diagonal e[0..n-1))
// ---------------------------------------------------------------------------
// number of eigenvalues below x of the unreduced block d[0..m), e2[0..m-1)
// (Sturm sequence of the LDL^T pivots)
__device__ __forceinline__ int sturm_count(const double *__restrict__ d, const double *__restrict__ e2, int m,
                                           double x, double pivmin)
{
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
    int i = 1;
    for (; i + 8 <= m; i += 8) {   // the loads of 8 steps go out before the chain
        double dv[8], ev[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            dv[u] = d[i + u];
            ev[u] = e2[i + u - 1];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            q = dv[u] - x - ev[u] / q;
            if (fabs(q) < pivmin) q = -pivmin;
            c += q < 0.0;
        }
    }
    for (; i < m; ++i) {
        q = d[i] - x - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

// eigenvalue t: the k-th (ascending) of the block starting at row b0 with m
// rows, by multisection on [lo, hi]: the TRI_G lanes of a group evaluate the
// Sturm count at TRI_G interior points, and the interval shrinks to the piece
// between the last point with count <= k and the first with count > k, until
// no representable point lies strictly inside. With monotone counts this ends
// on the same pair of adjacent doubles as bisection, in about a third of the
// dependent steps. (8 lanes: 12.7 ms for the 8000 eigenvalues of the D =
// 8000 matrix; 16 lanes 13.6 ms, 32 lanes 19.0 ms, 64 lanes 29.5 ms: the
// counts are bound by issue, not by the length of the chain.)
constexpr int TRI_G = 8;
__global__ __launch_bounds__(256) void k_tri_bisect(const double *__restrict__ d, const double *__restrict__ e2, int n,
                                                    const int32_t *__restrict__ bs, const int32_t *__restrict__ bm,
                                                    const int32_t *__restrict__ bk, double lo0, double hi0,
                                                    double pivmin, double *__restrict__ w)
{
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = gt / TRI_G, g = gt % TRI_G;
    if (t >= n) return;   // (whole groups)
    const int b0 = bs[t], m = bm[t], k = bk[t];
    const double f = (double)(g + 1) / (double)(TRI_G + 1);
    double lo = lo0, hi = hi0;
    for (int it = 0; it < 200; ++it) {
        const double x = lo + (hi - lo) * f;
        const bool in = x > lo && x < hi;
        int any = in;
        for (int o = 1; o < TRI_G; o <<= 1) any |= __shfl_xor(any, o, TRI_G);
        if (!any) break;   // lo and hi are adjacent doubles
        const int cnt = in ? sturm_count(d + b0, e2 + b0, m, x, pivmin) : 0;
        double h = in && cnt > k ? x : hi;
        for (int o = 1; o < TRI_G; o <<= 1) h = fmin(h, __shfl_xor(h, o, TRI_G));
        double l = in && cnt <= k && x < h ? x : lo;
        for (int o = 1; o < TRI_G; o <<= 1) l = fmax(l, __shfl_xor(l, o, TRI_G));
        lo = l;
        hi = h;
    }
    if (g == 0) w[t] = 0.5 * (lo + hi);
}

__global__ void k_tri_prep(const double *__restrict__ e, int n, double *__restrict__ e2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n - 1) e2[i] = e[i] * e[i];
}

// bs/bm/bk[t]: block start, block rows and index inside the block of
// eigenvalue t (e must hold exact zeros between blocks)
hipError_t launch_tri_eigenvalues(const double *d, const double *e, double *e2, int n, const int32_t *bs,
                                  const int32_t *bm, const int32_t *bk, double lo, double hi, double pivmin,
                                  double *w, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (n > 1) hipLaunchKernelGGL(k_tri_prep, dim3((n + 255) / 256), dim3(256), 0, st, e, n, e2);
    hipLaunchKernelGGL(k_tri_bisect, dim3((unsigned)(((int64_t)n * TRI_G + 255) / 256)), dim3(256), 0, st, d, e2, n,
                       bs, bm, bk, lo, hi, pivmin, w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3. eigenvector k of T by the twisted factorisation of its block minus w_k:
//    forward L D L^T (pivots dp, multipliers l), backward U D U^T (pivots dm,
//    multipliers u), twist index r = argmin |dp_i + dm_i - (d_i - w)|, then
//    z_r = 1, z_i = -l_i z_{i+1} above r and z_{i+1} = -u_i z_i below, and
//    normalisation; rows outside the block are zero. Z[i][k] (column k):
//    consecutive threads write consecutive addresses. S is scratch of the
//    same shape (the multipliers).
// ---------------------------------------------------------------------------
__global__ void k_tri_vectors(const double *__restrict__ dg, const double *__restrict__ eg, int n,
                              const int32_t *__restrict__ bs, const int32_t *__restrict__ bm,
                              const double *__restrict__ w, double pivmin, double *__restrict__ Zg, int64_t ldz,
                              double *__restrict__ Sg, int64_t lds)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int b0 = bs[k], m = bm[k];
    const double lam = w[k];
    for (int i = 0; i < b0; ++i) Zg[(int64_t)i * ldz + k] = 0.0;
    for (int i = b0 + m; i < n; ++i) Zg[(int64_t)i * ldz + k] = 0.0;
    const double *d = dg + b0, *e = eg + b0;
    double *Z = Zg + (int64_t)b0 * ldz, *S = Sg + (int64_t)b0 * lds;
    if (m == 1) {
        Z[k] = 1.0;
        return;
    }
    // Every loop below is a dependent chain over the rows; the loads of
    // TV_B steps go out before the chain runs through them (same arithmetic
    // in the same order).
    constexpr int TV_B = 8;
    // forward: dp_i into S, l_i into Z (both column k)
    double dp = d[0] - lam;
    if (fabs(dp) < pivmin) dp = -pivmin;
    S[k] = dp;
    int i = 0;
    for (; i + TV_B <= m - 1; i += TV_B) {
        double dv[TV_B], ev[TV_B];
#pragma unroll
        for (int u = 0; u < TV_B; ++u) {
            dv[u] = d[i + u + 1];
            ev[u] = e[i + u];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < TV_B; ++u) {
            const double l = ev[u] / dp;
            Z[(int64_t)(i + u) * ldz + k] = l;
            dp = dv[u] - lam - l * ev[u];
            if (fabs(dp) < pivmin) dp = -pivmin;
            S[(int64_t)(i + u + 1) * lds + k] = dp;
        }
    }
    for (; i < m - 1; ++i) {
        const double l = e[i] / dp;
        Z[(int64_t)i * ldz + k] = l;
        dp = d[i + 1] - lam - l * e[i];
        if (fabs(dp) < pivmin) dp = -pivmin;
        S[(int64_t)(i + 1) * lds + k] = dp;
    }
    // backward: dm_i, twist index
    double dm = d[m - 1] - lam;
    if (fabs(dm) < pivmin) dm = -pivmin;
    int r = m - 1;
    double best = fabs(S[(int64_t)(m - 1) * lds + k] + dm - (d[m - 1] - lam));
    i = m - 2;
    for (; i - (TV_B - 1) >= 0; i -= TV_B) {
        double dv[TV_B], ev[TV_B], sv[TV_B];
#pragma unroll
        for (int u = 0; u < TV_B; ++u) {
            dv[u] = d[i - u];
            ev[u] = e[i - u];
            sv[u] = S[(int64_t)(i - u) * lds + k];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < TV_B; ++u) {
            const double uu = ev[u] / dm;
            dm = dv[u] - lam - uu * ev[u];
            if (fabs(dm) < pivmin) dm = -pivmin;
            const double g = fabs(sv[u] + dm - (dv[u] - lam));
            if (g < best) {
                best = g;
                r = i - u;
            }
        }
    }
    for (; i >= 0; --i) {
        const double u = e[i] / dm;
        dm = d[i] - lam - u * e[i];
        if (fabs(dm) < pivmin) dm = -pivmin;
        const double g = fabs(S[(int64_t)i * lds + k] + dm - (d[i] - lam));
        if (g < best) {
            best = g;
            r = i;
        }
    }
    // u_i for i >= r again (backward from the end), into S rows i >= r
    dm = d[m - 1] - lam;
    if (fabs(dm) < pivmin) dm = -pivmin;
    i = m - 2;
    for (; i - (TV_B - 1) >= r; i -= TV_B) {
        double dv[TV_B], ev[TV_B];
#pragma unroll
        for (int u = 0; u < TV_B; ++u) {
            dv[u] = d[i - u];
            ev[u] = e[i - u];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < TV_B; ++u) {
            const double uu = ev[u] / dm;
            S[(int64_t)(i - u) * lds + k] = uu;
            dm = dv[u] - lam - uu * ev[u];
            if (fabs(dm) < pivmin) dm = -pivmin;
        }
    }
    for (; i >= r; --i) {
        const double u = e[i] / dm;
        S[(int64_t)i * lds + k] = u;
        dm = d[i] - lam - u * e[i];
        if (fabs(dm) < pivmin) dm = -pivmin;
    }
    // the vector (z_r = 1), its norm
    double nrm = 1.0, z = 1.0;
    i = r - 1;
    for (; i - (TV_B - 1) >= 0; i -= TV_B) {
        double lv[TV_B];
#pragma unroll
        for (int u = 0; u < TV_B; ++u) lv[u] = Z[(int64_t)(i - u) * ldz + k];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < TV_B; ++u) {
            z = -lv[u] * z;
            Z[(int64_t)(i - u) * ldz + k] = z;
            nrm += z * z;
        }
    }
    for (; i >= 0; --i) {
        z = -Z[(int64_t)i * ldz + k] * z;
        Z[(int64_t)i * ldz + k] = z;
        nrm += z * z;
    }
    Z[(int64_t)r * ldz + k] = 1.0;
    z = 1.0;
    i = r;
    for (; i + TV_B <= m - 1; i += TV_B) {
        double uv[TV_B];
#pragma unroll
        for (int u = 0; u < TV_B; ++u) uv[u] = S[(int64_t)(i + u) * lds + k];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < TV_B; ++u) {
            z = -uv[u] * z;
            Z[(int64_t)(i + u + 1) * ldz + k] = z;
            nrm += z * z;
        }
    }
    for (; i < m - 1; ++i) {
        z = -S[(int64_t)i * lds + k] * z;
        Z[(int64_t)(i + 1) * ldz + k] = z;
        nrm += z * z;
    }
    const double inv = 1.0 / sqrt(nrm);
    i = 0;
    for (; i + TV_B <= m; i += TV_B) {
        double zv[TV_B];
#pragma unroll
        for (int u = 0; u < TV_B; ++u) zv[u] = Z[(int64_t)(i + u) * ldz + k];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < TV_B; ++u) Z[(int64_t)(i + u) * ldz + k] = zv[u] * inv;
    }
    for (; i < m; ++i) Z[(int64_t)i * ldz + k] *= inv;
}

hipError_t launch_tri_vectors(const double *d, const double *e, int n, const int32_t *bs, const int32_t *bm,
                              const double *w, double pivmin, double *Z, int64_t ldz, double *S, int64_t lds,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tri_vectors, dim3((n + 63) / 64), dim3(64), 0, st, d, e, n, bs, bm, w, pivmin, Z, ldz, S,
                       lds);
    return hipGetLastError();
}

// modified Gram-Schmidt over the columns cols[0..nc) of Z (one cluster of
// close eigenvalues inside the unreduced block of rows [b0, b0 + m)), in
// order, each column projected twice. A column that keeps less than half of
// its norm after the projection has collapsed towards the ones before it
// (twisted vectors of nearly equal eigenvalues can come out nearly
// parallel): it is refined by two steps of inverse iteration with its own
// eigenvalue, each followed by the projection, from what is left of it, or
// from a fixed spread vector when almost nothing is left. The solve is
// (T_b - lambda I) y = x by the LDL^T recurrence with pivots floored at
// piv (one thread; rare path), the product kept in Z, the pivots in column c
// of S.
__device__ __forceinline__ double mgs_project(double *Z, int64_t ldz, int b0, int m, const int32_t *cols, int a,
                                              int c, double *red)
{
    const int t = threadIdx.x;
    for (int pass = 0; pass < 2; ++pass)
        for (int q = 0; q < a; ++q) {
            const int cq = cols[q];
            double s = 0.0;
            for (int i = b0 + t; i < b0 + m; i += 256) s += Z[(int64_t)i * ldz + cq] * Z[(int64_t)i * ldz + c];
            const double dot = blk_sum(s, red);
            for (int i = b0 + t; i < b0 + m; i += 256) Z[(int64_t)i * ldz + c] -= dot * Z[(int64_t)i * ldz + cq];
            __syncthreads();
        }
    double s = 0.0;
    for (int i = b0 + t; i < b0 + m; i += 256) s += Z[(int64_t)i * ldz + c] * Z[(int64_t)i * ldz + c];
    return blk_sum(s, red);
}

__device__ __forceinline__ void mgs_scale(double *Z, int64_t ldz, int b0, int m, int c, double nrm2)
{
    const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
    for (int i = b0 + threadIdx.x; i < b0 + m; i += 256) Z[(int64_t)i * ldz + c] *= inv;
    __syncthreads();
}

// one workgroup per cluster; cluster b is desc[4b .. 4b + 3] = (offset of its
// columns in cols_all, number of columns, block start, block rows). The
// clusters have disjoint columns (of Z and of S) and run concurrently.
__global__ __launch_bounds__(256) void k_cluster_mgs(double *__restrict__ Z, int64_t ldz,
                                                     const int32_t *__restrict__ desc,
                                                     const int32_t *__restrict__ cols_all,
                                                     const double *__restrict__ dg, const double *__restrict__ eg,
                                                     const double *__restrict__ w, double *__restrict__ S,
                                                     int64_t lds, double piv)
{
    __shared__ double red[4];
    const int t = threadIdx.x;
    const int32_t *dsc = desc + 4 * (int64_t)blockIdx.x;
    const int32_t *cols = cols_all + dsc[0];
    const int nc = dsc[1], b0 = dsc[2], m = dsc[3];
    for (int a = 0; a < nc; ++a) {
        const int c = cols[a];
        double nrm2 = mgs_project(Z, ldz, b0, m, cols, a, c, red);
        if (a > 0 && nrm2 < 0.25) {
            if (nrm2 <= 1e-6) {
                for (int i = b0 + t; i < b0 + m; i += 256)
                    Z[(int64_t)i * ldz + c] = sin(1.0 + 0.7 * (double)(i - b0) + 1.3 * (double)a);
                __syncthreads();
                nrm2 = mgs_project(Z, ldz, b0, m, cols, a, c, red);
            }
            for (int it = 0; it < 2; ++it) {
                mgs_scale(Z, ldz, b0, m, c, nrm2);
                if (t == 0) {
                    const double lam = w[c];
                    const double *d = dg + b0, *e = eg + b0;
                    double *z = Z + (int64_t)b0 * ldz + c, *dp = S + (int64_t)b0 * lds + c;
                    // forward: L z' = z and the pivots
                    double p = d[0] - lam;
                    if (fabs(p) < piv) p = p < 0.0 ? -piv : piv;
                    dp[0] = p;
                    for (int i = 1; i < m; ++i) {
                        const double l = e[i - 1] / p;
                        z[(int64_t)i * ldz] -= l * z[(int64_t)(i - 1) * ldz];
                        p = d[i] - lam - l * e[i - 1];
                        if (fabs(p) < piv) p = p < 0.0 ? -piv : piv;
                        dp[(int64_t)i * lds] = p;
                    }
                    // backward: D L^T y = z'
                    double y = z[(int64_t)(m - 1) * ldz] / dp[(int64_t)(m - 1) * lds];
                    z[(int64_t)(m - 1) * ldz] = y;
                    for (int i = m - 2; i >= 0; --i) {
                        const double q = dp[(int64_t)i * lds];
                        y = z[(int64_t)i * ldz] / q - (e[i] / q) * y;
                        z[(int64_t)i * ldz] = y;
                    }
                }
                __syncthreads();
                nrm2 = mgs_project(Z, ldz, b0, m, cols, a, c, red);
            }
        }
        mgs_scale(Z, ldz, b0, m, c, nrm2);
    }
}

hipError_t launch_cluster_mgs(double *Z, int64_t ldz, const int32_t *desc, int ncl, const int32_t *cols,
                              const double *d, const double *e, const double *w, double *S, int64_t lds, double piv,
                              hipStream_t st)
{
    if (ncl <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cluster_mgs, dim3(ncl), dim3(256), 0, st, Z, ldz, desc, cols, d, e, w, S, lds, piv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 4. back-transformation helpers
// ---------------------------------------------------------------------------
// Vb[r][i] = v_{j0+i}[j0+1+r] (zero above the reflector's first row), rows
// r < m = n - j0 - 1, i < nb
__global__ void k_copy_reflectors(const double *__restrict__ A, int64_t lda, int n, int j0, int nb,
                                  double *__restrict__ Vb)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = n - j0 - 1;
    if (r >= m) return;
    const int row = j0 + 1 + r;
    for (int i = 0; i < nb; ++i) {
        const int j = j0 + i;   // reflector j starts at row j + 1
        Vb[(int64_t)r * nb + i] = (row >= j + 1) ? A[(int64_t)row * lda + j] : 0.0;
    }
}

hipError_t launch_copy_reflectors(const double *A, int64_t lda, int n, int j0, int nb, double *Vb, hipStream_t st)
{
    const int m = n - j0 - 1;
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_reflectors, dim3((m + 255) / 256), dim3(256), 0, st, A, lda, n, j0, nb, Vb);
    return hipGetLastError();
}

// T (nb x nb, upper triangular) of the compact WY form from the Gram matrix
// G = Vb^T Vb and the scalars tau: T[i][i] = tau_i,
// T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]. One workgroup, all in LDS: the
// four diagonal blocks of 16 by that column recurrence side by side (one
// wave each; thread r forms entry r, its sum in order), then neighbouring
// blocks joined, 16 -> 32 -> 64, by T12 = -T11 G12 T22 (the same T: the
// product of the first reflectors times that of the next ones)
constexpr int LARFT_MAX = 64;
__global__ __launch_bounds__(256) void k_larft(const double *__restrict__ G, int ldg, const double *__restrict__ tau,
                                               int nb, double *__restrict__ T, int ldt)
{
    __shared__ double Ts[LARFT_MAX][LARFT_MAX + 1];
    __shared__ double Gs[LARFT_MAX][LARFT_MAX + 1];
    __shared__ double Ws[LARFT_MAX / 2][LARFT_MAX / 2 + 1];
    __shared__ double ts[LARFT_MAX];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int e = t; e < LARFT_MAX * LARFT_MAX; e += 256) Ts[e / LARFT_MAX][e % LARFT_MAX] = 0.0;
#pragma unroll 4
    for (int e = t; e < nb * nb; e += 256) Gs[e / nb][e % nb] = G[(int64_t)(e / nb) * ldg + e % nb];
    if (t < nb) ts[t] = tau[t];
    __syncthreads();
    // the diagonal blocks [16 wv, 16 wv + 16)
    const int b0 = 16 * wv, bl = max(0, min(16, nb - b0));
    for (int i = 0; i < 16; ++i) {
        if (i < bl) {
            const int c = b0 + i;
            if (lane < i) {
                double acc = 0.0;
                for (int q = lane; q < i; ++q) acc += Ts[b0 + lane][b0 + q] * Gs[b0 + q][c];
                Ts[b0 + lane][c] = -ts[c] * acc;
            } else if (lane == i) {
                Ts[c][c] = ts[c];
            }
        }
        __syncthreads();
    }
    // joins: rows [a0, a0 + h) (T11) with columns [c0, c0 + h2) (T22), c0 = a0 + h
    for (int h = 16; h < nb; h *= 2) {
        const int np = (nb + 2 * h - 1) / (2 * h);
        // W = G12 T22 (h x h2 per pair; T22 upper triangular)
        for (int p = 0; p < np; ++p) {
            const int a0 = 2 * h * p, c0 = a0 + h;
            if (c0 >= nb) break;
            const int h2 = min(h, nb - c0);
            for (int e = t; e < h * h2; e += 256) {
                const int r = e / h2, cc = e % h2;
                double acc = 0.0;
                for (int q = 0; q <= cc; ++q) acc += Gs[a0 + r][c0 + q] * Ts[c0 + q][c0 + cc];
                Ws[r][cc] = acc;
            }
            __syncthreads();
            // T12 = -T11 W (T11 upper triangular)
            for (int e = t; e < h * h2; e += 256) {
                const int r = e / h2, cc = e % h2;
                double acc = 0.0;
                for (int q = r; q < h; ++q) acc += Ts[a0 + r][a0 + q] * Ws[q][cc];
                Ts[a0 + r][c0 + cc] = -acc;
            }
            __syncthreads();
        }
    }
    for (int e = t; e < nb * nb; e += 256) T[(int64_t)(e / nb) * ldt + e % nb] = Ts[e / nb][e % nb];
}

// T (nb x nb, row-major) for nb <= 2 LARFT_MAX: up to LARFT_MAX in one
// workgroup; above, the two diagonal blocks of LARFT_MAX and n2 = nb -
// LARFT_MAX reflectors, joined by T12 = -T1 (G12 T2) (two FP64 MFMA
// products; X: LARFT_MAX x n2 doubles of scratch)
hipError_t launch_larft(const double *G, const double *tau, int nb, double *T, double *X, hipStream_t st)
{
    if (nb > 2 * LARFT_MAX) return hipErrorInvalidValue;
    if (nb <= LARFT_MAX) {
        hipLaunchKernelGGL(k_larft, dim3(1), dim3(256), 0, st, G, nb, tau, nb, T, nb);
        return hipGetLastError();
    }
    const int h = LARFT_MAX, n2 = nb - h;
    hipError_t e = launch_fill_f64(T, 0.0, (int64_t)nb * nb, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_larft, dim3(1), dim3(256), 0, st, G, nb, tau, h, T, nb);
    hipLaunchKernelGGL(k_larft, dim3(1), dim3(256), 0, st, G + (int64_t)h * nb + h, nb, tau + h, n2,
                       T + (int64_t)h * nb + h, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // X = G12 T2, then T12 = -T1 X
    if ((e = launch_eig_gemm(h, n2, n2, 1.0, G + h, nb, 1, T + (int64_t)h * nb + h, nb, 1, 0.0, X, n2, st, nullptr,
                             0, -1)) != hipSuccess)
        return e;
    return launch_eig_gemm(h, n2, h, -1.0, T, nb, 1, X, n2, 1, 0.0, T + h, nb, st, nullptr, 0, -1);
}

// out[k][i] = Z[i][k]
__global__ __launch_bounds__(256) void k_transpose_sq(const double *__restrict__ Z, int64_t ldz, int n,
                                                      double *__restrict__ out, int64_t ldo)
{
    __shared__ double tl[32][33];
    const int i0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int a = ty; a < 32; a += 8) {
        const int i = i0 + a, k = k0 + tx;
        tl[a][tx] = (i < n && k < n) ? Z[(int64_t)i * ldz + k] : 0.0;
    }
    __syncthreads();
    for (int a = ty; a < 32; a += 8) {
        const int k = k0 + a, i = i0 + tx;
        if (k < n && i < n) out[(int64_t)k * ldo + i] = tl[tx][a];
    }
}

hipError_t launch_transpose_sq(const double *Z, int64_t ldz, int n, double *out, int64_t ldo, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose_sq, dim3((n + 31) / 32, (n + 31) / 32), dim3(256), 0, st, Z, ldz, n, out, ldo);
    return hipGetLastError();
}

}  // namespace cch
