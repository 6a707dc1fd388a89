// Every eigenpair of a dense real symmetric matrix in FP64 on one GPU (the
// paper's Sec. 3.2 notes that often all eigenvectors are wanted and a dense
// diagonaliser is used then):
//   1. Householder tridiagonalisation Q^T A Q = T, one reflector per column.
//      Each column takes two launches: a one-workgroup step that applies the
//      previous reflector to the new column, finishes the previous w vector
//      and forms the new reflector; and a pass over the trailing block that
//      applies the previous rank-2 update to every row and, from the updated
//      row, forms the product with the new reflector (one read and one write
//      of the trailing block per column, the HBM-bound part).
//   2. Eigenvalues of T by bisection on Sturm counts, one thread each.
//   3. Eigenvectors of T by twisted factorisations, one thread each, with
//      modified Gram-Schmidt inside clusters of close eigenvalues.
//   4. Back-transformation Z = Q Z_T in blocks of 64 reflectors, each as
//      I - V T V^T (compact WY) by three FP64 MFMA products.
#include <algorithm>
#include <cmath>

#include "ccham_internal.h"

namespace cch {

typedef double ex4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// general FP64 MFMA product C = alpha A B + beta C (row-major C)
//   A(i, k) = A[i * sai + k * sak], B(k, j) = B[k * sbk + j * sbj]
// 64 x 64 tile per workgroup (4 waves of 32 x 32), K staged through LDS in
// slices of 16; loads follow whichever index of an operand has stride 1
// ---------------------------------------------------------------------------
constexpr int EG_T = 64, EG_K = 16;

// With P != nullptr the K range is split over blockIdx.z (kc each) and each
// split writes its unscaled partial product to P[z][M][N]; k_eig_gemm_sum adds
// the splits in order and applies alpha and beta (deterministic).
__global__ __launch_bounds__(256) void k_eig_gemm(int M, int N, int K, double alpha, const double *__restrict__ A,
                                                  int64_t sai, int64_t sak, const double *__restrict__ B, int64_t sbk,
                                                  int64_t sbj, double beta, double *__restrict__ C, int64_t ldc,
                                                  int kc, double *__restrict__ P)
{
    __shared__ double As[EG_K][EG_T + 1], Bs[EG_K][EG_T + 1];
    const int i0 = blockIdx.y * EG_T, j0 = blockIdx.x * EG_T;
    const int kb0 = P ? (int)blockIdx.z * kc : 0, kb1 = P ? min(K, kb0 + kc) : K;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    const bool a_kfast = sak == 1, b_jfast = sbj == 1;
    ex4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (ex4){0.0, 0.0, 0.0, 0.0};
    for (int k0 = kb0; k0 < kb1; k0 += EG_K) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int ii, kk;
            if (a_kfast) { kk = t & 15; ii = (t >> 4) + 16 * u; }
            else { ii = t & 63; kk = (t >> 6) + 4 * u; }
            const int i = i0 + ii, k = k0 + kk;
            As[kk][ii] = (i < M && k < kb1) ? A[(int64_t)i * sai + (int64_t)k * sak] : 0.0;
            int jj, kb;
            if (b_jfast) { jj = t & 63; kb = (t >> 6) + 4 * u; }
            else { kb = t & 15; jj = (t >> 4) + 16 * u; }
            const int j = j0 + jj, kq = k0 + kb;
            Bs[kb][jj] = (j < N && kq < kb1) ? B[(int64_t)kq * sbk + (int64_t)j * sbj] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < EG_K; ks += 4) {
            const int kk = ks + (lane >> 4);
            double af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = As[kk][wm * 32 + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bf[b] = Bs[kk][wn * 32 + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + wm * 32 + a * 16 + (lane >> 4) + 4 * v;
            if (i >= M) continue;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int j = j0 + wn * 32 + b * 16 + (lane & 15);
                if (j >= N) continue;
                if (P) {
                    P[((int64_t)blockIdx.z * M + i) * N + j] = acc[a][b][v];
                } else {
                    double *c = C + (int64_t)i * ldc + j;
                    *c = alpha * acc[a][b][v] + (beta == 0.0 ? 0.0 : beta * *c);
                }
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
                           hipStream_t st, double *P, int64_t p_cap)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    const dim3 g((N + EG_T - 1) / EG_T, (M + EG_T - 1) / EG_T);
    const int64_t tiles = (int64_t)g.x * g.y;
    int ns = 1;
    if (P && tiles < 512 && K >= 1024) {
        ns = (int)std::min<int64_t>({(K + 255) / 256, std::max<int64_t>(1, 1024 / tiles), 64});
        ns = (int)std::min<int64_t>(ns, p_cap / ((int64_t)M * N));
    }
    if (ns <= 1) {
        hipLaunchKernelGGL(k_eig_gemm, g, dim3(256), 0, st, M, N, K, alpha, A, sai, sak, B, sbk, sbj, beta, C, ldc,
                           K, (double *)nullptr);
        return hipGetLastError();
    }
    const int kc = ((K + ns - 1) / ns + EG_K - 1) / EG_K * EG_K;
    ns = (K + kc - 1) / kc;
    hipLaunchKernelGGL(k_eig_gemm, dim3(g.x, g.y, ns), dim3(256), 0, st, M, N, K, alpha, A, sai, sak, B, sbk, sbj,
                       beta, C, ldc, kc, P);
    const int64_t e = (int64_t)M * N;
    hipLaunchKernelGGL(k_eig_gemm_sum, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, M, N, ns, P, alpha, beta,
                       C, ldc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 1. tridiagonalisation (lower triangle convention: reflector j annihilates
//    A[j+2:, j]; v_j[j+1] = 1 is stored explicitly in A[j+1][j] and below)
// work vectors (length n each): vp = v_{j-1}, wp = w_{j-1}, vn = v_j, p = A v_j
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

// one workgroup: column j of A (rows j..n-1) after reflector j-1, its
// reflector, and w_{j-1} = p - (tau/2)(p^T v) v from the product of the last
// pass; j = 0: no previous reflector
__global__ __launch_bounds__(256) void k_trd_col(double *__restrict__ A, int64_t lda, int n, int j, TrdVec V)
{
    __shared__ double red[4];
    const int t = threadIdx.x;
    if (j > 0) {
        // w_{j-1} over rows j..n-1 (v_{j-1} is zero above row j)
        const double tau = V.tau[j - 1];
        double s = 0.0;
        for (int r = j + t; r < n; r += 256) s += V.p[r] * V.vn[r];
        const double pv = blk_sum(s, red);
        const double al = -0.5 * tau * pv;
        for (int r = j + t; r < n; r += 256) {
            const double v = V.vn[r];
            V.vp[r] = v;
            V.wp[r] = V.p[r] + al * v;
        }
        __syncthreads();
        // column j (rows j..n-1) minus v w^T + w v^T at column j
        const double vj = V.vp[j], wj = V.wp[j];
        for (int r = j + t; r < n; r += 256) {
            double *a = A + (int64_t)r * lda + j;
            *a = *a - V.vp[r] * wj - V.wp[r] * vj;
        }
        __syncthreads();
    }
    if (t == 0) V.d[j] = A[(int64_t)j * lda + j];
    if (j >= n - 1) return;
    // reflector on x = A[j+1:, j]
    const double alpha = A[(int64_t)(j + 1) * lda + j];
    double s = 0.0;
    for (int r = j + 2 + t; r < n; r += 256) {
        const double x = A[(int64_t)r * lda + j];
        s += x * x;
    }
    const double sig = blk_sum(s, red);
    double tau = 0.0, beta = alpha, scale = 0.0;
    if (sig > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + sig), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
    }
    for (int r = t; r < n; r += 256) {
        double v = 0.0;
        if (r == j + 1) v = 1.0;
        else if (r > j + 1) v = A[(int64_t)r * lda + j] * scale;
        V.vn[r] = v;
        if (r > j) A[(int64_t)r * lda + j] = v;   // kept for the back-transformation
    }
    if (t == 0) {
        V.e[j] = beta;
        V.tau[j] = tau;
    }
}

// rows r of the trailing block [j+1, n) x [j+1, n): apply reflector j-1's
// rank-2 update (when j > 0), then p[r] = tau_j * sum_c A[r][c] v_j[c].
// One wave per row, lanes over the columns, a fixed-order reduction.
__global__ __launch_bounds__(256) void k_trd_pass(double *__restrict__ A, int64_t lda, int n, int j, int upd,
                                                  TrdVec V)
{
    const int lane = threadIdx.x & 63;
    const int r = j + 1 + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;   // the whole wave
    double *row = A + (int64_t)r * lda;
    const double vr = upd ? V.vp[r] : 0.0, wr = upd ? V.wp[r] : 0.0;
    double s = 0.0;
    for (int c = j + 1 + lane; c < n; c += 64) {
        double a = row[c];
        if (upd) {
            a = a - vr * V.wp[c] - wr * V.vp[c];
            row[c] = a;
        }
        s += a * V.vn[c];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) V.p[r] = V.tau[j] * s;
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

hipError_t launch_trd_step(double *A, int64_t lda, int n, int j, const TrdVec &V, hipStream_t st)
{
    hipLaunchKernelGGL(k_trd_col, dim3(1), dim3(256), 0, st, A, lda, n, j, V);
    if (j < n - 1) {
        const int rows = n - j - 1;
        hipLaunchKernelGGL(k_trd_pass, dim3((rows + 3) / 4), dim3(256), 0, st, A, lda, n, j, j > 0 ? 1 : 0, V);
    }
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
    for (int i = 1; i < m; ++i) {
        q = d[i] - x - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

// eigenvalue t: the k-th (ascending) of the block starting at row b0 with m
// rows, by bisection on [lo, hi] to the last bits
__global__ void k_tri_bisect(const double *__restrict__ d, const double *__restrict__ e2, int n,
                             const int32_t *__restrict__ bs, const int32_t *__restrict__ bm,
                             const int32_t *__restrict__ bk, double lo0, double hi0, double pivmin,
                             double *__restrict__ w)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int b0 = bs[t], m = bm[t], k = bk[t];
    double lo = lo0, hi = hi0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;   // the interval is two adjacent doubles
        if (sturm_count(d + b0, e2 + b0, m, mid, pivmin) > k) hi = mid;
        else lo = mid;
    }
    w[t] = 0.5 * (lo + hi);
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
    hipLaunchKernelGGL(k_tri_bisect, dim3((n + 63) / 64), dim3(64), 0, st, d, e2, n, bs, bm, bk, lo, hi, pivmin, w);
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
    // forward: dp_i into S, l_i into Z (both column k)
    double dp = d[0] - lam;
    if (fabs(dp) < pivmin) dp = -pivmin;
    S[k] = dp;
    for (int i = 0; i < m - 1; ++i) {
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
    for (int i = m - 2; i >= 0; --i) {
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
    for (int i = m - 2; i >= r; --i) {
        const double u = e[i] / dm;
        S[(int64_t)i * lds + k] = u;
        dm = d[i] - lam - u * e[i];
        if (fabs(dm) < pivmin) dm = -pivmin;
    }
    // the vector (z_r = 1), its norm
    double nrm = 1.0, z = 1.0;
    for (int i = r - 1; i >= 0; --i) {
        z = -Z[(int64_t)i * ldz + k] * z;
        Z[(int64_t)i * ldz + k] = z;
        nrm += z * z;
    }
    Z[(int64_t)r * ldz + k] = 1.0;
    z = 1.0;
    for (int i = r; i < m - 1; ++i) {
        z = -S[(int64_t)i * lds + k] * z;
        Z[(int64_t)(i + 1) * ldz + k] = z;
        nrm += z * z;
    }
    const double inv = 1.0 / sqrt(nrm);
    for (int i = 0; i < m; ++i) Z[(int64_t)i * ldz + k] *= inv;
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
// order. A column that loses almost all of its norm to the ones before it
// (nearly parallel twisted vectors) is replaced by a fixed spread vector on
// the block's rows and orthogonalised again.
__global__ __launch_bounds__(256) void k_cluster_mgs(double *__restrict__ Z, int64_t ldz, int b0, int m,
                                                     const int32_t *__restrict__ cols, int nc)
{
    __shared__ double red[4];
    const int t = threadIdx.x;
    for (int a = 0; a < nc; ++a) {
        const int c = cols[a];
        for (int pass = 0; pass < 2; ++pass) {
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
            const double nrm2 = blk_sum(s, red);
            if (nrm2 > 1e-6 || pass == 1) {
                const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
                for (int i = b0 + t; i < b0 + m; i += 256) Z[(int64_t)i * ldz + c] *= inv;
                __syncthreads();
                break;
            }
            // nearly inside the span of the earlier columns: restart from a spread vector
            for (int i = b0 + t; i < b0 + m; i += 256)
                Z[(int64_t)i * ldz + c] = sin(1.0 + 0.7 * (double)(i - b0) + 1.3 * (double)a);
            __syncthreads();
        }
    }
}

hipError_t launch_cluster_mgs(double *Z, int64_t ldz, int b0, int m, const int32_t *cols, int nc, hipStream_t st)
{
    if (nc < 2) return hipSuccess;
    hipLaunchKernelGGL(k_cluster_mgs, dim3(1), dim3(256), 0, st, Z, ldz, b0, m, cols, nc);
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
// T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]
// one workgroup, T built in LDS column by column (thread r forms entry r of
// column i; the sum over q runs in order)
constexpr int LARFT_MAX = 64;
__global__ __launch_bounds__(64) void k_larft(const double *__restrict__ G, const double *__restrict__ tau, int nb,
                                              double *__restrict__ T)
{
    __shared__ double Ts[LARFT_MAX][LARFT_MAX + 1];
    const int r = threadIdx.x;
    for (int c = 0; c < nb; ++c) Ts[r][c] = 0.0;
    __syncthreads();
    for (int i = 0; i < nb; ++i) {
        const double ti = tau[i];
        if (r < i) {
            double s = 0.0;
            for (int q = r; q < i; ++q) s += Ts[r][q] * G[q * nb + i];
            Ts[r][i] = -ti * s;
        } else if (r == i) {
            Ts[r][i] = ti;
        }
        __syncthreads();
    }
    if (r < nb)
        for (int c = 0; c < nb; ++c) T[r * nb + c] = Ts[r][c];
}

hipError_t launch_larft(const double *G, const double *tau, int nb, double *T, hipStream_t st)
{
    if (nb > LARFT_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_larft, dim3(1), dim3(64), 0, st, G, tau, nb, T);
    return hipGetLastError();
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
