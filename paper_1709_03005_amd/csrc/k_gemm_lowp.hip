// Reduced-precision forms of the expansion product (the CI-contraction GEMM
// of the continuum classes, Eq. 8 followed by the (j, j') expansion):
//
//   FP32:        operands rounded to FP32, v_mfma_f32_16x16x4f32, FP32
//                accumulation over K chunks of 256, chunk results summed in
//                FP64.
//   split-BF16:  error-free slicing after Ozaki, Ogita, Oishi and Rump
//                (Numer. Algorithms, 2012): every row r of A and column c of
//                B is scaled by a power of two sigma so its entries lie in
//                [-1, 1], then cut into s slices of 8 bits, each an integer
//                in [-256, 256] (exact in BF16). A slice product summed over
//                256 consecutive k stays below 2^24 in magnitude, so the
//                v_mfma_f32_16x16x32_bf16 result of a chunk is exact; chunk
//                results are scaled by 2^-8(t+u) and summed in FP64, keeping
//                the slice pairs with t + u <= s + 1.
//
// Both share the epilogue of the FP64 kernel (delta_jj' H_T and O h_jj'
// terms, scatter into the lower triangle). MFMA f32/bf16 16x16 results:
// item v of lane l is D[4*(l/16) + v][l%16] (checked on gfx950).
#include "ccham_internal.h"

namespace cch {

struct ExpandEpi {
    double *H;
    int64_t ld;
    int64_t row0a, row0b;
    int nca, ncb;
    int ja0, jb0;
    const int32_t *rn, *rn2;
    const double *HT, *O;
    const double *h;
    int n_o, n_orb;
};

typedef float fx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int LBM = 64, LBN = 128;
constexpr int KCHUNK = 256;          // exact FP32 window for 8-bit slice products

__device__ __forceinline__ int xcd_remap_l(int b, int nb)
{
    const int per = nb / 8;
    if (b >= per * 8) return b;
    return (b % 8) * per + b / 8;
}

__device__ __forceinline__ void epilogue_store(const ExpandEpi &ep, int r, int c, int nrows, int N, double acc)
{
    if (r >= nrows || c >= N) return;
    const int n = ep.rn[r], n2 = ep.rn2[r];
    const int jj = c / ep.ncb, jp = c - jj * ep.ncb;
    const int64_t R = ep.row0a + (int64_t)n * ep.nca + jj;
    const int64_t C = ep.row0b + (int64_t)n2 * ep.ncb + jp;
    if (R < C) return;
    const int J = ep.ja0 + jj, Jp = ep.jb0 + jp;
    double val = acc;
    if (J == Jp) val += ep.HT[r];
    val += ep.O[r] * ep.h[(size_t)(ep.n_o + J) * ep.n_orb + (ep.n_o + Jp)];
    ep.H[R * ep.ld + C] = val;
}

// ---------------------------------------------------------------------------
// FP32 conversion of the K-major A and row-major B
// ---------------------------------------------------------------------------
__global__ void k_to_f32(const double *__restrict__ x, float *__restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

hipError_t launch_to_f32(const double *x, float *y, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, n);
    return hipGetLastError();
}

// C = A B: A K-major (At[k][r]) and B row-major, FP32 MFMA 16x16x4
__global__ __launch_bounds__(256) void k_expand_f32(const float *__restrict__ At, const float *__restrict__ B,
                                                    int nrows, int N, int K, ExpandEpi ep)
{
    constexpr int BK = 16;
    __shared__ float As[BK][LBM];
    __shared__ float Bs[BK][LBN];
    const int tiles_m = (nrows + LBM - 1) / LBM, tiles_n = (N + LBN - 1) / LBN;
    const int lb = xcd_remap_l(blockIdx.x, tiles_m * tiles_n);
    const int r0 = (lb % tiles_m) * LBM, c0 = (lb / tiles_m) * LBN;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    fx4 acc[2][4];
    double acc64[2][4][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[a][b] = (fx4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[a][b][v] = 0.0;
        }
    for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q, kk = e / LBM, rr = e % LBM;
            const int k = k0 + kk, r = r0 + rr;
            As[kk][rr] = (k < K && r < nrows) ? At[(size_t)k * nrows + r] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = threadIdx.x + 256 * q, kk = e / LBN, cc = e % LBN;
            const int k = k0 + kk, c = c0 + cc;
            Bs[kk][cc] = (k < K && c < N) ? B[(size_t)k * N + c] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            const int kk = ks + (lane >> 4);
            float af[2], bf[4];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = As[kk][wm * 32 + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 4; ++b) bf[b] = Bs[kk][wn * 64 + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        if (((k0 + BK) % KCHUNK) == 0 || k0 + BK >= K) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc64[a][b][v] += (double)acc[a][b][v];
                    acc[a][b] = (fx4){0.f, 0.f, 0.f, 0.f};
                }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + wm * 32 + a * 16 + 4 * (lane >> 4) + v;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = c0 + wn * 64 + b * 16 + (lane & 15);
                epilogue_store(ep, r, c, nrows, N, acc64[a][b][v]);
            }
        }
}

hipError_t launch_expand_f32(const float *At, const float *B, int nrows, int N, int K, const ExpandEpi &ep,
                             hipStream_t st)
{
    if (nrows <= 0 || N <= 0) return hipSuccess;
    const int tiles = ((nrows + LBM - 1) / LBM) * ((N + LBN - 1) / LBN);
    hipLaunchKernelGGL(k_expand_f32, dim3(tiles), dim3(256), 0, st, At, B, nrows, N, K, ep);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// split-BF16 slicing
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pow2_ceil(double m)
{
    // smallest power of two >= m (m > 0), 1 for m == 0
    if (!(m > 0.0)) return 1.0;
    int e;
    const double f = frexp(m, &e);   // m = f 2^e, f in [0.5, 1)
    return f == 0.5 ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

// rows of A (At[k][r], K-major): sigma[r] and slices S[t][r][k] (k contiguous, ldk)
__global__ __launch_bounds__(256) void k_slice_rows(const double *__restrict__ At, int nrows, int K, int s,
                                                    double *__restrict__ sigma, __bf16 *__restrict__ S,
                                                    int ldk)
{
    const int r = blockIdx.x;
    double m = 0.0;
    for (int k = threadIdx.x; k < K; k += 256) m = fmax(m, fabs(At[(size_t)k * nrows + r]));
    __shared__ double red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    const double sg = pow2_ceil(red[0]);
    if (threadIdx.x == 0) sigma[r] = sg;
    for (int k = threadIdx.x; k < ldk; k += 256) {
        double x = k < K ? At[(size_t)k * nrows + r] / sg : 0.0;
        for (int t = 0; t < s; ++t) {
            const double y = x * 256.0;
            const double a = trunc(y);
            x = y - a;
            S[((size_t)t * nrows + r) * ldk + k] = (__bf16)(float)a;
        }
    }
}

// columns of B (B[k][c], row-major): sigma[c] and slices S[t][c][k] (k contiguous)
__global__ __launch_bounds__(256) void k_slice_cols(const double *__restrict__ B, int K, int N, int s,
                                                    double *__restrict__ sigma, __bf16 *__restrict__ S, int ldk)
{
    // block: 64 columns; max over k, then slices written with k contiguous via LDS
    __shared__ double red[4][64];
    __shared__ float tile[8][64][33];   // [slice][column][k] for 32 k at a time
    const int c0 = blockIdx.x * 64;
    const int cx = threadIdx.x & 63, ky = threadIdx.x >> 6;
    const int c = c0 + cx;
    double m = 0.0;
    if (c < N)
        for (int k = ky; k < K; k += 4) m = fmax(m, fabs(B[(size_t)k * N + c]));
    red[ky][cx] = m;
    __syncthreads();
    const double sg = pow2_ceil(fmax(fmax(red[0][cx], red[1][cx]), fmax(red[2][cx], red[3][cx])));
    if (ky == 0 && c < N) sigma[c] = sg;
    for (int k0 = 0; k0 < ldk; k0 += 32) {
        __syncthreads();
        for (int kk = ky; kk < 32; kk += 4) {
            const int k = k0 + kk;
            double x = (k < K && c < N) ? B[(size_t)k * N + c] / sg : 0.0;
            for (int t = 0; t < s; ++t) {
                const double y = x * 256.0;
                const double a = trunc(y);
                x = y - a;
                tile[t][cx][kk] = (float)a;
            }
        }
        __syncthreads();
        // write S[t][c][k0 .. k0+32): 32 consecutive k per column
        for (int e = threadIdx.x; e < s * 64 * 32; e += 256) {
            const int t = e / (64 * 32), rem = e % (64 * 32), col = rem / 32, kk = rem % 32;
            if (c0 + col < N && k0 + kk < ldk) S[((size_t)t * N + c0 + col) * ldk + k0 + kk] = (__bf16)tile[t][col][kk];
        }
    }
}

hipError_t launch_slices(const double *At, int nrows, const double *B, int K, int N, int s, int ldk,
                         double *sigA, __bf16 *SA, double *sigB, __bf16 *SB, hipStream_t st)
{
    if (s < 1 || s > 8) return hipErrorInvalidValue;
    if (nrows > 0) hipLaunchKernelGGL(k_slice_rows, dim3(nrows), dim3(256), 0, st, At, nrows, K, s, sigA, SA, ldk);
    if (N > 0) hipLaunchKernelGGL(k_slice_cols, dim3((N + 63) / 64), dim3(256), 0, st, B, K, N, s, sigB, SB, ldk);
    return hipGetLastError();
}

// C = A B from slices: tile 64 (r) x 128 (c), 4 waves 2 x 2 of 32 x 64;
// K in steps of 32 (one bf16 MFMA), exact FP32 windows of KCHUNK.
__global__ __launch_bounds__(256) void k_expand_bf16split(const __bf16 *__restrict__ SA,
                                                          const __bf16 *__restrict__ SB,
                                                          const double *__restrict__ sigA,
                                                          const double *__restrict__ sigB, int s, int nrows,
                                                          int N, int ldk, ExpandEpi ep)
{
    constexpr int BK = 64;
    __shared__ __attribute__((aligned(16))) __bf16 As[LBM][BK + 8];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[LBN][BK + 8];
    const int tiles_m = (nrows + LBM - 1) / LBM, tiles_n = (N + LBN - 1) / LBN;
    const int lb = xcd_remap_l(blockIdx.x, tiles_m * tiles_n);
    const int r0 = (lb % tiles_m) * LBM, c0 = (lb / tiles_m) * LBN;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    double acc64[2][4][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[a][b][v] = 0.0;
    for (int t = 1; t <= s; ++t) {
        for (int u = 1; t + u <= s + 1; ++u) {
            const double scale = ldexp(1.0, -8 * (t + u));
            const __bf16 *At_ = SA + (size_t)(t - 1) * nrows * ldk;
            const __bf16 *Bu_ = SB + (size_t)(u - 1) * N * ldk;
            fx4 acc[2][4];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = (fx4){0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < ldk; k0 += BK) {
                __syncthreads();
                // A tile: 64 rows x 64 k (8 bf16 per 16-byte load)
                for (int e = threadIdx.x; e < LBM * BK / 8; e += 256) {
                    const int rr = e / (BK / 8), kc = (e % (BK / 8)) * 8;
                    const int r = r0 + rr;
                    bf16x8 v = {};
                    if (r < nrows) v = *(const bf16x8 *)(At_ + (size_t)r * ldk + k0 + kc);
                    *(bf16x8 *)&As[rr][kc] = v;
                }
                for (int e = threadIdx.x; e < LBN * BK / 8; e += 256) {
                    const int cc = e / (BK / 8), kc = (e % (BK / 8)) * 8;
                    const int c = c0 + cc;
                    bf16x8 v = {};
                    if (c < N) v = *(const bf16x8 *)(Bu_ + (size_t)c * ldk + k0 + kc);
                    *(bf16x8 *)&Bs[cc][kc] = v;
                }
                __syncthreads();
#pragma unroll
                for (int ks = 0; ks < BK; ks += 32) {
                    const int kk = ks + 8 * (lane >> 4);
                    bf16x8 af[2], bfr[4];
#pragma unroll
                    for (int a = 0; a < 2; ++a) af[a] = *(const bf16x8 *)&As[wm * 32 + a * 16 + (lane & 15)][kk];
#pragma unroll
                    for (int b = 0; b < 4; ++b) bfr[b] = *(const bf16x8 *)&Bs[wn * 64 + b * 16 + (lane & 15)][kk];
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
                }
                if (((k0 + BK) % KCHUNK) == 0 || k0 + BK >= ldk) {
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc64[a][b][v] += scale * (double)acc[a][b][v];
                            acc[a][b] = (fx4){0.f, 0.f, 0.f, 0.f};
                        }
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + wm * 32 + a * 16 + 4 * (lane >> 4) + v;
            const double sa = r < nrows ? sigA[r] : 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = c0 + wn * 64 + b * 16 + (lane & 15);
                const double sb = c < N ? sigB[c] : 0.0;
                epilogue_store(ep, r, c, nrows, N, acc64[a][b][v] * sa * sb);
            }
        }
}

// The same product with every slice of a K step in LDS at once (S <= 4):
// each A and B tile is read from memory once per K step instead of once per
// slice pair, and the pairs of one level t + u share an FP32 accumulator.
// Exactness: a level holds at most s pairs, each product of two slices is at
// most 2^16 in magnitude, and the accumulators are folded into FP64 every
// 64 k, so a sum never exceeds s * 64 * 2^16 <= 2^24.
constexpr int FBK = 32, FKW = 64;

template <int S>
__global__ __launch_bounds__(256) void k_expand_bf16fused(const __bf16 *__restrict__ SA,
                                                          const __bf16 *__restrict__ SB,
                                                          const double *__restrict__ sigA,
                                                          const double *__restrict__ sigB, int nrows, int N,
                                                          int ldk, ExpandEpi ep)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[S][LBM][FBK + 8];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[S][LBN][FBK + 8];
    const int tiles_m = (nrows + LBM - 1) / LBM, tiles_n = (N + LBN - 1) / LBN;
    const int lb = xcd_remap_l(blockIdx.x, tiles_m * tiles_n);
    const int r0 = (lb % tiles_m) * LBM, c0 = (lb / tiles_m) * LBN;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    double acc64[2][4][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[a][b][v] = 0.0;
    fx4 acc[S][2][4];   // level t + u - 2
#pragma unroll
    for (int l = 0; l < S; ++l)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[l][a][b] = (fx4){0.f, 0.f, 0.f, 0.f};
    // the next K step's tiles are loaded into registers while the current
    // one is multiplied from LDS
    bf16x8 pa[S], pb[S][2];
    auto gload = [&](int k0) {
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const __bf16 *At_ = SA + (size_t)t * nrows * ldk;
            const __bf16 *Bt_ = SB + (size_t)t * N * ldk;
            const int rr = threadIdx.x >> 2, kc = (threadIdx.x & 3) * 8;
            const int r = r0 + rr;
            pa[t] = r < nrows ? *(const bf16x8 *)(At_ + (size_t)r * ldk + k0 + kc) : (bf16x8){};
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int e = threadIdx.x + 256 * q;
                const int c = c0 + (e >> 2);
                pb[t][q] = c < N ? *(const bf16x8 *)(Bt_ + (size_t)c * ldk + k0 + (e & 3) * 8) : (bf16x8){};
            }
        }
    };
    gload(0);
    for (int k0 = 0; k0 < ldk; k0 += FBK) {
        __syncthreads();   // the previous step is done with the LDS tiles
#pragma unroll
        for (int t = 0; t < S; ++t) {
            *(bf16x8 *)&As[t][threadIdx.x >> 2][(threadIdx.x & 3) * 8] = pa[t];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int e = threadIdx.x + 256 * q;
                *(bf16x8 *)&Bs[t][e >> 2][(e & 3) * 8] = pb[t][q];
            }
        }
        __syncthreads();
        if (k0 + FBK < ldk) gload(k0 + FBK);
        const int kk = 8 * (lane >> 4);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            bf16x8 af[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = *(const bf16x8 *)&As[t][wm * 32 + a * 16 + (lane & 15)][kk];
#pragma unroll
            for (int u = 0; u < S - t; ++u) {
                bf16x8 bfr[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) bfr[b] = *(const bf16x8 *)&Bs[u][wn * 64 + b * 16 + (lane & 15)][kk];
                const int l = t + u;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[l][a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[l][a][b], 0, 0, 0);
            }
        }
        if (((k0 + FBK) % FKW) == 0 || k0 + FBK >= ldk) {
#pragma unroll
            for (int l = 0; l < S; ++l) {
                const double scale = ldexp(1.0, -8 * (l + 2));
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc64[a][b][v] += scale * (double)acc[l][a][b][v];
                        acc[l][a][b] = (fx4){0.f, 0.f, 0.f, 0.f};
                    }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + wm * 32 + a * 16 + 4 * (lane >> 4) + v;
            const double sa = r < nrows ? sigA[r] : 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = c0 + wn * 64 + b * 16 + (lane & 15);
                const double sb = c < N ? sigB[c] : 0.0;
                epilogue_store(ep, r, c, nrows, N, acc64[a][b][v] * sa * sb);
            }
        }
}

hipError_t launch_expand_bf16split(const __bf16 *SA, const __bf16 *SB, const double *sigA, const double *sigB,
                                   int s, int nrows, int N, int ldk, const ExpandEpi &ep, hipStream_t st)
{
    if (nrows <= 0 || N <= 0) return hipSuccess;
    if (ldk % 64) return hipErrorInvalidValue;
    const int tiles = ((nrows + LBM - 1) / LBM) * ((N + LBN - 1) / LBN);
    switch (s) {
    case 1: hipLaunchKernelGGL(k_expand_bf16fused<1>, dim3(tiles), dim3(256), 0, st, SA, SB, sigA, sigB, nrows, N,
                               ldk, ep); break;
    case 2: hipLaunchKernelGGL(k_expand_bf16fused<2>, dim3(tiles), dim3(256), 0, st, SA, SB, sigA, sigB, nrows, N,
                               ldk, ep); break;
    case 3: hipLaunchKernelGGL(k_expand_bf16fused<3>, dim3(tiles), dim3(256), 0, st, SA, SB, sigA, sigB, nrows, N,
                               ldk, ep); break;
    case 4: hipLaunchKernelGGL(k_expand_bf16fused<4>, dim3(tiles), dim3(256), 0, st, SA, SB, sigA, sigB, nrows, N,
                               ldk, ep); break;
    default:
        hipLaunchKernelGGL(k_expand_bf16split, dim3(tiles), dim3(256), 0, st, SA, SB, sigA, sigB, s, nrows, N, ldk,
                           ep);
    }
    return hipGetLastError();
}

}  // namespace cch
