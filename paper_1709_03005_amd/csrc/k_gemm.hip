// Expansion of the contracted symbols over the continuum pairs (j, j')
// (Sec. 2.1, end; Sec. 3.1 "expansion"): the integral labels of a
// contracted element keep their target part (P, Q) while (j, j') runs over
// the continuum orbitals of the two symmetries. Written as one dense product
// per target-symmetry pair:
//   Ht[(n,n'), (j,j')] = sum_{PQ} Gamma_{nn',PQ} (PQ|jj')
//                      - sum_{PQ} Gamma^alpha_{nn',PQ} (Pj'|jQ)
//                      + delta_{jj'} (C^T H_T C')_{nn'} + (C^T O C')_{nn'} h_{jj'}
// K0 lays the integral rows out as B[(PQ)][(j,j')]; K5 multiplies with FP64
// MFMA (v_mfma_f64_16x16x4) and scatters each (n,n',j,j') to its row
// (i,n,j) / column (i',n',j') of the contracted matrix (lower triangle).
#include <algorithm>

#include "ccham_internal.h"

namespace cch {

// ---------------------------------------------------------------------------
// K0: B[k][jj*ncb + jj'] for one symmetry pair.
//   k <  n_slot: (P Q | J J')    = ttcc[P][Q][J][J']       (row copy)
//   k >= n_slot: -(P J' | J Q)   = -tctc[P][J'][Q][J]     (tile transpose)
// ---------------------------------------------------------------------------
// B[k][jj][jj'] = (P Q | ja0+jj, jb0+jj'): the slab of slot k is one contiguous
// nca x ncb block of B, gathered from nca rows of ttcc; a workgroup copies
// RJ_PER consecutive elements of a slab (all its loads issued before its stores)
constexpr int RJ_U = 4, RJ_PER = 256 * RJ_U;

__global__ __launch_bounds__(256) void k_relayout_J(const double *__restrict__ ttcc, int n_o, int n_cont,
                                                    const int32_t *__restrict__ slotP,
                                                    const int32_t *__restrict__ slotQ, int ja0, int nca,
                                                    int jb0, int ncb, double *__restrict__ B)
{
    const int k = blockIdx.y;
    const int P = slotP[k], Q = slotQ[k];
    const double *src = ttcc + ((size_t)P * n_o + Q) * n_cont * n_cont + (size_t)ja0 * n_cont + jb0;
    double *dst = B + (size_t)k * nca * ncb;
    const int64_t slab = (int64_t)nca * ncb, e0 = (int64_t)blockIdx.x * RJ_PER + threadIdx.x;
    double v[RJ_U];
#pragma unroll
    for (int u = 0; u < RJ_U; ++u) {
        const int64_t e = e0 + 256 * u;
        v[u] = e < slab ? src[(e / ncb) * n_cont + e % ncb] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < RJ_U; ++u) {
        const int64_t e = e0 + 256 * u;
        if (e < slab) dst[e] = v[u];
    }
}

__global__ __launch_bounds__(256) void k_relayout_K(const double *__restrict__ tctc, int n_o, int n_cont,
                                                    const int32_t *__restrict__ slotP,
                                                    const int32_t *__restrict__ slotQ, int n_slot, int ja0,
                                                    int nca, int jb0, int ncb, double *__restrict__ B)
{
    __shared__ double tile[32][33];
    const int k = blockIdx.z;
    const int P = slotP[k], Q = slotQ[k];
    const int jj0 = blockIdx.x * 32, jp0 = blockIdx.y * 32;   // jj (unprimed) / jj' tiles
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;    // 32 x 8
    // read tctc[P][J'][Q][J]: contiguous in J
    for (int r = ty; r < 32; r += 8) {
        const int jp = jp0 + r, jj = jj0 + tx;
        double v = 0.0;
        if (jp < ncb && jj < nca)
            v = tctc[(((size_t)P * n_cont + (jb0 + jp)) * n_o + Q) * n_cont + (ja0 + jj)];
        tile[r][tx] = v;
    }
    __syncthreads();
    // write B[n_slot + k][jj][jj']: contiguous in jj'
    double *dst = B + (size_t)(n_slot + k) * nca * ncb;
    for (int r = ty; r < 32; r += 8) {
        const int jj = jj0 + r, jp = jp0 + tx;
        if (jj < nca && jp < ncb) dst[(size_t)jj * ncb + jp] = -tile[tx][r];
    }
}

// the same rows from the symmetry-packed layout: one record per target pair,
// the (tt|cc) rows of this launch contiguous (row length ncb), the (tc|tc)
// block read row by row over j and turned through LDS
__global__ __launch_bounds__(256) void k_relayout_Jp(const double *__restrict__ ttcc, PackedCC pk, int n_o,
                                                     const int32_t *__restrict__ slotP,
                                                     const int32_t *__restrict__ slotQ, int nca, int ncb,
                                                     double *__restrict__ B)
{
    const int k = blockIdx.y;
    const double *src = ttcc + pk.rec[(size_t)slotP[k] * n_o + slotQ[k]] + pk.boffJ;
    double *dst = B + (size_t)k * nca * ncb;
    const int64_t slab = (int64_t)nca * ncb, e0 = (int64_t)blockIdx.x * RJ_PER + threadIdx.x;
    double v[RJ_U];
#pragma unroll
    for (int u = 0; u < RJ_U; ++u) {
        const int64_t e = e0 + 256 * u;
        v[u] = e < slab ? src[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < RJ_U; ++u) {
        const int64_t e = e0 + 256 * u;
        if (e < slab) dst[e] = v[u];
    }
}

__global__ __launch_bounds__(256) void k_relayout_Kp(const double *__restrict__ tctc, PackedCC pk, int n_o,
                                                     const int32_t *__restrict__ slotP,
                                                     const int32_t *__restrict__ slotQ, int n_slot, int nca,
                                                     int ncb, double *__restrict__ B)
{
    __shared__ double tile[32][33];
    const int k = blockIdx.z;
    const double *src = tctc + pk.rec[(size_t)slotP[k] * n_o + slotQ[k]] + pk.boffK;
    const int jj0 = blockIdx.x * 32, jp0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // (P j' | Q j): row j' of the block, contiguous in j
    for (int r = ty; r < 32; r += 8) {
        const int jp = jp0 + r, jj = jj0 + tx;
        tile[r][tx] = (jp < ncb && jj < nca) ? src[(int64_t)jp * pk.nca_full + pk.jr0 + jj] : 0.0;
    }
    __syncthreads();
    double *dst = B + (size_t)(n_slot + k) * nca * ncb;
    for (int r = ty; r < 32; r += 8) {
        const int jj = jj0 + r, jp = jp0 + tx;
        if (jj < nca && jp < ncb) dst[(size_t)jj * ncb + jp] = -tile[tx][r];
    }
}

hipError_t launch_relayout(const double *ttcc, const double *tctc, int n_o, int n_cont,
                           const int32_t *slotP, const int32_t *slotQ, int n_slot, int ja0, int nca,
                           int jb0, int ncb, double *B, hipStream_t st, const PackedCC *pk)
{
    if (n_slot <= 0 || nca <= 0 || ncb <= 0) return hipSuccess;
    if (pk) {
        hipLaunchKernelGGL(k_relayout_Jp, dim3((int)(((int64_t)nca * ncb + RJ_PER - 1) / RJ_PER), n_slot), dim3(256),
                           0, st, ttcc, *pk, n_o, slotP, slotQ, nca, ncb, B);
        hipLaunchKernelGGL(k_relayout_Kp, dim3((nca + 31) / 32, (ncb + 31) / 32, n_slot), dim3(256), 0, st, tctc, *pk,
                           n_o, slotP, slotQ, n_slot, nca, ncb, B);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_relayout_J, dim3((int)(((int64_t)nca * ncb + RJ_PER - 1) / RJ_PER), n_slot), dim3(256), 0, st,
                       ttcc, n_o, n_cont, slotP, slotQ, ja0, nca, jb0, ncb, B);
    hipLaunchKernelGGL(k_relayout_K, dim3((nca + 31) / 32, (ncb + 31) / 32, n_slot), dim3(256), 0, st, tctc,
                       n_o, n_cont, slotP, slotQ, n_slot, ja0, nca, jb0, ncb, B);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K5: C = A * B with A given K-major (At[k][r]), FP64 MFMA 4x4x4 (four
// blocks). Workgroup tile 64 (r) x 128 (col), 4 waves in 2 x 2, each 32 x 64 =
// 8 x 4 instructions of 4 rows x 16 columns. K staged through LDS in slices
// of 16. Operand layout of the four-block 4x4x4 f64 MFMA (lane l = j + 4 blk +
// 16 i, checked on gfx950): A[blk][i][k] at lane i + 4 blk + 16 k, B[blk][k][j]
// at lane j + 4 blk + 16 k, D[blk][i][j] at lane j + 4 blk + 16 i. With the
// same A slab in every block, an instruction multiplies 4 rows by 16 columns
// (B's column 4 blk + j); on this chip it issues faster per flop than the
// 16x16x4 form.
// ---------------------------------------------------------------------------
typedef double dx4 __attribute__((ext_vector_type(4)));

struct ExpandEpi {
    double *H;            // contracted matrix, row-major
    int64_t ld;
    int64_t row0a, row0b; // first row of symmetry a / b
    int nca, ncb;         // continuum orbitals of a / b
    int ja0, jb0;         // first global continuum index of a / b
    const int32_t *rn, *rn2;
    const double *HT, *O; // per GEMM row
    const double *h;      // one-electron matrix [n_orb][n_orb]
    int n_o, n_orb;
};

constexpr int GBN = 128, GBK = 16;

__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    // consecutive logical tiles land on one XCD (blocks are dealt round-robin
    // over the 8 XCDs), so tiles sharing a B column panel share an L2
    const int per = nb / 8;
    if (b >= per * 8) return b;
    return (b % 8) * per + b / 8;
}

// One output tile (BM rows x 128 columns) of the expansion product; 4 waves,
// BM/32 x (4/(BM/32)) of them, each 32 rows x (128 / waves_n) columns.
template <int BM>
__device__ __forceinline__ void expand_tile_f64(const double *__restrict__ At, const double *__restrict__ B,
                                                int nrows, int N, int K, const ExpandEpi &ep, int tm, int tn,
                                                double (*As)[BM], double (*Bs)[GBN])
{
    constexpr int WAVES_M = BM / 32, WAVES_N = 4 / WAVES_M;
    constexpr int WCOLS = GBN / WAVES_N, NT = WCOLS / 16;   // MFMA tiles along N per wave
    constexpr int AQ = BM * GBK / 256, BQ = GBN * GBK / 256;
    const int r0 = tm * BM, c0 = tn * GBN;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wm = wv % WAVES_M, wn = wv / WAVES_M;

    // 4x4x4 FP64 MFMA (four blocks sharing the A slab): one instruction is 4
    // rows x 16 columns x 4 k; lane l holds row 4 m + (l >> 4), column 16 n +
    // (l & 15) of the wave's 32 x WCOLS tile
    double acc[8][NT];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = 0.0;

    double ra[AQ], rb[BQ];
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int kk = e / BM, rr = e % BM;
            const int k = k0 + kk, r = r0 + rr;
            ra[q] = (k < K && r < nrows) ? At[(size_t)k * nrows + r] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int kk = e / GBN, cc = e % GBN;
            const int k = k0 + kk, c = c0 + cc;
            rb[q] = (k < K && c < N) ? B[(size_t)k * N + c] : 0.0;
        }
    };
    gload(0);
    for (int k0 = 0; k0 < K; k0 += GBK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < AQ; ++q) {
            const int e = threadIdx.x + 256 * q;
            As[e / BM][e % BM] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < BQ; ++q) {
            const int e = threadIdx.x + 256 * q;
            Bs[e / GBN][e % GBN] = rb[q];
        }
        __syncthreads();
        if (k0 + GBK < K) gload(k0 + GBK);
#pragma unroll
        for (int ks = 0; ks < GBK; ks += 4) {
            const int kk = ks + (lane >> 4);
            double bf[NT];
#pragma unroll
            for (int b = 0; b < NT; ++b) bf[b] = Bs[kk][wn * WCOLS + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                const double af = As[kk][wm * 32 + 4 * a + (lane & 3)];
#pragma unroll
                for (int b = 0; b < NT; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_4x4x4f64(af, bf[b], acc[a][b], 0, 0, 0);
            }
        }
    }
    __syncthreads();   // the LDS tiles are reused by the next tile of a persistent loop

    // epilogue: scatter into the contracted matrix (lower triangle only)
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        {
            const int r = r0 + wm * 32 + 4 * a + (lane >> 4);
            if (r >= nrows) continue;
            const int n = ep.rn[r], n2 = ep.rn2[r];
            const double ht = ep.HT[r], ov = ep.O[r];
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const int c = c0 + wn * WCOLS + b * 16 + (lane & 15);
                if (c >= N) continue;
                const int jj = c / ep.ncb, jp = c - jj * ep.ncb;
                const int64_t R = ep.row0a + (int64_t)n * ep.nca + jj;
                const int64_t C = ep.row0b + (int64_t)n2 * ep.ncb + jp;
                if (R < C) continue;
                const int J = ep.ja0 + jj, Jp = ep.jb0 + jp;
                double val = acc[a][b];
                if (J == Jp) val += ht;
                val += ov * ep.h[(size_t)(ep.n_o + J) * ep.n_orb + (ep.n_o + Jp)];
                ep.H[R * ep.ld + C] = val;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_expand_f64(const double *__restrict__ At, const double *__restrict__ B,
                                                    int nrows, int N, int K, ExpandEpi ep)
{
    __shared__ double As[GBK][64];
    __shared__ double Bs[GBK][GBN];
    const int tiles_m = (nrows + 63) / 64;
    const int tiles_n = (N + GBN - 1) / GBN;
    const int lb = xcd_remap(blockIdx.x, tiles_m * tiles_n);
    expand_tile_f64<64>(At, B, nrows, N, K, ep, lb % tiles_m, lb / tiles_m, As, Bs);
}

hipError_t launch_expand_f64(const double *At, const double *B, int nrows, int N, int K, const ExpandEpi &ep,
                             hipStream_t st)
{
    if (nrows <= 0 || N <= 0) return hipSuccess;
    const int tiles = ((nrows + 63) / 64) * ((N + GBN - 1) / GBN);
    hipLaunchKernelGGL(k_expand_f64, dim3(tiles), dim3(256), 0, st, At, B, nrows, N, K, ep);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Persistent form over many (instance, symmetry pair) products: a fixed grid
// walks the concatenated tile list (static round-robin); descriptor d owns
// tiles [first[d], first[d] + tiles_m * tiles_n).
// ---------------------------------------------------------------------------
struct GemmTask {
    const double *At;
    const double *B;
    int nrows, N, K;
    int tiles_m, tiles_n;
    int64_t first;
    ExpandEpi ep;
};

template <int BM>
__global__ __launch_bounds__(256) void k_expand_f64_batched(const GemmTask *__restrict__ tasks, int ntask,
                                                            int64_t total)
{
    __shared__ double As[GBK][BM];
    __shared__ double Bs[GBK][GBN];
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = ntask - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tasks[mid].first <= t) lo = mid;
            else hi = mid - 1;
        }
        const GemmTask &g = tasks[lo];
        const int64_t local = t - g.first;
        expand_tile_f64<BM>(g.At, g.B, g.nrows, g.N, g.K, g.ep, (int)(local % g.tiles_m),
                            (int)(local / g.tiles_m), As, Bs);
    }
}

int expand_tiles(int nrows, int N, int bm) { return ((nrows + bm - 1) / bm) * ((N + GBN - 1) / GBN); }

hipError_t launch_expand_f64_batched(const GemmTask *tasks, int ntask, int64_t total, int bm, int grid,
                                     hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>(total, grid);
    if (bm == 32)
        hipLaunchKernelGGL((k_expand_f64_batched<32>), dim3(g), dim3(256), 0, st, tasks, ntask, total);
    else
        hipLaunchKernelGGL((k_expand_f64_batched<64>), dim3(g), dim3(256), 0, st, tasks, ntask, total);
    return hipGetLastError();
}

}  // namespace cch
