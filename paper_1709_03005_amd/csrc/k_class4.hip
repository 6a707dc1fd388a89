// Class 4: continuum x L2 elements with the one-dimensional contraction of
// Eq. 5, Ht[(i,n,j), l] = sum_m c_imn <eta_im u_j | H | chi_l>
// (Sec. 2.2 "Class 4"; Sec. 3.1: the work is split over the L2 functions).
//
// For one L2 function chi_l the connected target determinants D_m (from the
// excitation scan) give a prototype symbolic element whose integral labels
// carry the continuum index j in one slot; contracting the coefficients over
// m (Eq. 8 in one dimension) and expanding over j is a product
//     out[n][j] = sum_t (coef_t c_{m_t n}) X_t[j]
// where each term t is a row of the one-electron integrals h[H][j] or of
// the (tt|tc) integrals (ab|c j), read for a tile of j:
//   single substitution (chi_l = D_m + h, h alpha), sign s:
//       s [ h_{hj} + sum_{k in D_m} (KK|Hj) - sum_{k in D_m, alpha} (KH|Kj) ]
//   double (chi_l = D_m - p + h1 + h2), sign s:
//       s [ (P H1|H2 j) d(sp,sh1) d(alpha,sh2) - (P H2|H1 j) d(sp,sh2) d(alpha,sh1) ]
// One workgroup per (l, tile of 64 j); pairs are turned into terms in
// order, so the accumulation order is fixed.
#include <algorithm>

#include "ccham_internal.h"

namespace cch {

struct Class4Args {
    const uint64_t *tdets;   // target dets of the symmetry [M][W]
    const double *ci;        // [M][S]
    int S;
    const double *h;         // [n_orb][n_orb]
    const double *tttc;      // [n_o][n_o][n_o][n_cont]
    int n_o, n_orb, n_cont;
    int ja0, nc;             // continuum range of the symmetry
    const int64_t *row_off, *row_cnt;   // L2 x target pairs per L2 row
    PairList pl;
    double *H;
    int64_t ld;
    int64_t row_l2;          // first L2 row of the matrix
    int64_t col0;            // first column of the symmetry block
    int pairs_per_chunk;
};

constexpr int C4_TERMS = 1024;
constexpr int C4_NQ = 16;          // states per thread: S <= 64 per pass

struct C4Shared {
    const double *trow[C4_TERMS];
    double tcoef[C4_TERMS];
    int32_t tm[C4_TERMS];
    int32_t pcount[64], poff[65];
};

// one L2 row l and one tile of 64 continuum orbitals
template <int W>
__device__ __forceinline__ void class4_row(const Class4Args &a, int l, int jtile, C4Shared &sh)
{
    const double **trow = sh.trow;
    double *tcoef = sh.tcoef;
    int32_t *tm = sh.tm;
    int32_t *pcount = sh.pcount, *poff = sh.poff;
    const int jj0 = jtile * 64;
    __syncthreads();   // the LDS term lists are reused by the next row of a persistent loop
    const int jl = threadIdx.x & 63;          // j within the tile
    const int nq0 = threadIdx.x >> 6;         // first state of this thread
    const int64_t p0 = a.row_off[l], np = a.row_cnt[l];
    const int jj = jj0 + jl;
    const bool jok = jj < a.nc;

    for (int nbase = 0; nbase < a.S; nbase += 4 * C4_NQ) {
        double acc[C4_NQ];
#pragma unroll
        for (int q = 0; q < C4_NQ; ++q) acc[q] = 0.0;
        for (int64_t c0 = 0; c0 < np; c0 += a.pairs_per_chunk) {
            const int nc_pairs = (int)min<int64_t>(a.pairs_per_chunk, np - c0);
            __syncthreads();
            // count terms of each pair
            if (threadIdx.x < nc_pairs) {
                const int64_t pi = p0 + c0 + threadIdx.x;
                const int deg = a.pl.deg[pi];
                const uint64_t lab = a.pl.label[pi];
                int cnt = 0;
                if (deg == 1) {
                    const int h = lab_field(lab, 1);
                    if ((h & 1) == 0) {
                        const uint64_t *d = a.tdets + (size_t)a.pl.y[pi] * W;
                        int ne = 0, na = 0;
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            ne += __popcll(d[w]);
                            na += __popcll(d[w] & 0x5555555555555555ull);
                        }
                        cnt = 1 + ne + na;
                    }
                } else {
                    const int pt = lab_field(lab, 0), h1 = lab_field(lab, 1), h2 = lab_field(lab, 2);
                    cnt = ((pt & 1) == (h1 & 1) && (h2 & 1) == 0) + ((pt & 1) == (h2 & 1) && (h1 & 1) == 0);
                }
                pcount[threadIdx.x] = cnt;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int s = 0;
                for (int t = 0; t < nc_pairs; ++t) {
                    poff[t] = s;
                    s += pcount[t];
                }
                poff[nc_pairs] = s;
            }
            __syncthreads();
            // generate the terms of each pair at its offset
            if (threadIdx.x < nc_pairs) {
                const int64_t pi = p0 + c0 + threadIdx.x;
                const int deg = a.pl.deg[pi];
                const uint64_t lab = a.pl.label[pi];
                const double s = (double)a.pl.phase[pi];
                const int m = a.pl.y[pi];
                int o = poff[threadIdx.x];
                const size_t n_o = a.n_o;
                if (deg == 1) {
                    const int h = lab_field(lab, 1);
                    if ((h & 1) == 0) {
                        const int H = h >> 1;
                        trow[o] = a.h + (size_t)H * a.n_orb + a.n_o + a.ja0;
                        tcoef[o] = s;
                        tm[o++] = m;
                        const uint64_t *d = a.tdets + (size_t)m * W;
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            uint64_t x = d[w];
                            while (x) {
                                const int k = 64 * w + (int)__builtin_ctzll(x);
                                x &= x - 1;
                                const size_t K = k >> 1;
                                trow[o] = a.tttc + ((K * n_o + K) * n_o + H) * a.n_cont + a.ja0;
                                tcoef[o] = s;
                                tm[o++] = m;
                                if ((k & 1) == 0) {
                                    trow[o] = a.tttc + ((K * n_o + H) * n_o + K) * a.n_cont + a.ja0;
                                    tcoef[o] = -s;
                                    tm[o++] = m;
                                }
                            }
                        }
                    }
                } else {
                    const int pt = lab_field(lab, 0), h1 = lab_field(lab, 1), h2 = lab_field(lab, 2);
                    const size_t P = pt >> 1, H1 = h1 >> 1, H2 = h2 >> 1;
                    if ((pt & 1) == (h1 & 1) && (h2 & 1) == 0) {
                        trow[o] = a.tttc + ((P * n_o + H1) * n_o + H2) * a.n_cont + a.ja0;
                        tcoef[o] = s;
                        tm[o++] = m;
                    }
                    if ((pt & 1) == (h2 & 1) && (h1 & 1) == 0) {
                        trow[o] = a.tttc + ((P * n_o + H2) * n_o + H1) * a.n_cont + a.ja0;
                        tcoef[o] = -s;
                        tm[o++] = m;
                    }
                }
            }
            __syncthreads();
            const int nt = poff[nc_pairs];
            for (int t = 0; t < nt; ++t) {
                const double x = jok ? trow[t][jj] : 0.0;
                const double cx = tcoef[t] * x;
                const double *crow = a.ci + (size_t)tm[t] * a.S + nbase;
#pragma unroll
                for (int q = 0; q < C4_NQ; ++q) {
                    const int n = nq0 + 4 * q;
                    if (nbase + n < a.S) acc[q] = fma(crow[n], cx, acc[q]);
                }
            }
        }
        if (jok) {
            double *out = a.H + (a.row_l2 + l) * a.ld + a.col0 + jj;
#pragma unroll
            for (int q = 0; q < C4_NQ; ++q) {
                const int n = nbase + nq0 + 4 * q;
                if (n < a.S) out[(size_t)n * a.nc] = acc[q];
            }
        }
    }
}

template <int W>
__global__ __launch_bounds__(256) void k_class4(Class4Args a, int n_l2)
{
    __shared__ C4Shared sh;
    if ((int)blockIdx.x >= n_l2) return;
    class4_row<W>(a, blockIdx.x, blockIdx.y, sh);
}

hipError_t launch_class4(int W, const Class4Args &a, int n_l2, hipStream_t st)
{
    if (n_l2 <= 0 || a.nc <= 0 || a.S <= 0) return hipSuccess;
    const dim3 g(n_l2, (a.nc + 63) / 64), b(256);
    switch (W) {
    case 1: hipLaunchKernelGGL((k_class4<1>), g, b, 0, st, a, n_l2); break;
    case 2: hipLaunchKernelGGL((k_class4<2>), g, b, 0, st, a, n_l2); break;
    case 3: hipLaunchKernelGGL((k_class4<3>), g, b, 0, st, a, n_l2); break;
    case 4: hipLaunchKernelGGL((k_class4<4>), g, b, 0, st, a, n_l2); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// persistent form over many (instance, symmetry) blocks with the same word count
struct C4Task {
    Class4Args a;
    int n_l2, jtiles;
    int64_t first;
};

template <int W>
__global__ __launch_bounds__(256) void k_class4_batched(const C4Task *__restrict__ tasks, int ntask, int64_t total)
{
    __shared__ C4Shared sh;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = ntask - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tasks[mid].first <= t) lo = mid;
            else hi = mid - 1;
        }
        const C4Task &k = tasks[lo];
        const int64_t local = t - k.first;
        class4_row<W>(k.a, (int)(local / k.jtiles), (int)(local % k.jtiles), sh);
    }
}

hipError_t launch_class4_batched(int W, const C4Task *tasks, int ntask, int64_t total, int grid, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    const dim3 g((unsigned)std::min<int64_t>(total, grid)), bl(256);
    switch (W) {
    case 1: hipLaunchKernelGGL((k_class4_batched<1>), g, bl, 0, st, tasks, ntask, total); break;
    case 2: hipLaunchKernelGGL((k_class4_batched<2>), g, bl, 0, st, tasks, ntask, total); break;
    case 3: hipLaunchKernelGGL((k_class4_batched<3>), g, bl, 0, st, tasks, ntask, total); break;
    case 4: hipLaunchKernelGGL((k_class4_batched<4>), g, bl, 0, st, tasks, ntask, total); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace cch
