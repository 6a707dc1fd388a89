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
//   single substitution (chi_l = D_m + h, h of the continuum spin sigma_m), sign s:
//       s [ h_{hj} + sum_{k in D_m} (KK|Hj) - sum_{k in D_m, spin sigma_m} (KH|Kj) ]
//   double (chi_l = D_m - p + h1 + h2), sign s:
//       s [ (P H1|H2 j) d(sp,sh1) d(sigma_m,sh2) - (P H2|H1 j) d(sp,sh2) d(sigma_m,sh1) ]
// (sigma_m the continuum spin given with D_m, alpha unless stated).
// The product runs on the FP64 matrix cores: for a block of 64 terms the
// A operand is (coef_t c_{m_t n}) (terms x states, staged in LDS from the CI
// rows) and the B operand the gathered integral rows X_t[j] (terms x j),
// read straight from memory, 16 states x 16 continuum orbitals per MFMA
// tile. One workgroup per (l, block of 512 j); each of its four waves takes
// pairs of j tiles and every state tile, so each integral value is read once
// per workgroup. Pairs are turned into terms in order and the term blocks are
// added in order, so the accumulation order is fixed.
#include <algorithm>

#include "ccham_internal.h"

namespace cch {


constexpr int C4_TERMS = 1024;
constexpr int C4_TB = 64;          // terms per MFMA block (16 k-steps)

constexpr int C4_LA = 64 + 1;      // LDS row stride of the staged A operand

struct C4Shared {
    const double *trow[C4_TERMS];
    double tcoef[C4_TERMS];
    int32_t tm[C4_TERMS];
    int32_t poff[65];
    double A[C4_TB * C4_LA];       // coef_t c[m_t][n], a block of terms x 64 states
};

typedef double c4x4 __attribute__((ext_vector_type(4)));

// one L2 row l and one block of C4_JB continuum orbitals
template <int W>
__device__ __forceinline__ void class4_row(const Class4Args &a, int l, int jblk, C4Shared &sh)
{
    const double **trow = sh.trow;
    double *tcoef = sh.tcoef;
    int32_t *tm = sh.tm;
    int32_t *poff = sh.poff;
    const int j0 = jblk * C4_JB, jn = min(C4_JB, a.nc - j0);
    __syncthreads();   // the LDS term lists are reused by the next row of a persistent loop
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    const int64_t p0 = a.row_off[l], np = a.row_cnt[l];
    const int jtiles = (jn + 15) / 16;
    double *out = a.H + (a.row_l2 + l) * a.ld + a.col0 + j0;
    bool have = false;   // some term block has written the outputs

    for (int64_t c0 = 0; c0 < np; c0 += a.pairs_per_chunk) {
        const int nc_pairs = (int)min<int64_t>(a.pairs_per_chunk, np - c0);
        __syncthreads();
        // count the terms of each pair; offsets by a scan across wave 0
        if (threadIdx.x < 64) {
            int cnt = 0;
            if (threadIdx.x < nc_pairs) {
                const int64_t pi = p0 + c0 + threadIdx.x;
                const int deg = a.pl.deg[pi];
                const uint64_t lab = a.pl.label[pi];
                const int sg = a.cspin ? a.cspin[a.pl.y[pi]] : 0;   // continuum spin
                if (deg == 1) {
                    const int h = lab_field(lab, 1);
                    if ((h & 1) == sg) {
                        const uint64_t *d = a.tdets + (size_t)a.pl.y[pi] * W;
                        const uint64_t mask = sg ? 0xAAAAAAAAAAAAAAAAull : 0x5555555555555555ull;
                        int ne = 0, ns = 0;
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            ne += __popcll(d[w]);
                            ns += __popcll(d[w] & mask);
                        }
                        cnt = 1 + ne + ns;
                    }
                } else {
                    const int pt = lab_field(lab, 0), h1 = lab_field(lab, 1), h2 = lab_field(lab, 2);
                    cnt = ((pt & 1) == (h1 & 1) && (h2 & 1) == sg) + ((pt & 1) == (h2 & 1) && (h1 & 1) == sg);
                }
            }
            int incl = cnt;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o, 64);
                if ((int)threadIdx.x >= o) incl += y;
            }
            if ((int)threadIdx.x < nc_pairs) poff[threadIdx.x] = incl - cnt;
            if ((int)threadIdx.x == nc_pairs - 1) poff[nc_pairs] = incl;
        }
        __syncthreads();
        // generate the terms of each pair at its offset
        if (threadIdx.x < nc_pairs) {
            const int64_t pi = p0 + c0 + threadIdx.x;
            const int deg = a.pl.deg[pi];
            const uint64_t lab = a.pl.label[pi];
            const double s = (double)a.pl.phase[pi];
            const int m = a.pl.y[pi];
            const int sg = a.cspin ? a.cspin[m] : 0;
            int o = poff[threadIdx.x];
            const size_t n_o = a.n_o;
            if (deg == 1) {
                const int h = lab_field(lab, 1);
                if ((h & 1) == sg) {
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
                            if ((k & 1) == sg) {
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
                if ((pt & 1) == (h1 & 1) && (h2 & 1) == sg) {
                    trow[o] = a.tttc + ((P * n_o + H1) * n_o + H2) * a.n_cont + a.ja0;
                    tcoef[o] = s;
                    tm[o++] = m;
                }
                if ((pt & 1) == (h2 & 1) && (h1 & 1) == sg) {
                    trow[o] = a.tttc + ((P * n_o + H2) * n_o + H1) * a.n_cont + a.ja0;
                    tcoef[o] = -s;
                    tm[o++] = m;
                }
            }
        }
        __syncthreads();
        const int nt = poff[nc_pairs];
        // out[n][j] (+)= sum_t (coef_t c[m_t][n]) X_t[j], blocks of C4_TB terms:
        // the A operand (coef_t c[m_t][n]) of a block and 64 states is staged in
        // LDS; each wave takes pairs of 16-orbital j tiles and all state tiles of
        // the pass, so an integral value is loaded once per workgroup
        for (int tb = 0; tb < nt; tb += C4_TB) {
            const int tn = min(C4_TB, nt - tb);
            for (int nb = 0; nb < a.S; nb += 64) {
                __syncthreads();   // the previous block's A is no longer read
                for (int e = threadIdx.x; e < C4_TB * 64; e += blockDim.x) {
                    const int t = e >> 6, n = nb + (e & 63);
                    sh.A[t * C4_LA + (e & 63)] =
                        (t < tn && n < a.S) ? tcoef[tb + t] * a.ci[(size_t)tm[tb + t] * a.S + n] : 0.0;
                }
                __syncthreads();
                const int nts = min(4, (a.S - nb + 15) / 16);
                for (int jt = 2 * wv; jt < jtiles; jt += 8) {
                    const int ja = 16 * jt + lo, jb = ja + 16;
                    c4x4 acc[4][2];
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[q][0] = acc[q][1] = (c4x4){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
                    for (int u = 0; u < C4_TB / 4; ++u) {
                        if (4 * u < tn) {
                            const int t = 4 * u + hi;
                            const double *tr = t < tn ? trow[tb + t] : nullptr;
                            const double b0 = (tr && ja < jn) ? tr[j0 + ja] : 0.0;
                            const double b1 = (tr && jb < jn) ? tr[j0 + jb] : 0.0;
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                if (q < nts) {
                                    const double av = sh.A[t * C4_LA + 16 * q + lo];
                                    acc[q][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, acc[q][0], 0, 0, 0);
                                    acc[q][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, acc[q][1], 0, 0, 0);
                                }
                            }
                        }
                    }
                    // lane holds state nb + 16 q + hi + 4 v of orbitals ja and jb
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int nn = nb + 16 * q + hi + 4 * v;
                            if (q < nts && nn < a.S) {
                                double *o = out + (size_t)nn * a.nc;
                                if (ja < jn) o[ja] = have ? o[ja] + acc[q][0][v] : acc[q][0][v];
                                if (jb < jn) o[jb] = have ? o[jb] + acc[q][1][v] : acc[q][1][v];
                            }
                        }
                }
            }
            have = true;
        }
    }
    if (!have) {
        // no terms: the row of the block is zero
        for (int e = threadIdx.x; e < a.S * jn; e += blockDim.x) out[(size_t)(e / jn) * a.nc + e % jn] = 0.0;
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
    const dim3 g(n_l2, (a.nc + C4_JB - 1) / C4_JB), b(256);
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
