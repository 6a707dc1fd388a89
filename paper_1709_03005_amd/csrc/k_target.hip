// Target-space pieces of the continuum-continuum blocks (classes 1, 3, 5,
// 6, 7; Sec. 2.1-2.2 and Eq. 8):
//   * Slater-Condon values H_T[m, m'] of the connected target pairs;
//   * the CI projection (C_i^T H_T C_i')_{nn'} and overlap (C_i^T O C_i')_{nn'}
//     as a row-wise sparse product followed by a small dense product;
//   * the contracted symbolic coefficients D^beta of Eq. 8 for the integral
//     labels (P Q | j j') and (P j' | j Q): spin-summed and alpha-resolved
//     transition densities Gamma_{nn',PQ} = sum_mm' c_imn c_i'm'n' <m|E_PQ|m'>,
//     accumulated per label from the pairs bucketed by label (deterministic).
#include "ccham_internal.h"

namespace cch {

// ---------------------------------------------------------------------------
// H_T values of the connected pairs
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(256) void k_pair_values(TgtInts I, const uint64_t *__restrict__ da,
                                                     const uint64_t *__restrict__ db, PairList pl,
                                                     int64_t n, double *__restrict__ hv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int deg = pl.deg[i];
    const uint64_t lab = pl.label[i];
    int h[2] = {lab_field(lab, 1), lab_field(lab, 3)};
    int p[2] = {lab_field(lab, 0), lab_field(lab, 2)};
    uint64_t A[W], B[W];
    int dm = 0;   // alpha electrons of the bra minus those of the ket
#pragma unroll
    for (int w = 0; w < W; ++w) {
        A[w] = da[(size_t)pl.x[i] * W + w];
        B[w] = db[(size_t)pl.y[i] * W + w];
        dm += __popcll(A[w] & 0x5555555555555555ull) - __popcll(B[w] & 0x5555555555555555ull);
    }
    // target determinants of different M_S (given with continuum electrons of
    // different spin): the spin-free H_T has no element between them
    hv[i] = dm ? 0.0 : sc_value<W>(I, A, B, deg, h, p, pl.phase[i]);
}

hipError_t launch_pair_values(int W, TgtInts I, const uint64_t *da, const uint64_t *db, PairList pl,
                              int64_t n, double *hv, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    switch (W) {
    case 1: hipLaunchKernelGGL((k_pair_values<1>), g, b, 0, st, I, da, db, pl, n, hv); break;
    case 2: hipLaunchKernelGGL((k_pair_values<2>), g, b, 0, st, I, da, db, pl, n, hv); break;
    case 3: hipLaunchKernelGGL((k_pair_values<3>), g, b, 0, st, I, da, db, pl, n, hv); break;
    case 4: hipLaunchKernelGGL((k_pair_values<4>), g, b, 0, st, I, da, db, pl, n, hv); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Y[m][n'] = sum_{pairs (m, m')} H_T[m,m'] c'[m'][n'],  Yo = same over
// degree-0 pairs with weight 1. One wave per bra row, pairs in order.
// ---------------------------------------------------------------------------
// Y[m][n] = sum over the connected pairs p of row m of hv[p] cb[y_p][n]
// (Yo likewise with weight 1 on degree-0 pairs): one wave per row m, its lanes
// split into G pair groups x (64 / G) states; the G partial sums of a state
// are combined by xor-shuffles over the group bits (fixed order).
__global__ __launch_bounds__(256) void k_spmm_rows(int M, const int64_t *__restrict__ row_off,
                                                   const int64_t *__restrict__ row_cnt, PairList pl,
                                                   const double *__restrict__ hv,
                                                   const double *__restrict__ cb, int Sb, int lg_states,
                                                   double *__restrict__ Y, double *__restrict__ Yo)
{
    const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (m >= M) return;   // whole waves
    const int ns = 1 << lg_states;              // state lanes (power of two, <= 64)
    const int ng = 64 >> lg_states;             // pair groups
    const int nl = lane & (ns - 1), g = lane >> lg_states;
    const int64_t p0 = row_off[m], p1 = p0 + row_cnt[m];
    for (int n0 = 0; n0 < Sb; n0 += ns) {
        const int n = n0 + nl;
        double acc = 0.0, acco = 0.0;
        if (n < Sb) {
            for (int64_t p = p0 + g; p < p1; p += ng) {
                const double c = cb[(size_t)pl.y[p] * Sb + n];
                acc = fma(hv[p], c, acc);
                if (pl.deg[p] == 0) acco += c;
            }
        }
        for (int o = ns; o < 64; o <<= 1) {
            acc += __shfl_xor(acc, o, 64);
            acco += __shfl_xor(acco, o, 64);
        }
        if (g == 0 && n < Sb) {
            Y[(size_t)m * Sb + n] = acc;
            Yo[(size_t)m * Sb + n] = acco;
        }
    }
}

// HT[r] = sum_m ca[m][na[r]] Y[m][nb[r]],  O[r] likewise with Yo.
__global__ __launch_bounds__(256) void k_project(int M, const double *__restrict__ ca, int Sa,
                                                 const double *__restrict__ Y,
                                                 const double *__restrict__ Yo, int Sb,
                                                 const int32_t *__restrict__ rn,
                                                 const int32_t *__restrict__ rn2,
                                                 double *__restrict__ HT, double *__restrict__ O)
{
    const int r = blockIdx.x;
    const int n = rn[r], n2 = rn2[r];
    double a = 0.0, b = 0.0;
    for (int m = threadIdx.x; m < M; m += 256) {
        const double c = ca[(size_t)m * Sa + n];
        a = fma(c, Y[(size_t)m * Sb + n2], a);
        b = fma(c, Yo[(size_t)m * Sb + n2], b);
    }
    __shared__ double ra[256], rb[256];
    ra[threadIdx.x] = a;
    rb[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            ra[threadIdx.x] += ra[threadIdx.x + o];
            rb[threadIdx.x] += rb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        HT[r] = ra[0];
        O[r] = rb[0];
    }
}

// Target energies on the diagonal (Sec. 3.1, classes 1, 3, 5, 6 and 7): the
// target-only part of every state row (n, n') is replaced by delta_nn' E[n]
// for a symmetry with itself (E given) and by zero between two symmetries.
__global__ __launch_bounds__(256) void k_energy_rows(int nrows, const int32_t *__restrict__ rn,
                                                     const int32_t *__restrict__ rn2,
                                                     const double *__restrict__ E, double *__restrict__ HT)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < nrows) HT[r] = (E != nullptr && rn[r] == rn2[r]) ? E[rn[r]] : 0.0;
}

hipError_t launch_energy_rows(int nrows, const int32_t *rn, const int32_t *rn2, const double *E, double *HT,
                              hipStream_t st)
{
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_energy_rows, dim3((nrows + 255) / 256), dim3(256), 0, st, nrows, rn, rn2, E, HT);
    return hipGetLastError();
}

hipError_t launch_projection(int M, const int64_t *row_off, const int64_t *row_cnt, PairList pl,
                             const double *hv, const double *ca, int Sa, const double *cb, int Sb,
                             int nrows, const int32_t *rn, const int32_t *rn2, double *Y, double *Yo,
                             double *HT, double *O, hipStream_t st)
{
    if (M > 0) {
        int lg = 0;   // state lanes: the power of two >= Sb, at most 64
        while ((1 << lg) < Sb && lg < 6) ++lg;
        hipLaunchKernelGGL(k_spmm_rows, dim3((M + 3) / 4), dim3(256), 0, st, M, row_off, row_cnt, pl,
                           hv, cb, Sb, lg, Y, Yo);
    }
    hipLaunchKernelGGL(k_project, dim3(nrows), dim3(256), 0, st, M, ca, Sa, Y, Yo, Sb, rn, rn2, HT, O);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// bucketing of pairs by integral label (P, Q): key = slot of a degree-1
// pair; degree-0 pairs are recorded per bra row; degree 2 has no density
// term. Counting sort with a per-bucket ordering by pair index so the
// accumulation order is fixed.
// ---------------------------------------------------------------------------
__global__ void k_slot_count(PairList pl, int64_t n, const int32_t *__restrict__ pqidx, int n_o,
                             int32_t *__restrict__ key, int64_t *__restrict__ count,
                             int64_t *__restrict__ d0)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int d = pl.deg[i];
    int k = -1;
    if (d == 1) {
        const uint64_t lab = pl.label[i];
        const int P = lab_field(lab, 0) >> 1, Q = lab_field(lab, 1) >> 1;
        k = pqidx[P * n_o + Q];
    } else if (d == 0) {
        d0[pl.x[i]] = i;     // distinct determinants: at most one per bra row
    }
    key[i] = k;
    if (k >= 0) atomicAdd((unsigned long long *)&count[k], 1ull);
}

__global__ void k_slot_scatter(int64_t n, const int32_t *__restrict__ key,
                               const int64_t *__restrict__ start, int64_t *__restrict__ cursor,
                               int64_t *__restrict__ sorted)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = key[i];
    if (k < 0) return;
    const int64_t pos = start[k] + (int64_t)atomicAdd((unsigned long long *)&cursor[k], 1ull);
    sorted[pos] = i;
}

// sort inside each bucket (values are distinct pair indices), one workgroup
// per bucket: chunks of BS_CHUNK sorted in LDS by a bitonic network (padded
// with the largest value), then neighbouring runs merged pass by pass between
// sorted and tmp: an element goes to its index in its own run plus the number
// of the other run's elements below it (binary search). O(n log^2 n) per
// bucket; the result is the ascending order.
constexpr int BS_CHUNK = 512;
__global__ __launch_bounds__(256) void k_bucket_sort(const int64_t *__restrict__ start,
                                                     const int64_t *__restrict__ count,
                                                     int64_t *__restrict__ sorted,
                                                     int64_t *__restrict__ tmp)
{
    __shared__ int64_t buf[BS_CHUNK];
    const int k = blockIdx.x;
    const int64_t s0 = start[k], n = count[k];
    if (n <= 1) return;
    const int64_t big = 0x7fffffffffffffffLL;
    for (int64_t c0 = 0; c0 < n; c0 += BS_CHUNK) {
        const int cn = (int)min((int64_t)BS_CHUNK, n - c0);
        int p2 = 1;
        while (p2 < cn) p2 <<= 1;
        for (int a = threadIdx.x; a < p2; a += 256) buf[a] = a < cn ? sorted[s0 + c0 + a] : big;
        __syncthreads();
        for (int size = 2; size <= p2; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int a = threadIdx.x; a < p2 / 2; a += 256) {
                    const int i = 2 * a - (a & (stride - 1)), jx = i + stride;   // bit `stride` of i clear
                    const bool up = (i & size) == 0;
                    const int64_t x = buf[i], y = buf[jx];
                    if ((x > y) == up) {
                        buf[i] = y;
                        buf[jx] = x;
                    }
                }
                __syncthreads();
            }
        for (int a = threadIdx.x; a < cn; a += 256) sorted[s0 + c0 + a] = buf[a];
        __syncthreads();
    }
    int64_t *src = sorted + s0, *dst = tmp + s0;
    for (int64_t run = BS_CHUNK; run < n; run *= 2) {
        for (int64_t a = threadIdx.x; a < n; a += 256) {
            const int64_t r0 = a / (2 * run) * (2 * run);
            const int64_t mid = min(n, r0 + run), end = min(n, r0 + 2 * run);
            const int64_t v = src[a];
            int64_t lo = mid, hi = end, pos = a - r0;   // v in the left run: count the right run's smaller
            if (a >= mid) {
                lo = r0;
                hi = mid;
                pos = a - mid;
            }
            const int64_t base = lo;
            while (lo < hi) {
                const int64_t m = (lo + hi) / 2;
                if (src[m] < v) lo = m + 1;
                else hi = m;
            }
            dst[r0 + pos + (lo - base)] = v;
        }
        __syncthreads();
        int64_t *t = src;
        src = dst;
        dst = t;
    }
    if (src != sorted + s0) {
        for (int64_t a = threadIdx.x; a < n; a += 256) sorted[s0 + a] = src[a];
    }
}

hipError_t launch_bucket(PairList pl, int64_t n, const int32_t *pqidx, int n_o, int n_slot, int M,
                         int32_t *key, int64_t *count, int64_t *start, int64_t *cursor,
                         int64_t *sorted, int64_t *tmp, int64_t *d0, hipStream_t st)
{
    hipError_t e;
    if ((e = launch_fill_i64(count, 0, n_slot + 1, st)) != hipSuccess) return e;
    if ((e = launch_fill_i64(cursor, 0, n_slot + 1, st)) != hipSuccess) return e;
    if ((e = launch_fill_i64(d0, -1, M, st)) != hipSuccess) return e;
    if (n > 0) {
        const dim3 g((unsigned)((n + 255) / 256));
        hipLaunchKernelGGL(k_slot_count, g, dim3(256), 0, st, pl, n, pqidx, n_o, key, count, d0);
        if ((e = launch_exclusive_scan(count, start, n_slot, nullptr, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_slot_scatter, g, dim3(256), 0, st, n, key, start, cursor, sorted);
        hipLaunchKernelGGL(k_bucket_sort, dim3(n_slot), dim3(256), 0, st, start, count, sorted, tmp);
    } else {
        if ((e = launch_exclusive_scan(count, start, n_slot, nullptr, st)) != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gamma: one workgroup per label slot k = (P, Q).
//   J[r] = sum over degree-1 pairs with label (P,Q) of s c_a[m][n] c_b[m'][n']
//          (+ for P == Q the degree-0 pairs weighted by the occupation of P)
//   K[r] = the exchange weights: excitations from a hole of the bra's continuum
//          spin to a particle of the ket's (alpha -> alpha when both continuum
//          electrons are alpha) / occupation of P with the continuum spin.
// Output Kt-major: At[k][r] = J, At[n_slot + k][r] = K.
// ---------------------------------------------------------------------------
constexpr int GAM_BATCH = 16;
constexpr int GAM_RPT = 8;      // rows per thread per pass

template <int W>
__global__ __launch_bounds__(256) void k_gamma(PairList pl, const int64_t *__restrict__ start,
                                               const int64_t *__restrict__ count,
                                               const int64_t *__restrict__ sorted,
                                               const int64_t *__restrict__ d0, int M0,
                                               const int32_t *__restrict__ slotP,
                                               const int32_t *__restrict__ slotQ, int n_slot,
                                               const uint64_t *__restrict__ da,
                                               const int8_t *__restrict__ spa,
                                               const int8_t *__restrict__ spb,
                                               const double *__restrict__ ca, int Sa,
                                               const double *__restrict__ cb, int Sb, int nrows,
                                               const int32_t *__restrict__ rn,
                                               const int32_t *__restrict__ rn2,
                                               double *__restrict__ At)
{
    extern __shared__ double sh[];
    double *sa = sh;                            // [GAM_BATCH][Sa]
    double *sb = sh + GAM_BATCH * Sa;           // [GAM_BATCH][Sb]
    __shared__ double wj[GAM_BATCH], wk[GAM_BATCH];
    const int k = blockIdx.x;
    const int P = slotP[k], Q = slotQ[k];
    const int64_t s1 = start[k], n1 = count[k];
    const int64_t n0 = (P == Q) ? M0 : 0;
    const int64_t ntot = n1 + n0;

    for (int rbase = 0; rbase < nrows; rbase += 256 * GAM_RPT) {
        double J[GAM_RPT], K[GAM_RPT];
#pragma unroll
        for (int q = 0; q < GAM_RPT; ++q) J[q] = K[q] = 0.0;
        for (int64_t e0 = 0; e0 < ntot; e0 += GAM_BATCH) {
            const int ne = (int)min<int64_t>(GAM_BATCH, ntot - e0);
            __syncthreads();
            // stage weights and CI rows of this batch
            for (int t = threadIdx.x; t < ne; t += 256) {
                const int64_t e = e0 + t;
                const int64_t pidx = e < n1 ? sorted[s1 + e] : d0[e - n1];
                double a = 0.0, b = 0.0;
                if (pidx < 0) {
                    // no identical ket for this bra row
                } else if (e < n1) {
                    // particle p (in the bra), hole q (in the ket); the Coulomb weight
                    // needs equal continuum spins and a spin-conserving excitation, the
                    // exchange weight a particle of the ket's continuum spin and a hole
                    // of the bra's (the spin-flip pairs of doublet-coupled triplets)
                    const int s = pl.phase[pidx];
                    const uint64_t lab = pl.label[pidx];
                    const int sp = lab_field(lab, 0) & 1, sq = lab_field(lab, 1) & 1;
                    const int sx = spa ? spa[pl.x[pidx]] : 0, sy = spb ? spb[pl.y[pidx]] : 0;
                    a = (sx == sy && sp == sq) ? (double)s : 0.0;
                    b = (sp == sy && sq == sx) ? (double)s : 0.0;
                } else {
                    // occupation of spatial orbital P in the bra determinant (both spins;
                    // the continuum spin's for the exchange weight)
                    const uint64_t *d = da + (size_t)pl.x[pidx] * W;
                    const int ka = 2 * P, kb = 2 * P + 1;
                    const int oa = (int)((d[ka >> 6] >> (ka & 63)) & 1ull);
                    const int ob = (int)((d[kb >> 6] >> (kb & 63)) & 1ull);
                    const int sx = spa ? spa[pl.x[pidx]] : 0;
                    a = (double)(oa + ob);
                    b = (double)(sx ? ob : oa);
                }
                wj[t] = a;
                wk[t] = b;
            }
            for (int t = threadIdx.x; t < ne * Sa; t += 256) {
                const int ee = t / Sa, n = t % Sa;
                const int64_t e = e0 + ee;
                const int64_t pidx = e < n1 ? sorted[s1 + e] : d0[e - n1];
                sa[ee * Sa + n] = pidx < 0 ? 0.0 : ca[(size_t)pl.x[pidx] * Sa + n];
            }
            for (int t = threadIdx.x; t < ne * Sb; t += 256) {
                const int ee = t / Sb, n = t % Sb;
                const int64_t e = e0 + ee;
                const int64_t pidx = e < n1 ? sorted[s1 + e] : d0[e - n1];
                sb[ee * Sb + n] = pidx < 0 ? 0.0 : cb[(size_t)pl.y[pidx] * Sb + n];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < GAM_RPT; ++q) {
                const int r = rbase + threadIdx.x + 256 * q;
                if (r < nrows) {
                    const int n = rn[r], n2 = rn2[r];
                    double j = J[q], kk = K[q];
                    for (int ee = 0; ee < ne; ++ee) {
                        const double cc = sa[ee * Sa + n] * sb[ee * Sb + n2];
                        j = fma(wj[ee], cc, j);
                        kk = fma(wk[ee], cc, kk);
                    }
                    J[q] = j;
                    K[q] = kk;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < GAM_RPT; ++q) {
            const int r = rbase + threadIdx.x + 256 * q;
            if (r < nrows) {
                At[(size_t)k * nrows + r] = J[q];
                At[(size_t)(n_slot + k) * nrows + r] = K[q];
            }
        }
    }
}

hipError_t launch_gamma(int W, PairList pl, const int64_t *start, const int64_t *count,
                        const int64_t *sorted, const int64_t *d0, int M0, const int32_t *slotP, const int32_t *slotQ, int n_slot,
                        const uint64_t *da, const int8_t *spa, const int8_t *spb, const double *ca, int Sa,
                        const double *cb, int Sb, int nrows, const int32_t *rn, const int32_t *rn2, double *At,
                        hipStream_t st)
{
    if (n_slot <= 0 || nrows <= 0) return hipSuccess;
    const size_t shm = sizeof(double) * GAM_BATCH * (size_t)(Sa + Sb);
    const dim3 g(n_slot), b(256);
    switch (W) {
    case 1: hipLaunchKernelGGL((k_gamma<1>), g, b, shm, st, pl, start, count, sorted, d0, M0, slotP, slotQ, n_slot, da, spa, spb, ca, Sa, cb, Sb, nrows, rn, rn2, At); break;
    case 2: hipLaunchKernelGGL((k_gamma<2>), g, b, shm, st, pl, start, count, sorted, d0, M0, slotP, slotQ, n_slot, da, spa, spb, ca, Sa, cb, Sb, nrows, rn, rn2, At); break;
    case 3: hipLaunchKernelGGL((k_gamma<3>), g, b, shm, st, pl, start, count, sorted, d0, M0, slotP, slotQ, n_slot, da, spa, spb, ca, Sa, cb, Sb, nrows, rn, rn2, At); break;
    case 4: hipLaunchKernelGGL((k_gamma<4>), g, b, shm, st, pl, start, count, sorted, d0, M0, slotP, slotQ, n_slot, da, spa, spb, ca, Sa, cb, Sb, nrows, rn, rn2, At); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace cch
