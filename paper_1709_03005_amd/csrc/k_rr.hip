// Rayleigh-Ritz eigenproblem of the Davidson solver (Sec. 3.2 lists
// Davidson among the diagonalisers): G (m x m, symmetric, m <= 96) ->
// ascending theta and orthonormal eigenvectors Y (column e at Y[q*ldy + e]),
// FP64, one workgroup, all of it in LDS.
//
// k_rr_eig, the main path:
//   1. G is scaled by a power of two and reduced to tridiagonal form
//      T = Q^T G Q by Householder reflectors (kept below the subdiagonal);
//   2. every eigenvalue of T by multisection: Sturm counts from the
//      leading-minor recurrence (rescaled by powers of two) at many shifts
//      at once, one thread per shift;
//   3. one eigenvector of T per thread from the twisted factorisation of
//      T - lambda I at the twist index of smallest |gamma|;
//   4. modified Gram-Schmidt (two passes) inside clusters of eigenvalues
//      closer than 1e-3 ||T||, then the reflectors applied to the vectors;
//   5. one Newton-Schulz step Y <- Y (3I - Y^T Y) / 2 on FP64 MFMA, which
//      takes the orthogonality defect from ~1e-13 to rounding level.
// A failed check (a non-finite value, a twisted residual above 1e-10 ||T||,
// a cluster vector that loses 99% of its norm to the projections, or a
// defect above 1e-8 before the Newton-Schulz step, as with exactly
// repeated eigenvalues) reruns the problem by cyclic Jacobi in the same
// launch and counts the event. k_jacobi_eig is the Jacobi path alone.
#include <cfloat>

#include "ccham_internal.h"

namespace cch {

constexpr int RR_MAX = 96, RR_LD = RR_MAX + 1, RR_NT = 512, RR_NW = RR_NT / 64;
typedef double rr_dx4 __attribute__((ext_vector_type(4)));

constexpr int RR_SL = 4;     // row slices of the Householder products (x 2 column halves = 8 waves)
constexpr int RR_G = 512;    // shifts of the first multisection pass

struct RRShared {
    double A[RR_MAX][RR_LD];
    double Z[RR_MAX][RR_LD];
    double d[RR_MAX], e[RR_MAX], lam[RR_MAX], tau[RR_MAX], hinv[RR_MAX];
    double sc[6][RR_MAX];        // per-phase scratch vectors
    double red[2][32];           // alternating reduction buffers
    union {
        int cnt[RR_NT];                  // Sturm counts; Jacobi pairing tables
        double dbl[RR_NT / 2];           // 16 x 16 Gram matrix of a reflector block
    } u;
    unsigned long long open_mask[2];   // eigenvalues still bracketed (multisection)
    int flag, nrot;
};
static_assert(sizeof(RRShared) <= 160 * 1024, "LDS budget");

__device__ __forceinline__ double rr_wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double rr_wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block reductions with one barrier: consecutive calls must alternate the
// buffer, so that a buffer is written again only after a later barrier.
__device__ __forceinline__ double rr_block_sum(double v, double *red)
{
    v = rr_wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

__device__ __forceinline__ double rr_block_max(double v, double *red)
{
    v = rr_wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, red[w]);
    return s;
}

// Cross-lane helpers on doubles as two 32-bit halves: DPP moves (row shifts
// and row broadcasts) and readlane with a wave-uniform lane index.
struct RrI2 {
    int x, y;
};

template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ double rr_dpp(double v)
{
    RrI2 a = __builtin_bit_cast(RrI2, v);
    a.x = __builtin_amdgcn_update_dpp(0, a.x, CTRL, ROW_MASK, BANK_MASK, true);
    a.y = __builtin_amdgcn_update_dpp(0, a.y, CTRL, ROW_MASK, BANK_MASK, true);
    return __builtin_bit_cast(double, a);
}

__device__ __forceinline__ double rr_rl(double v, int lane)
{
    RrI2 a = __builtin_bit_cast(RrI2, v);
    a.x = __builtin_amdgcn_readlane(a.x, lane);
    a.y = __builtin_amdgcn_readlane(a.y, lane);
    return __builtin_bit_cast(double, a);
}

// sum over the 64 lanes, returned to every lane: partial sums of 4 within
// each row of 16 (row_shr 1..3), of 8 and 16 (row_shr 4, 8 on the upper
// banks), then rows 0+1 and 2+3 (row_bcast15) and all four (row_bcast31)
// collect in lane 63. Fixed order, so every wave gets the same bits.
__device__ __forceinline__ double rr_wsum(double v)
{
    double s = v + rr_dpp<0x111, 0xf, 0xf>(v);
    s += rr_dpp<0x112, 0xf, 0xf>(v);
    s += rr_dpp<0x113, 0xf, 0xf>(v);
    s += rr_dpp<0x114, 0xf, 0xe>(s);
    s += rr_dpp<0x118, 0xf, 0xc>(s);
    s += rr_dpp<0x142, 0xa, 0xf>(s);
    s += rr_dpp<0x143, 0xc, 0xf>(s);
    return rr_rl(s, 63);
}

// element i (wave-uniform, < 128) of a vector held as lo = x[lane], hi = x[lane + 64]
__device__ __forceinline__ double rr_get(double lo, double hi, int i)
{
    return i < 64 ? rr_rl(lo, i) : rr_rl(hi, i - 64);
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi, parallel (round-robin tournament) ordering: m/2 disjoint
// rotations per round, m-1 rounds per sweep; a rotation is skipped when
// |a_pq| <= 1e-16 sqrt(|a_pp a_qq|), and the sweeps stop after one with no
// rotation. Reads G itself (unscaled) and writes theta and Y.
// 1/q from the hardware estimate and two Newton-Raphson corrections
// r <- r + r (1 - q r), each squaring the relative error: a short dependent
// chain for the recurrences below, within about one ulp of the quotient
__device__ __forceinline__ double rr_recip(double q)
{
    double r = __builtin_amdgcn_rcp(q);
    double e = fma(-q, r, 1.0);
    r = fma(r, e, r);
    e = fma(-q, r, 1.0);
    return fma(r, e, r);
}

// 1/sqrt(x), x > 0, from the hardware estimate and two Newton-Raphson
// corrections r <- r + r (1 - x r^2) / 2
__device__ __forceinline__ double rr_rsqrt(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    double e = fma(-x * r, r, 1.0);
    r = fma(0.5 * r, e, r);
    e = fma(-x * r, r, 1.0);
    return fma(0.5 * r, e, r);
}

// a value every lane holds alike (read from LDS), as a wave-uniform scalar
__device__ __forceinline__ double rr_uni(double v)
{
    RrI2 a = __builtin_bit_cast(RrI2, v);
    a.x = __builtin_amdgcn_readfirstlane(a.x);
    a.y = __builtin_amdgcn_readfirstlane(a.y);
    return __builtin_bit_cast(double, a);
}

// ---------------------------------------------------------------------------
__device__ void rr_jacobi(RRShared &sh, const double *__restrict__ G, int ldg, int m, double *__restrict__ theta,
                          double *__restrict__ Y, int ldy, int max_sweeps)
{
    double(*A)[RR_LD] = sh.A;
    double(*Z)[RR_LD] = sh.Z;
    double *cs = sh.sc[3], *sn = sh.sc[4];
    int *pp = sh.u.cnt, *qq = sh.u.cnt + RR_MAX / 2, *perm = sh.u.cnt + RR_MAX;
    const int me = (m + 1) & ~1;     // even size (a padded index is inert)
    const int half = me / 2;
    const int nthr = blockDim.x;
    __syncthreads();
    for (int t = threadIdx.x; t < me * me; t += nthr) {
        const int i = t / me, j = t % me;
        A[i][j] = (i < m && j < m) ? 0.5 * (G[(int64_t)i * ldg + j] + G[(int64_t)j * ldg + i]) : 0.0;
        Z[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (threadIdx.x == 0) sh.nrot = 0;
        __syncthreads();
        for (int round = 0; round < me - 1; ++round) {
            if (threadIdx.x < half) {
                const int k = threadIdx.x;
                const int s0 = k, s1 = me - 1 - k;
                int p = s0 == 0 ? 0 : 1 + (s0 - 1 + round) % (me - 1);
                int q = 1 + (s1 - 1 + round) % (me - 1);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                pp[k] = p;
                qq[k] = q;
                const double apq = A[p][q];
                double c = 1.0, s = 0.0;
                if (fabs(apq) > 1e-16 * sqrt(fabs(A[p][p] * A[q][q])) && fabs(apq) > 1e-300) {
                    sh.nrot = 1;
                    const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                cs[k] = c;
                sn[k] = s;
            }
            __syncthreads();
            // A <- J^T A J on 2x2 blocks (row pair k, column pair l), Z <- Z J
            const int nblk = half * half;
            for (int t = threadIdx.x; t < nblk + half * me; t += nthr) {
                if (t < nblk) {
                    const int k = t / half, l = t % half;
                    const int p = pp[k], q = qq[k], r = pp[l], u = qq[l];
                    const double ck = cs[k], sk = sn[k], cl = cs[l], sl = sn[l];
                    const double apr = A[p][r], apu = A[p][u], aqr = A[q][r], aqu = A[q][u];
                    const double bpr = ck * apr - sk * aqr, bpu = ck * apu - sk * aqu;
                    const double bqr = sk * apr + ck * aqr, bqu = sk * apu + ck * aqu;
                    A[p][r] = cl * bpr - sl * bpu;
                    A[p][u] = sl * bpr + cl * bpu;
                    A[q][r] = cl * bqr - sl * bqu;
                    A[q][u] = sl * bqr + cl * bqu;
                } else {
                    const int e = t - nblk;
                    const int l = e / me, i = e % me;
                    const int r = pp[l], u = qq[l];
                    const double cl = cs[l], sl = sn[l];
                    const double zr = Z[i][r], zu = Z[i][u];
                    Z[i][r] = cl * zr - sl * zu;
                    Z[i][u] = sl * zr + cl * zu;
                }
            }
            __syncthreads();
        }
        if (sh.nrot == 0) break;
        __syncthreads();
    }
    // ascending order (stable), written out
    if (threadIdx.x == 0) {
        for (int i = 0; i < m; ++i) perm[i] = i;
        for (int i = 1; i < m; ++i) {
            const int v = perm[i];
            int j = i - 1;
            while (j >= 0 && A[perm[j]][perm[j]] > A[v][v]) {
                perm[j + 1] = perm[j];
                --j;
            }
            perm[j + 1] = v;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += nthr) theta[e] = A[perm[e]][perm[e]];
    for (int t = threadIdx.x; t < m * m; t += nthr) {
        const int q = t / m, e = t % m;
        Y[(int64_t)q * ldy + e] = Z[q][perm[e]];
    }
}

__global__ __launch_bounds__(RR_NT) void k_jacobi_eig(const double *__restrict__ G, int ldg, int m,
                                                      double *__restrict__ theta, double *__restrict__ Y, int ldy,
                                                      int max_sweeps)
{
    __shared__ RRShared sh;
    rr_jacobi(sh, G, ldg, m, theta, Y, ldy, max_sweeps);
}

// Sturm count: eigenvalues of T below x, from the signs of the leading
// principal minors of T - xI (p_{i+1} = (d_i - x) p_i - e_{i-1}^2 p_{i-1});
// an exact zero minor counts as negative. d and e^2 come from registers
// (d_i in lane i of dl0 / dl1, e_i^2 in lane i of ql0 / ql1). The pair
// (p_i, p_{i-1}) is rescaled by 2^-+500 every fourth step: T is scaled to
// entries below 2 and couplings below eps (|d_i| + |d_{i+1}|) are zeroed,
// so four steps can neither overflow nor underflow from [2^-500, 2^500].
__device__ __forceinline__ int rr_sturm(double dl0, double dl1, double ql0, double ql1, int n, double x)
{
    double pp = 1.0, p = rr_rl(dl0, 0) - x;
    p = (p == 0.0) ? -DBL_MIN : p;
    int c = p < 0.0;
    auto step = [&](int i, double di, double qi) {
        double q = fma(di - x, p, -(qi * pp));
        q = (q == 0.0) ? (p > 0.0 ? -DBL_MIN : DBL_MIN) : q;
        c += (q < 0.0) != (p < 0.0);
        pp = p;
        p = q;
        if ((i & 3) == 0) {
            const double mx = fmax(fabs(p), fabs(pp));
            const double f = mx > 0x1p+500 ? 0x1p-500 : (mx < 0x1p-500 ? 0x1p+500 : 1.0);
            p *= f;
            pp *= f;
        }
    };
    const int n0 = n < 64 ? n : 64;
    int i = 1;
    for (; i < n0; ++i) step(i, rr_rl(dl0, i), rr_rl(ql0, i - 1));
    if (i < n) {
        step(i, rr_rl(dl1, 0), rr_rl(ql0, 63));
        for (++i; i < n; ++i) step(i, rr_rl(dl1, i - 64), rr_rl(ql1, i - 65));
    }
    return c;
}

__global__ __launch_bounds__(RR_NT) void k_rr_eig(const double *__restrict__ G, int ldg, int m,
                                                  double *__restrict__ theta, double *__restrict__ Y, int ldy,
                                                  int32_t *__restrict__ nfallback)
{
    __shared__ RRShared sh;
    double(*A)[RR_LD] = sh.A;
    double(*Z)[RR_LD] = sh.Z;
    const int tid = threadIdx.x, lane = tid & 63;
    // the wave index as a scalar: loops over row slices are then uniform, so
    // readlane takes its index from an SGPR and the loops can be pipelined
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = m;
    int rp = 0;
    auto bmax = [&](double v) {
        const double r = rr_block_max(v, sh.red[rp]);
        rp ^= 1;
        return r;
    };

    // ---- load, symmetrise, scale by a power of two --------------------------
    if (tid == 0) sh.flag = 0;
    double amax = 0.0;
    for (int t = tid; t < RR_MAX * RR_MAX; t += RR_NT) {
        const int i = t / RR_MAX, j = t % RR_MAX;
        double v = 0.0;
        if (i < n && j < n) v = 0.5 * (G[(int64_t)i * ldg + j] + G[(int64_t)j * ldg + i]);
        A[i][j] = v;
        Z[i][j] = 0.0;
        amax = fmax(amax, fabs(v));
    }
    amax = bmax(amax);
    if (amax == 0.0) {
        for (int e = tid; e < n; e += RR_NT) theta[e] = 0.0;
        for (int t = tid; t < n * n; t += RR_NT) Y[(int64_t)(t / n) * ldy + t % n] = (t / n == t % n) ? 1.0 : 0.0;
        return;
    }
    bool bad = !isfinite(amax);
    const double scale = bad ? 1.0 : ldexp(1.0, -ilogb(amax));
    for (int t = tid; t < n * RR_MAX; t += RR_NT) {
        const int i = t / RR_MAX, j = t % RR_MAX;
        A[i][j] *= scale;
    }
    __syncthreads();

    if (!bad) {
        // ---- Householder reduction to tridiagonal form ------------------------
        // Step k: x = row k of the trailing matrix, H_k = I - tau v v^T with
        // v_{k+1} = 1 and v_r = x_r * hinv[k] below; row k keeps x afterwards.
        // Thread (wave w, lane l) owns column c = l + 64 (w & 1) over the rows
        // k+1+s, k+1+s+RR_SL, ... of slice s = w >> 1. Broadcast operands (x_r,
        // v_r, w_r) are LDS reads at one address per wave, not lane reads; wave 0
        // alone forms sigma, beta, tau and hinv, which the others read after the
        // barrier; each wave keeps its own copy of v and w (rows of Z, free here),
        // so no barrier separates writing them from reading them. A lane whose
        // column is not updated stores into the padding column RR_MAX. Up to 64
        // columns the 8 waves are 8 row slices over one column half.
        {
            const int nsl = n <= 64 ? 2 * RR_SL : RR_SL;
            const int half = n <= 64 ? 0 : wv & 1, slice = n <= 64 ? wv : wv >> 1;
            const int col = lane + 64 * half;
            const int cc = col < RR_MAX ? col : RR_MAX - 1;   // in-bounds column for loads
            double *vw = &Z[2 * RR_SL + 2 * wv][0];             // this wave's v (then w at +RR_LD)
            for (int k = 0; k + 2 < n; ++k) {
                const double x0 = lane < n ? A[k][lane] : 0.0;
                const double x1 = lane + 64 < n ? A[k][lane + 64] : 0.0;
                // row k+1 before the barrier: other waves update it afterwards
                const double y0 = lane < n ? A[k + 1][lane] : 0.0;
                const double y1 = lane + 64 < n ? A[k + 1][lane + 64] : 0.0;
                const bool act = col < n && col >= k + 1;
                const int cst = act ? col : RR_MAX;   // store column
                // partial S_c = sum over this slice's rows r >= k+2 of A[r][c] x_r
                {
                    double s0 = 0.0, s1 = 0.0;
                    int r = k + 2 + slice;
                    for (; r + nsl < n; r += 2 * nsl) {
                        s0 = fma(A[r][cc], A[k][r], s0);
                        s1 = fma(A[r + nsl][cc], A[k][r + nsl], s1);
                    }
                    if (r < n) s0 = fma(A[r][cc], A[k][r], s0);
                    Z[slice][col < RR_MAX ? col : RR_MAX] = act ? s0 + s1 : 0.0;
                }
                if (wv == 0) {
                    const double sig =
                        rr_wsum((lane >= k + 2 ? x0 * x0 : 0.0) + (lane + 64 >= k + 2 ? x1 * x1 : 0.0));
                    const double alpha = rr_get(x0, x1, k + 1);
                    if (lane == 0) {
                        if (sig == 0.0) {
                            sh.tau[k] = 0.0;
                            sh.e[k] = alpha;
                            sh.hinv[k] = 0.0;
                        } else {
                            // short dependent chain: sqrt and the two quotients from the
                            // refined hardware estimates (about one ulp each)
                            const double s2 = fma(alpha, alpha, sig);
                            const double beta = -copysign(s2 * rr_rsqrt(s2), alpha);
                            sh.tau[k] = fma(-alpha, rr_recip(beta), 1.0);   // (beta - alpha) / beta
                            sh.e[k] = beta;
                            sh.hinv[k] = rr_recip(alpha - beta);
                        }
                    }
                }
                __syncthreads();
                const double t = rr_uni(sh.tau[k]);
                if (t == 0.0) {   // no reflection: row k+1 stays; nothing read Z
                    continue;
                }
                const double inv = rr_uni(sh.hinv[k]);
                const double v0 = lane == k + 1 ? 1.0 : (lane >= k + 2 ? x0 * inv : 0.0);
                const double v1 = lane + 64 == k + 1 ? 1.0 : (lane + 64 >= k + 2 ? x1 * inv : 0.0);
                // p_c = t (A[k+1][c] + inv S_c): v_{k+1} = 1, v_r = x_r inv below
                double p0 = 0.0, p1 = 0.0;
                for (int q = 0; q < nsl; ++q) {
                    p0 += Z[q][lane];
                    p1 += Z[q][lane + 64 < RR_MAX ? lane + 64 : RR_MAX];
                }
                p0 = lane < n ? t * fma(inv, p0, y0) : 0.0;
                p1 = lane + 64 < n ? t * fma(inv, p1, y1) : 0.0;
                const double K = 0.5 * t * rr_wsum(p0 * v0 + p1 * v1);
                const double w0 = p0 - K * v0, w1 = p1 - K * v1;
                vw[lane] = v0;
                vw[RR_LD + lane] = w0;
                if (lane + 64 < RR_MAX) {
                    vw[lane + 64] = v1;
                    vw[RR_LD + lane + 64] = w1;
                }
                // A' -= v w^T + w v^T on this thread's column and slice; loads and
                // stores through one column index (idle lanes: the padding column),
                // four rows loaded before any is stored
                {
                    const double vc = half ? v1 : v0, wc = half ? w1 : w0;
                    int r = k + 1 + slice;
                    for (; r + 3 * nsl < n; r += 4 * nsl) {
                        double a[4], vr[4], wr[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            a[u] = A[r + u * nsl][cst];
                            vr[u] = vw[r + u * nsl];
                            wr[u] = vw[RR_LD + r + u * nsl];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) A[r + u * nsl][cst] = a[u] - (vr[u] * wc + wr[u] * vc);
                    }
                    for (; r < n; r += nsl) A[r][cst] = A[r][cst] - (vw[r] * wc + vw[RR_LD + r] * vc);
                }
                __syncthreads();
            }
        }
        for (int i = tid; i < n; i += RR_NT) sh.d[i] = A[i][i];
        if (tid == 0 && n >= 2) sh.e[n - 2] = A[n - 2][n - 1];
        __syncthreads();
        for (int t = tid; t < RR_MAX * RR_MAX; t += RR_NT) Z[t / RR_MAX][t % RR_MAX] = 0.0;
        // negligible couplings split T into independent blocks
        double *e2 = sh.sc[2];
        for (int i = tid; i + 1 < n; i += RR_NT) {
            double ei = sh.e[i];
            if (fabs(ei) <= DBL_EPSILON * (fabs(sh.d[i]) + fabs(sh.d[i + 1]))) ei = 0.0;
            sh.e[i] = ei;
            e2[i] = ei * ei;
        }
        __syncthreads();
        // d and e^2 in registers of every wave (element i in lane i / i - 64)
        const double dl0 = lane < n ? sh.d[lane] : 0.0, dl1 = lane + 64 < n ? sh.d[lane + 64] : 0.0;
        const double ql0 = lane + 1 < n ? e2[lane] : 0.0, ql1 = lane + 65 < n ? e2[lane + 64] : 0.0;

        // ---- eigenvalues by multisection ---------------------------------------
        double glo = INFINITY, ghi = -INFINITY;
        for (int i = tid; i < n; i += RR_NT) {
            const double r = (i > 0 ? fabs(sh.e[i - 1]) : 0.0) + (i + 1 < n ? fabs(sh.e[i]) : 0.0);
            glo = fmin(glo, sh.d[i] - r);
            ghi = fmax(ghi, sh.d[i] + r);
        }
        double gl = -bmax(-glo);
        double gu = bmax(ghi);
        const double tnorm = fmax(fabs(gl), fabs(gu));
        gl -= 2.0 * n * DBL_EPSILON * tnorm + 2.0 * DBL_MIN;
        gu += 2.0 * n * DBL_EPSILON * tnorm + 2.0 * DBL_MIN;
        const double tolabs = 2.0 * DBL_EPSILON * tnorm;
        double *lo = sh.sc[0], *hi = sh.sc[1];
        int *cnt = sh.u.cnt;
        if (tid < RR_G) {   // RR_G shifts over the Gershgorin interval (whole waves)
            const double fr = (double)(tid + 1) / (double)(RR_G + 1);
            cnt[tid] = rr_sturm(dl0, dl1, ql0, ql1, n, fma(gu - gl, fr, gl));
        }
        __syncthreads();
        if (tid < n) {
            // a transition cnt[a] <= j < cnt[b] (virtual ends gl, gu) by bisection on
            // the index; it holds even where rounding makes the counts non-monotone
            int a = -1, b = RR_G;
            while (b - a > 1) {
                const int mid = (a + b) >> 1;
                if (cnt[mid] <= tid) a = mid;
                else b = mid;
            }
            const double l = a < 0 ? gl : fma(gu - gl, (double)(a + 1) / (double)(RR_G + 1), gl);
            const double h = b >= RR_G ? gu : fma(gu - gl, (double)(b + 1) / (double)(RR_G + 1), gl);
            if (!(l < h)) sh.flag = 1;
            lo[tid] = l;
            hi[tid] = h;
            // start of the Laguerre iteration: the idx-th of the k eigenvalues in
            // the interval starts at fraction (idx + 1/2) / k of it
            const int cl = a < 0 ? 0 : cnt[a], ch = b >= RR_G ? n : cnt[b];
            sh.sc[3][tid] = (tid - cl + 0.5) / (double)max(ch - cl, 1);
        }
        __syncthreads();
        // Laguerre's method on det(T - xI) from the middle of each isolating
        // interval (waves 0-1, one eigenvalue per lane): G = P'/P and
        // H = G^2 - P''/P from the pivot recurrences q_i = d_i - x - e_{i-1}^2 / q_{i-1}
        // and their first two derivatives; cubic convergence at simple roots.
        // A step leaving the interval, a non-finite value or no convergence in
        // 16 steps, or a result whose Sturm counts do not bracket index j,
        // leaves the interval to the multisection below.
        if (wv < 2) {
            const int j = tid, jc = j < n ? j : 0;
            const double l0 = lo[jc], h0 = hi[jc], nd = (double)n;
            double x = fma(h0 - l0, fmin(fmax(sh.sc[3][jc], 0.0), 1.0), l0);
            bool conv = j >= n, ok = false;
            for (int it = 0; it < 16; ++it) {
                if (__all(conv)) break;
                double q = rr_rl(dl0, 0) - x;
                q = (q == 0.0) ? -DBL_MIN : q;
                double qp = -1.0, qpp = 0.0, rq = rr_recip(q);
                double Gs = qp * rq, Hs = Gs * Gs;
                auto lag = [&](double di, double e2p) {
                    const double qn = (di - x) - e2p * rq;
                    const double qpn = -1.0 + e2p * qp * rq * rq;
                    const double qppn = e2p * (qpp - 2.0 * qp * qp * rq) * rq * rq;
                    q = (qn == 0.0) ? -DBL_MIN : qn;
                    qp = qpn;
                    qpp = qppn;
                    rq = rr_recip(q);
                    const double t = qp * rq;
                    Gs += t;
                    Hs += t * t - qpp * rq;
                };
                {
                    int i = 1;
                    for (; i < n && i < 64; ++i) lag(rr_rl(dl0, i), rr_rl(ql0, i - 1));
                    if (i < n) lag(rr_rl(dl1, 0), rr_rl(ql0, 63));
                    for (++i; i < n; ++i) lag(rr_rl(dl1, i - 64), rr_rl(ql1, i - 65));
                }
                if (!conv) {
                    const double sq = sqrt(fmax((nd - 1.0) * (nd * Hs - Gs * Gs), 0.0));
                    const double den = fabs(Gs + sq) >= fabs(Gs - sq) ? Gs + sq : Gs - sq;
                    const double a = nd / den;
                    const double xn = x - a;
                    if (!(den != 0.0) || !isfinite(xn) || !(xn >= l0 && xn <= h0)) {
                        conv = true;
                    } else {
                        x = xn;
                        if (fabs(a) <= 2.0 * DBL_EPSILON * tnorm) {
                            conv = true;
                            ok = true;
                        }
                    }
                }
            }
            const double dl = 4.0 * DBL_EPSILON * tnorm;
            const int c1 = rr_sturm(dl0, dl1, ql0, ql1, n, x - dl);
            const int c2 = rr_sturm(dl0, dl1, ql0, ql1, n, x + dl);
            if (j < n && ok && c1 <= j && j < c2) {
                lo[j] = x;
                hi[j] = x;
            }
        }
        // multisection for what Laguerre left: the open eigenvalues (ballot of
        // waves 0-1) share the RR_G shifts, up to 64 each
        auto open = [&](int j) {
            return (hi[j] - lo[j]) > fmax(tolabs, 2.0 * DBL_EPSILON * fmax(fabs(lo[j]), fabs(hi[j])));
        };
        for (int pass = 0; pass < 96; ++pass) {
            __syncthreads();
            if (wv < 2) {
                const unsigned long long mk = __ballot(tid < n && open(tid));
                if (lane == 0) sh.open_mask[wv] = mk;
            }
            __syncthreads();
            const unsigned long long m0 = sh.open_mask[0], m1 = sh.open_mask[1];
            const int c0 = __popcll(m0), na = c0 + __popcll(m1);
            if (na == 0) break;
            const int per = max(2, min(64, RR_G / na));
            const int slot = tid / per, sft = tid % per;
            if (slot < na) {
                // eigenvalue of this slot: the slot-th set bit of (m0, m1)
                unsigned long long mk = slot < c0 ? m0 : m1;
                for (int q = slot < c0 ? slot : slot - c0; q > 0; --q) mk &= mk - 1;
                const int j = __builtin_ctzll(mk) + (slot < c0 ? 0 : 64);
                const double fr = (double)(sft + 1) / (double)(per + 1);
                cnt[tid] = rr_sturm(dl0, dl1, ql0, ql1, n, fma(hi[j] - lo[j], fr, lo[j]));
            }
            __syncthreads();
            if (tid < n && ((tid < 64 ? m0 >> tid : m1 >> (tid - 64)) & 1ull)) {
                const int myslot = tid < 64 ? __popcll(m0 & ((1ull << tid) - 1ull))
                                            : c0 + __popcll(m1 & ((1ull << (tid - 64)) - 1ull));
                const double l0 = lo[tid], h0 = hi[tid];
                double l = l0, h = h0;
                for (int q = 0; q < per; ++q) {
                    const double x = fma(h0 - l0, (double)(q + 1) / (double)(per + 1), l0);
                    if (cnt[myslot * per + q] <= tid) l = fmax(l, x);
                    else h = fmin(h, x);
                }
                lo[tid] = l;
                hi[tid] = h;
            }
        }
        if (tid < n) sh.lam[tid] = 0.5 * (lo[tid] + hi[tid]);
        __syncthreads();

        // ---- eigenvectors of T: twisted factorisations, one per thread ------
        if (wv < 2) {   // d, e, e^2 by readlane: the loops below are wave-uniform
            const int j = tid, jc = j < n ? j : 0;   // jc: in-bounds column for idle lanes
            const double lj = sh.lam[jc];
            // top-down pivots delta+ kept in column j
            double dp = rr_rl(dl0, 0) - lj;
            if (dp == 0.0) dp = -DBL_MIN;
            if (j < n) Z[0][j] = dp;
            auto fwd = [&](int i, double di, double qi) {
                double x = (di - lj) - qi * rr_recip(dp);
                if (x == 0.0) x = -DBL_MIN;
                dp = x;
                if (j < n) Z[i][j] = x;
            };
            {
                int i = 1;
                for (; i < n && i < 64; ++i) fwd(i, rr_rl(dl0, i), rr_rl(ql0, i - 1));
                if (i < n) fwd(i, rr_rl(dl1, 0), rr_rl(ql0, 63));
                for (++i; i < n; ++i) fwd(i, rr_rl(dl1, i - 64), rr_rl(ql1, i - 65));
            }
            // bottom-up pivots delta-, twist index of smallest |gamma|
            double dm = rr_get(dl0, dl1, n - 1) - lj;
            if (dm == 0.0) dm = -DBL_MIN;
            double best = fabs(Z[n - 1][jc]);
            int r = n - 1;
            auto bwd = [&](int i, double dv, double qi) {
                const double di = dv - lj;
                dm = di - qi * rr_recip(dm);
                if (dm == 0.0) dm = -DBL_MIN;
                const double g = fabs(Z[i][jc] + dm - di);
                if (g < best) {
                    best = g;
                    r = i;
                }
            };
            {
                int i = n - 2;
                for (; i >= 64; --i) bwd(i, rr_rl(dl1, i - 64), rr_rl(ql1, i - 64));
                for (; i >= 0; --i) bwd(i, rr_rl(dl0, i), rr_rl(ql0, i));
            }
            if (j < n) {
                // ratios below the twist: z_{i+1} / z_i = -e_i / delta-_{i+1}
                dm = rr_get(dl0, dl1, n - 1) - lj;
                if (dm == 0.0) dm = -DBL_MIN;
                for (int i = n - 2; i >= r; --i) {
                    const double ei = sh.e[i];
                    const double rho = -ei * rr_recip(dm);
                    Z[i + 1][j] = rho;
                    dm = (sh.d[i] - lj) + ei * rho;
                    if (dm == 0.0) dm = -DBL_MIN;
                }
                Z[r][j] = 1.0;
                for (int i = r; i + 1 < n; ++i) Z[i + 1][j] *= Z[i][j];
                // above the twist: z_i = -(e_i / delta+_i) z_{i+1}
                for (int i = r - 1; i >= 0; --i) Z[i][j] = -(sh.e[i] * rr_recip(Z[i][j])) * Z[i + 1][j];
                double nn = 0.0;
                for (int i = 0; i < n; ++i) nn += Z[i][j] * Z[i][j];
                const double inv = 1.0 / sqrt(nn);
                for (int i = 0; i < n; ++i) Z[i][j] *= inv;
                if (!(nn > 0.0) || !isfinite(nn) || !(best * inv <= 1e-10 * tnorm)) sh.flag = 1;
            }
        }
        {
            // ---- clusters: modified Gram-Schmidt, two passes (one wave) ------
            const int close = tid + 1 < n && sh.lam[tid + 1] - sh.lam[tid] < 1e-3 * tnorm;
            if (__syncthreads_or(close) && wv == 0) {
                int j0 = 0;
                while (j0 < n) {
                    int j1 = j0;
                    while (j1 + 1 < n && sh.lam[j1 + 1] - sh.lam[j1] < 1e-3 * tnorm) ++j1;
                    for (int a = j0 + 1; a <= j1; ++a) {
                        for (int rep = 0; rep < 2; ++rep)
                            for (int b = j0; b < a; ++b) {
                                double s = 0.0;
                                for (int i = lane; i < n; i += 64) s += Z[i][b] * Z[i][a];
                                s = rr_wsum(s);
                                for (int i = lane; i < n; i += 64) Z[i][a] -= s * Z[i][b];
                            }
                        double nn = 0.0;
                        for (int i = lane; i < n; i += 64) nn += Z[i][a] * Z[i][a];
                        nn = rr_wsum(nn);
                        if (!(nn >= 1e-4)) {
                            if (lane == 0) sh.flag = 1;
                            nn = 1.0;
                        }
                        const double inv = 1.0 / sqrt(nn);
                        for (int i = lane; i < n; i += 64) Z[i][a] *= inv;
                    }
                    j0 = j1 + 1;
                }
            }
            __syncthreads();
        }

        // ---- back-transformation Z <- H_0 H_1 ... H_{n-3} Z --------------------
        // the reflector rows first become the vectors themselves (v_{k+1} = 1,
        // v_r = x_r hinv below)
        for (int t = tid; t < n * n; t += RR_NT) {
            const int k = t / n, r = t % n;
            if (k + 2 < n && r >= k + 1 && sh.tau[k] != 0.0) A[k][r] = r == k + 1 ? 1.0 : A[k][r] * sh.hinv[k];
        }
        __syncthreads();
        {
            // blocks of 16 reflectors k0..k0+15 as I - V T V^T (T upper triangular,
            // T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] V[:, 0:i]^T v_i), applied
            // last block first: Z <- Z - V (T (V^T Z)) on FP64 MFMA 16x16x4. Wave w
            // < nt takes the 16 columns 16w.. of Z: W = V^T Z_w, W' = T W (the MFMA
            // result items are exactly the next B operand: item v of lane l is row
            // l/16 + 4v), Z_w -= V W'; a wave touches only its own columns of Z.
            // Meanwhile the last wave (never one of the nt <= 6 column waves) forms
            // S = V^T V and T of the next block into the other of two buffers (lane
            // j owns row j of T, so the recurrence needs no barrier): one barrier
            // per block.
            const int nref = n - 2, nt = (n + 15) / 16, ks = (n + 3) / 4;
            const int nblk = nref > 0 ? (nref + 15) / 16 : 0, tw = RR_NW - 1;
            double *Tb0 = &sh.sc[0][0], *Tb1 = Tb0 + 256;   // 16 x 16 each (sc is free here)
            double *Sm = sh.u.dbl;                           // 16 x 16
            const int li = lane & 15, lk = lane >> 4;
            // entry r of reflector k with tau_k = tk (zero outside the vector, or if
            // no reflection)
            auto vv = [&](int k, double tk, int r) -> double {
                return (tk != 0.0 && r > k && r < n) ? A[k][r] : 0.0;
            };
            auto tau_of = [&](int k) -> double { return k < nref ? sh.tau[k] : 0.0; };
            auto make_t = [&](int k0, double *Tm) {
                const int s_lo = (k0 + 1) / 4;   // rows r <= k0 hold no entry of the block
                const double tl = tau_of(k0 + li);
                rr_dx4 a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
                int s4 = s_lo;
                for (; s4 + 1 < ks; s4 += 2) {
                    const double x0 = vv(k0 + li, tl, 4 * s4 + lk), x1 = vv(k0 + li, tl, 4 * s4 + 4 + lk);
                    a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, x0, a0, 0, 0, 0);
                    a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, x1, a1, 0, 0, 0);
                }
                if (s4 < ks) {
                    const double x0 = vv(k0 + li, tl, 4 * s4 + lk);
                    a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, x0, a0, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) Sm[(lk + 4 * v) * 16 + li] = a0[v] + a1[v];
                // T by columns; lane j < 16 owns row j; T[j][l] = 0 for l < j, so the
                // inner sum runs over l < i for every lane
                const int j = lane & 15;
                for (int i = 0; i < 16; ++i) {
                    double y0 = 0.0, y1 = 0.0;
                    int l = 0;
                    for (; l + 1 < i; l += 2) {
                        y0 = fma(Tm[j * 16 + l], Sm[l * 16 + i], y0);
                        y1 = fma(Tm[j * 16 + l + 1], Sm[(l + 1) * 16 + i], y1);
                    }
                    if (l < i) y0 = fma(Tm[j * 16 + l], Sm[l * 16 + i], y0);
                    const double ti = tau_of(k0 + i);
                    if (lane < 16) Tm[j * 16 + i] = j < i ? -ti * (y0 + y1) : (j == i ? ti : 0.0);
                }
            };
            if (nblk > 0 && wv == tw) make_t(16 * (nblk - 1), Tb0);
            __syncthreads();
            for (int blk = nblk - 1, buf = 0; blk >= 0; --blk, buf ^= 1) {
                const int k0 = 16 * blk;
                double *Tcur = buf ? Tb1 : Tb0;
                if (wv == tw && blk > 0) make_t(16 * (blk - 1), buf ? Tb0 : Tb1);
                if (wv < nt) {
                    const int c0 = 16 * wv, s_lo = (k0 + 1) / 4;
                    const double tl = tau_of(k0 + li);
                    rr_dx4 w0 = {0.0, 0.0, 0.0, 0.0}, w1 = {0.0, 0.0, 0.0, 0.0};
                    const bool cok = c0 + li < n;
                    int s4 = s_lo;
                    for (; s4 + 1 < ks; s4 += 2) {
                        const int r = 4 * s4 + lk;
                        const double z0 = (r < n && cok) ? Z[r][c0 + li] : 0.0;
                        const double z1 = (r + 4 < n && cok) ? Z[r + 4][c0 + li] : 0.0;
                        w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(vv(k0 + li, tl, r), z0, w0, 0, 0, 0);
                        w1 = __builtin_amdgcn_mfma_f64_16x16x4f64(vv(k0 + li, tl, r + 4), z1, w1, 0, 0, 0);
                    }
                    if (s4 < ks) {
                        const int r = 4 * s4 + lk;
                        const double z0 = (r < n && cok) ? Z[r][c0 + li] : 0.0;
                        w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(vv(k0 + li, tl, r), z0, w0, 0, 0, 0);
                    }
                    rr_dx4 accW;
#pragma unroll
                    for (int v = 0; v < 4; ++v) accW[v] = w0[v] + w1[v];
                    rr_dx4 accP = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        accP = __builtin_amdgcn_mfma_f64_16x16x4f64(Tcur[li * 16 + 4 * q + lk], accW[q], accP, 0, 0, 0);
                    double td[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) td[q] = tau_of(k0 + 4 * q + lk);
                    for (int rt = (k0 + 1) / 16; rt < nt; ++rt) {
                        const int r0 = 16 * rt;
                        rr_dx4 accD = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            accD = __builtin_amdgcn_mfma_f64_16x16x4f64(vv(k0 + 4 * q + lk, td[q], r0 + li), accP[q],
                                                                        accD, 0, 0, 0);
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = r0 + lk + 4 * v;
                            if (row < n && cok) Z[row][c0 + li] -= accD[v];
                        }
                    }
                }
                __syncthreads();
            }
        }

        // ---- Newton-Schulz: S = Z^T Z into A, then Y = Z (3I - S) / 2 ---------
        const int nt = (n + 15) / 16, kq = (n + 3) / 4;
        for (int tile = wv; tile < nt * nt; tile += RR_NW) {
            const int a0 = (tile / nt) * 16, b0 = (tile % nt) * 16;
            rr_dx4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int kk = 0; kk < kq; ++kk) {
                const int i = kk * 4 + (lane >> 4);
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Z[i][a0 + (lane & 15)], Z[i][b0 + (lane & 15)], acc, 0,
                                                           0, 0);
            }
            for (int q = 0; q < 4; ++q) A[a0 + (lane >> 4) + 4 * q][b0 + (lane & 15)] = acc[q];
        }
        __syncthreads();
        double defect = 0.0;
        for (int t = tid; t < n * RR_MAX; t += RR_NT) {
            const int a = t / RR_MAX, b = t % RR_MAX;
            if (b < n) defect = fmax(defect, fabs(A[a][b] - (a == b ? 1.0 : 0.0)));
        }
        defect = bmax(defect);
        if (!(defect <= 1e-8)) sh.flag = 1;
        for (int t = tid; t < RR_MAX * RR_MAX; t += RR_NT) {
            const int a = t / RR_MAX, b = t % RR_MAX;
            A[a][b] = (a == b ? 1.5 : 0.0) - 0.5 * A[a][b];
        }
        __syncthreads();
        if (!sh.flag) {
            for (int tile = wv; tile < nt * nt; tile += RR_NW) {
                const int i0 = (tile / nt) * 16, b0 = (tile % nt) * 16;
                rr_dx4 acc = {0.0, 0.0, 0.0, 0.0};
                for (int kk = 0; kk < kq; ++kk) {
                    const int a = kk * 4 + (lane >> 4);
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Z[i0 + (lane & 15)][a], A[a][b0 + (lane & 15)], acc,
                                                               0, 0, 0);
                }
                for (int q = 0; q < 4; ++q) {
                    const int i = i0 + (lane >> 4) + 4 * q, b = b0 + (lane & 15);
                    if (i < n && b < n) Y[(int64_t)i * ldy + b] = acc[q];
                }
            }
            for (int e = tid; e < n; e += RR_NT) theta[e] = sh.lam[e] / scale;
            return;
        }
    }
    // ---- fallback: cyclic Jacobi on G ------------------------------------------
    if (tid == 0 && nfallback) atomicAdd(nfallback, 1);
    rr_jacobi(sh, G, ldg, m, theta, Y, ldy, 40);
}

hipError_t launch_jacobi_eig(const double *G, int ldg, int m, double *theta, double *Y, int ldy, hipStream_t st)
{
    if (m <= 0 || m > RR_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jacobi_eig, dim3(1), dim3(RR_NT), 0, st, G, ldg, m, theta, Y, ldy, 40);
    return hipGetLastError();
}

hipError_t launch_rr_eig(const double *G, int ldg, int m, double *theta, double *Y, int ldy, int32_t *nfallback,
                         hipStream_t st)
{
    if (m <= 0 || m > RR_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rr_eig, dim3(1), dim3(RR_NT), 0, st, G, ldg, m, theta, Y, ldy, nfallback);
    return hipGetLastError();
}

}  // namespace cch
