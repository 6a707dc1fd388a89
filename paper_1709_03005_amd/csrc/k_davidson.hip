// Block Davidson pieces in FP64 (the paper names Davidson among the
// diagonalisers of Sec. 3.2 without detail; the solver is the block
// Davidson-Liu iteration with a diagonal correction and thick restart):
//   K8  W = H V for a block of b vectors (dense H streamed once: HBM-bound)
//   K9  tall-skinny products X^T Y (Gram blocks, projections) and V C
//       updates; modified Gram-Schmidt of a block in one workgroup
//   K10 residuals and the diagonal (Jacobi) correction (the Rayleigh-Ritz
//       eigenproblem is in k_rr.hip).
// Vectors are stored one per row: V[q][i], leading dimension ldv.
#include <algorithm>

#include "ccham_internal.h"

namespace cch {

// ---------------------------------------------------------------------------
// K8 on the matrix cores: W^T = V^T H (H symmetric), FP64 MFMA 16x16x4.
// Each wave owns a 16-column strip of H and a range of rows of H (split-K
// across blockIdx.y); the B operand is 4 rows x 16 columns of H (four 128-byte
// row segments per instruction), the A operand 16 vectors x 4 rows of V
// (zero rows for q >= b). Partial sums per split go to Wp[ks][q][r] and are
// reduced in a fixed order.
// ---------------------------------------------------------------------------
typedef double dx4m __attribute__((ext_vector_type(4)));
constexpr int MVM_UNROLL = 8;      // MFMA k-steps per register block (32 rows)
constexpr int MVM_NS = 4;          // 16-column strips per wave (share the V fragment)

__global__ __launch_bounds__(256) void k_matvec_mfma(const double *__restrict__ H, int64_t ld, int D,
                                                     const double *__restrict__ V, int64_t ldv, int b,
                                                     int rows_per_split, double *__restrict__ Wp)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r0 = (blockIdx.x * 4 + wv) * (16 * MVM_NS);
    const int q = lane & 15;                    // vector of the A operand
    const int kq = lane >> 4;                   // k within a 4-step
    const int cb = blockIdx.y * rows_per_split;
    const int ce = min(D, cb + rows_per_split);
    const bool qok = q < b;
    const double *vrow = V + (int64_t)(qok ? q : 0) * ldv;
    const double *hcol[MVM_NS];
    bool colok[MVM_NS];
#pragma unroll
    for (int t = 0; t < MVM_NS; ++t) {
        const int col = r0 + 16 * t + (lane & 15);
        colok[t] = col < D;
        hcol[t] = H + (colok[t] ? col : 0);
    }
    dx4m acc[MVM_NS];
#pragma unroll
    for (int t = 0; t < MVM_NS; ++t) acc[t] = (dx4m){0.0, 0.0, 0.0, 0.0};
    for (int c0 = cb; c0 < ce; c0 += 4 * MVM_UNROLL) {
        double bv[MVM_UNROLL][MVM_NS], av[MVM_UNROLL];
#pragma unroll
        for (int u = 0; u < MVM_UNROLL; ++u) {
            const int c = c0 + 4 * u + kq;
            const bool ok = c < ce;
            av[u] = (ok && qok) ? vrow[c] : 0.0;
#pragma unroll
            for (int t = 0; t < MVM_NS; ++t)
                bv[u][t] = (ok && colok[t]) ? __builtin_nontemporal_load(hcol[t] + (int64_t)c * ld) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < MVM_UNROLL; ++u)
#pragma unroll
            for (int t = 0; t < MVM_NS; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u][t], acc[t], 0, 0, 0);
    }
    // item v of lane l: row (vector) l/16 + 4v, column (r) l%16 of the strip
#pragma unroll
    for (int t = 0; t < MVM_NS; ++t) {
        const int col = r0 + 16 * t + (lane & 15);
        if (colok[t]) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int qq = (lane >> 4) + 4 * v;
                if (qq < b) Wp[((int64_t)blockIdx.y * 16 + qq) * D + col] = acc[t][v];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K8 from the lower triangle only (H symmetric): every element H[r][c] with
// r > c is read once and used twice, for W[.][c] += H[r][c] V[.][r] (the
// column product) and W[.][r] += H[r][c] V[.][c] (the row product); the
// diagonal once. Half the bytes of the full product for twice the MFMA work
// per byte.
//
// The lower triangle is cut into strips of SV_CW columns; a strip's rows
// (from its diagonal down) into items of rb rows, one workgroup (8 waves)
// per item, two workgroups per compute unit (at most 128 registers a lane).
// An item is walked in chunks of SV_CH rows and, inside a chunk, in tiles of
// SV_CH x SV_SB staged through LDS with the chunk's V rows and the tile's V
// columns (the next tile is loaded into registers while the current one is
// multiplied). The waves take turns by sub-block parity: in a tile, the four
// waves of one parity form the column product of one 16-column strip each
// over the tile's rows (accumulated over the whole item), the other four the
// row product of 16 rows each over the tile's columns (accumulated over the
// chunk). A chunk's row sums (the two parities added in LDS) go to
// P2[strip][q][row]; at the end of the item the column sums go to
// P1[item][q][col]. k_symv_reduce adds, for row i, P2 of every strip left of
// and including i's, then P1 of every item of i's strip, in a fixed order
// (deterministic). Tiles on the diagonal zero the elements above it (and, in
// the row product, the diagonal itself); tiles wholly above it are skipped.
//
// The products run on the 4x4x4 FP64 MFMA (four blocks): the B operand is a
// 4 x 16 slab of the tile (block b takes its columns 4b..4b+3), the A operand
// the 4 x 4 slab of V for one group of four vectors (the same in every
// block), so a launch pays for ceil(b / 4) groups, not for 16 vectors. Lane
// l = j + 4 blk + 16 i holds D[blk][i][j]: vector 4 g + (l >> 4), column (or
// row) l & 15 of the strip. On this chip the 4x4x4 form also issues faster
// per flop than the 16x16x4 one.
// ---------------------------------------------------------------------------
constexpr int SV_CW = 512, SV_SB = 64, SV_CH = 64, SV_NSB = SV_CW / SV_SB;
constexpr int SV_LS = SV_SB + 1;     // LDS row strides in doubles (odd: conflict-free column reads)
constexpr int SV_LR = SV_CH + 1;

__host__ __device__ inline int sv_items(int D, int J, int rb) { return (D - J * SV_CW + rb - 1) / rb; }

template <int NG>
__global__ __launch_bounds__(512, 4) void k_symv(const double *__restrict__ H, int64_t ld, int D,
                                                  const double *__restrict__ V, int64_t ldv, int b, int rb,
                                                  double *__restrict__ P1, double *__restrict__ P2)
{
    __shared__ double Hs[SV_CH * SV_LS];
    __shared__ double Vc[16 * SV_LS];
    __shared__ double Vr[16 * SV_LR];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    int J = 0, base = 0;
    for (;;) {
        const int n = sv_items(D, J, rb);
        if ((int)blockIdx.x < base + n) break;
        base += n;
        ++J;
    }
    const int J0 = J * SV_CW;
    const int R0 = J0 + ((int)blockIdx.x - base) * rb, R1 = min(D, R0 + rb);
    const int nsb_d = min(SV_NSB, (D - J0 + SV_SB - 1) / SV_SB);
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 ph[4];
    double pv[2], pr[2];
    auto load_tile = [&](int r0, int c0, bool first) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int g = tid + 512 * i, row = g >> 5, c = c0 + 2 * (g & 31), r = r0 + row;
            d2 v = (d2){0.0, 0.0};
            if (r < R1) {
                const double *src = H + (int64_t)r * ld + c;
                if (c + 1 < D) v = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(src));
                else if (c < D) v.x = src[0];
            }
            ph[i] = v;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = tid + 512 * i, q = e >> 6, c = c0 + (e & 63);
            pv[i] = (q < b && c < D) ? V[(int64_t)q * ldv + c] : 0.0;
        }
        if (first) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int e = tid + 512 * i, q = e >> 6, r = r0 + (e & 63);
                pr[i] = (q < b && r < R1) ? V[(int64_t)q * ldv + r] : 0.0;
            }
        }
    };
    auto store_tile = [&](bool first) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int g = tid + 512 * i, row = g >> 5, cl = 2 * (g & 31);
            Hs[row * SV_LS + cl] = ph[i].x;
            Hs[row * SV_LS + cl + 1] = ph[i].y;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = tid + 512 * i;
            Vc[(e >> 6) * SV_LS + (e & 63)] = pv[i];
        }
        if (first) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int e = tid + 512 * i;
                Vr[(e >> 6) * SV_LR + (e & 63)] = pr[i];
            }
        }
    };
    auto nsb_of = [&](int r0) { return r0 < R1 ? min(nsb_d, (r0 + SV_CH - J0 + SV_SB - 1) / SV_SB) : 0; };
    const int st = w & 3, par = w >> 2;
    double acc1[SV_NSB / 2][NG];
#pragma unroll
    for (int m = 0; m < SV_NSB / 2; ++m)
#pragma unroll
        for (int g = 0; g < NG; ++g) acc1[m][g] = 0.0;
    const int p4 = lane & 3;
    load_tile(R0, J0, true);
    for (int r0 = R0; r0 < R1; r0 += SV_CH) {
        const int nsb = nsb_of(r0), nsb_next = nsb_of(r0 + SV_CH);
        double acc2[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) acc2[g] = 0.0;
#pragma unroll
        for (int s = 0; s < SV_NSB; ++s) {
            if (s < nsb) {
                const int c0 = J0 + SV_SB * s;
                __syncthreads();
                store_tile(s == 0);
                __syncthreads();
                {
                    const bool more = s + 1 < nsb;
                    if (more || nsb_next > 0) load_tile(more ? r0 : r0 + SV_CH, more ? c0 + SV_SB : J0, !more);
                }
                const bool diag = r0 <= c0 + SV_SB - 1;
                if ((s & 1) == par) {
                    // column product: strip st, 64 rows
#pragma unroll 2
                    for (int u = 0; u < SV_CH / 4; ++u) {
                        const int rl = 4 * u + hi, cl = 16 * st + lo;
                        double h = Hs[rl * SV_LS + cl];
                        if (diag && r0 + rl < c0 + cl) h = 0.0;
#pragma unroll
                        for (int g = 0; g < NG; ++g) {
                            const double a = Vr[(4 * g + p4) * SV_LR + rl];
                            acc1[s >> 1][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, h, acc1[s >> 1][g], 0, 0, 0);
                        }
                    }
                } else {
                    // row product: rows 16 st.., 64 columns, two chains
#pragma unroll 2
                    for (int u = 0; u < SV_SB / 4; ++u) {
                        const int cl = 4 * u + hi, rl = 16 * st + lo;
                        double h = Hs[rl * SV_LS + cl];
                        if (diag && r0 + rl <= c0 + cl) h = 0.0;
#pragma unroll
                        for (int g = 0; g < NG; ++g) {
                            const double a = Vc[(4 * g + p4) * SV_LS + cl];
                            acc2[g] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, h, acc2[g], 0, 0, 0);
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (par == 1) {
#pragma unroll
            for (int g = 0; g < NG; ++g) Vr[(st * 4 + g) * 64 + lane] = acc2[g];
        }
        __syncthreads();
        if (par == 0) {
            const int r = r0 + 16 * st + lo;
            if (r < R1) {
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const int q = 4 * g + hi;
                    if (q < b) P2[((int64_t)J * b + q) * D + r] = acc2[g] + Vr[(st * 4 + g) * 64 + lane];
                }
            }
        }
    }
    const int64_t item = blockIdx.x;
#pragma unroll
    for (int m = 0; m < SV_NSB / 2; ++m) {
        const int c = J0 + SV_SB * (2 * m + par) + 16 * st + lo;
        if (c < D) {
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int q = 4 * g + hi;
                if (q < b) P1[(item * b + q) * SV_CW + (c - J0)] = acc1[m][g];
            }
        }
    }
}

__global__ void k_symv_reduce(const double *__restrict__ P1, const double *__restrict__ P2, int D, int b, int rb,
                              double *__restrict__ Wo, int64_t ldw)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (i >= D || q >= b) return;
    const int J = i / SV_CW;
    int base = 0;
    for (int j = 0; j < J; ++j) base += sv_items(D, j, rb);
    const int n = sv_items(D, J, rb);
    // P2 of strips 0 .. J, then P1 of the items of strip J, in that order;
    // the loads go out eight at a time (one at a time left about one load in
    // flight per wave)
    double s = 0.0;
    int j = 0;
    for (; j + 8 <= J + 1; j += 8) {
        double u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = P2[((int64_t)(j + k) * b + q) * D + i];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) s += u[k];
    }
    for (; j <= J; ++j) s += P2[((int64_t)j * b + q) * D + i];
    const double *p1 = P1 + ((int64_t)base * b + q) * SV_CW + (i - J * SV_CW);
    const int64_t st1 = (int64_t)b * SV_CW;
    int t = 0;
    for (; t + 8 <= n; t += 8) {
        double u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = p1[(t + k) * st1];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) s += u[k];
    }
    for (; t < n; ++t) s += p1[t * st1];
    Wo[(int64_t)q * ldw + i] = s;
}

// item height of the symmetric product: the largest of 2048 .. 128 rows that
// still gives at least 4096 items (eight rounds of two workgroups per
// compute unit: short tails)
static int symv_rows_per_item(int D)
{
    int rb = 2048;
    for (; rb > 128; rb /= 2) {
        int64_t items = 0;
        for (int J = 0; J * SV_CW < D; ++J) items += sv_items(D, J, rb);
        if (items >= 4096) break;
    }
    return rb;
}

static int64_t symv_items(int D, int rb)
{
    int64_t items = 0;
    for (int J = 0; J * SV_CW < D; ++J) items += sv_items(D, J, rb);
    return items;
}

// the symmetric product pays off once the matrix is large enough to fill the
// chip with its items; below, the full product with split-K
constexpr int SYMV_MIN_D = 16384;

__global__ void k_matvec_reduce(const double *__restrict__ Wp, int ks, int D, int b, double *__restrict__ Wo,
                                int64_t ldw)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (r >= D || q >= b) return;
    double s = 0.0;
    for (int k = 0; k < ks; ++k) s += Wp[((int64_t)k * 16 + q) * D + r];
    Wo[(int64_t)q * ldw + r] = s;
}

// number of row splits for the MFMA mat-vec (enough waves to cover HBM latency)
int matvec_splits(int D)
{
    const int waves = (D + 16 * MVM_NS - 1) / (16 * MVM_NS);
    int ks = (4096 + waves - 1) / waves;
    ks = std::max(1, std::min(ks, 64));
    return ks;
}

hipError_t launch_matvec(const double *H, int64_t ld, int D, const double *V, int64_t ldv, int b, double *W,
                         int64_t ldw, double *Wp, hipStream_t st)
{
    if (D <= 0 || b <= 0) return hipSuccess;
    if (D >= SYMV_MIN_D) {
        const int rb = symv_rows_per_item(D);
        const int64_t items = symv_items(D, rb);
        const int nstrip = (D + SV_CW - 1) / SV_CW;
        double *P1 = Wp, *P2 = Wp + items * 16 * SV_CW;
        (void)nstrip;
        for (int q0 = 0; q0 < b; q0 += 16) {
            const int bb = std::min(16, b - q0);
            const double *Vq = V + (int64_t)q0 * ldv;
            switch ((bb + 3) / 4) {   // groups of four vectors on the 4x4x4 FP64 MFMA
            case 1: hipLaunchKernelGGL(k_symv<1>, dim3((unsigned)items), dim3(512), 0, st, H, ld, D, Vq, ldv, bb, rb, P1, P2); break;
            case 2: hipLaunchKernelGGL(k_symv<2>, dim3((unsigned)items), dim3(512), 0, st, H, ld, D, Vq, ldv, bb, rb, P1, P2); break;
            case 3: hipLaunchKernelGGL(k_symv<3>, dim3((unsigned)items), dim3(512), 0, st, H, ld, D, Vq, ldv, bb, rb, P1, P2); break;
            default: hipLaunchKernelGGL(k_symv<4>, dim3((unsigned)items), dim3(512), 0, st, H, ld, D, Vq, ldv, bb, rb, P1, P2); break;
            }
            hipLaunchKernelGGL(k_symv_reduce, dim3((D + 255) / 256, bb), dim3(256), 0, st, P1, P2, D, bb, rb,
                               W + (int64_t)q0 * ldw, ldw);
        }
        return hipGetLastError();
    }
    const int ks = matvec_splits(D);
    int rps = (D + ks - 1) / ks;
    rps = (rps + 4 * MVM_UNROLL - 1) / (4 * MVM_UNROLL) * (4 * MVM_UNROLL);
    const int ksu = (D + rps - 1) / rps;
    for (int q0 = 0; q0 < b; q0 += 16) {
        const int bb = std::min(16, b - q0);
        hipLaunchKernelGGL(k_matvec_mfma, dim3((D + 64 * MVM_NS - 1) / (64 * MVM_NS), ksu), dim3(256), 0, st, H, ld,
                           D, V + (int64_t)q0 * ldv, ldv, bb, rps, Wp);
        hipLaunchKernelGGL(k_matvec_reduce, dim3((D + 255) / 256, bb), dim3(256), 0, st, Wp, ksu, D, bb,
                           W + (int64_t)q0 * ldw, ldw);
    }
    return hipGetLastError();
}

// doubles of the Wp scratch launch_matvec needs for dimension D
int64_t matvec_scratch_doubles(int D)
{
    const int64_t full = (int64_t)16 * D * (matvec_splits(D) + 1);
    if (D < SYMV_MIN_D) return full;
    const int rb = symv_rows_per_item(D);
    const int64_t nstrip = (D + SV_CW - 1) / SV_CW;
    return std::max(full, symv_items(D, rb) * 16 * SV_CW + nstrip * 16 * (int64_t)D);
}

// ---------------------------------------------------------------------------
// K9: tall-skinny products out[a][c] = sum_i X[a][i] Y[c][i]
// ---------------------------------------------------------------------------
constexpr int TN_CHUNK = 1024;   // row chunk of the residual norms

// out[a*ldo + c] (or out[c*ldo + a] when transpose) = X[a] . Y[c], a < na,
// c < nc <= 96, on FP64 MFMA: one wave per 16 x 16 output tile and slice of
// the long dimension, 4 waves per workgroup share a split and sum their tiles
// in LDS; the splits are summed in order by k_tn_sum (deterministic).
// A lane loads 4 consecutive doubles of one X row and one Y row per 16-row
// step (32-byte pieces, 128 contiguous bytes per row); the four MFMAs of a
// step take k = 4 (l / 16) + j for lane l and j = 0..3 in both operands.
typedef double tnx4 __attribute__((ext_vector_type(4)));
constexpr int TN_SPLIT_MAX = 64, TN_LD = 96, TN_U = 4;

int tn_splits(int D)
{
    return std::max(1, std::min(TN_SPLIT_MAX, (D + 255) / 256));
}

int64_t tn_part_doubles()
{
    return (int64_t)TN_SPLIT_MAX * TN_LD * TN_LD;
}

__device__ __forceinline__ void tn_load4(const double *row, int k, int D, bool ok, double *v)
{
    if (ok && k + 3 < D) {
        const double4 q = *reinterpret_cast<const double4 *>(row + k);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (ok && k + j < D) ? row[k + j] : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_tn_mfma(const double *__restrict__ X1, int64_t ldx1, int na1,
                                                 const double *__restrict__ X2, int64_t ldx2, int na,
                                                 const double *__restrict__ Y, int64_t ldy, int nc, int D,
                                                 int rows_per_split, double *__restrict__ part)
{
    __shared__ double red[4][16][17];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nct = (nc + 15) / 16;
    const int a0 = (blockIdx.x / nct) * 16, c0 = (blockIdx.x % nct) * 16;
    const int split = blockIdx.y;
    const int kb = split * rows_per_split, ke = min(D, kb + rows_per_split);
    const int ra = a0 + (lane & 15), rc = c0 + (lane & 15);
    const bool oka = ra < na, okc = rc < nc;
    // rows a < na1 of X come from X1, the rest from X2
    const double *xr = !oka ? X1 : (ra < na1 ? X1 + (int64_t)ra * ldx1 : X2 + (int64_t)(ra - na1) * ldx2);
    const double *yr = Y + (int64_t)(okc ? rc : 0) * ldy;
    tnx4 acc = {0.0, 0.0, 0.0, 0.0};
    // TN_U steps of 16 rows per trip: every load of the trip is issued before
    // its MFMAs (steps past the end of the split load zeros)
    for (int k0 = kb + 16 * wv; k0 < ke; k0 += 64 * TN_U) {
        double xv[TN_U][4], yv[TN_U][4];
#pragma unroll
        for (int u = 0; u < TN_U; ++u) {
            const int k = k0 + 64 * u + 4 * (lane >> 4);
            tn_load4(xr, k, ke, oka, xv[u]);
            tn_load4(yr, k, ke, okc, yv[u]);
        }
#pragma unroll
        for (int u = 0; u < TN_U; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[u][j], yv[u][j], acc, 0, 0, 0);
    }
    // item v of lane l: row (a) l/16 + 4v, column (c) l%16
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wv][(lane >> 4) + 4 * v][lane & 15] = acc[v];
    __syncthreads();
    const int r = threadIdx.x >> 4, c = threadIdx.x & 15;
    if (a0 + r < na && c0 + c < nc)
        part[((int64_t)split * TN_LD + a0 + r) * TN_LD + c0 + c] = red[0][r][c] + red[1][r][c] + red[2][r][c] +
                                                                   red[3][r][c];
}

__global__ void k_tn_sum(const double *__restrict__ part, int nsplit, int na, int nc, double *__restrict__ out,
                         int64_t ldo, int transpose, double *__restrict__ outT, int cT)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= na * nc) return;
    const int a = t / nc, c = t % nc;
    // four interleaved partial sums (loads in flight), added in a fixed order
    const double *pp = part + (int64_t)a * TN_LD + c;
    const int64_t st = (int64_t)TN_LD * TN_LD;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = 0;
    for (; q + 3 < nsplit; q += 4) {
        s0 += pp[q * st];
        s1 += pp[(q + 1) * st];
        s2 += pp[(q + 2) * st];
        s3 += pp[(q + 3) * st];
    }
    for (; q < nsplit; ++q) s0 += pp[q * st];
    const double s = (s0 + s1) + (s2 + s3);
    if (transpose) out[(int64_t)c * ldo + a] = s;
    else out[(int64_t)a * ldo + c] = s;
    if (outT && c < cT) outT[(int64_t)c * ldo + a] = s;   // mirror of the columns before cT
}

// out[a*ldo + c] (or out[c*ldo + a] when transpose) = X[a] . Y[c], where
// X[a] = X1[a] for a < na1 and X2[a - na1] for na1 <= a < na; na, nc <= 96,
// every row 32-byte aligned (leading dimensions multiples of 4). With outT,
// also outT[c*ldo + a] = X[a] . Y[c] for c < cT (the mirror image of a block of
// new rows of a symmetric matrix, for the columns that precede them).
hipError_t launch_tn(const double *X1, int64_t ldx1, int na1, const double *X2, int64_t ldx2, int na,
                     const double *Y, int64_t ldy, int nc, int D, double *part, double *out, int64_t ldo,
                     int transpose, hipStream_t st, double *outT, int cT)
{
    if (na <= 0 || nc <= 0) return hipSuccess;
    if (na1 < 0 || na1 > na || na > TN_LD || nc > TN_LD || (ldx1 & 3) || (ldy & 3) || ((uintptr_t)X1 & 31) ||
        ((uintptr_t)Y & 31))
        return hipErrorInvalidValue;
    if (na1 < na && (X2 == nullptr || (ldx2 & 3) || ((uintptr_t)X2 & 31))) return hipErrorInvalidValue;
    const int ns = tn_splits(D);
    const int rps = ((D + ns - 1) / ns + 15) / 16 * 16;
    const int tiles = ((na + 15) / 16) * ((nc + 15) / 16);
    hipLaunchKernelGGL(k_tn_mfma, dim3(tiles, ns), dim3(256), 0, st, X1, ldx1, na1, X2, ldx2, na, Y, ldy, nc, D, rps,
                       part);
    hipLaunchKernelGGL(k_tn_sum, dim3((na * nc + 255) / 256), dim3(256), 0, st, part, ns, na, nc, out, ldo,
                       transpose, outT, cT);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// out[e][i] = beta * base[e][i] + alpha * sum_{q<m} V[q][i] C[q*ldc + e], e < ne,
// where V[q] = V1[q] for q < m1 and V2[q - m1] for m1 <= q < m
// grid (D/256, ceil(ne/NE)): NE outputs per thread, C slice staged in LDS.
// Each grid row reads every input vector once, so wider slices read them
// fewer times; the sum over q runs in the same order for any NE. A thread
// loads NN_QB rows of V at a time before it multiplies (one row per step
// left a wave with a single load in flight, at about one wave per SIMD).
// ---------------------------------------------------------------------------
constexpr int NN_QB = 16;

// acc[e] += V[q][i] cs[q][e] for q in [q0, q1), V[q] = Vp[(q - qoff) ldv]
template <int NE>
__device__ __forceinline__ void nn_accum(const double *__restrict__ Vp, int64_t ldv, int q0, int q1, int qoff, int i,
                                         const double *cs, double (&acc)[NE])
{
    int q = q0;
    for (; q + NN_QB <= q1; q += NN_QB) {
        double v[NN_QB];
#pragma unroll
        for (int u = 0; u < NN_QB; ++u) v[u] = Vp[(int64_t)(q + u - qoff) * ldv + i];
        __builtin_amdgcn_sched_barrier(0);   // all NN_QB loads go out before the products
#pragma unroll
        for (int u = 0; u < NN_QB; ++u) {
            double c[NE];
#pragma unroll
            for (int e = 0; e < NE; ++e) c[e] = cs[(q + u) * NE + e];
#pragma unroll
            for (int e = 0; e < NE; ++e) acc[e] = fma(v[u], c[e], acc[e]);
        }
    }
    for (; q < q1; ++q) {
        const double v = Vp[(int64_t)(q - qoff) * ldv + i];
#pragma unroll
        for (int e = 0; e < NE; ++e) acc[e] = fma(v, cs[q * NE + e], acc[e]);
    }
}

template <int NE>
__global__ __launch_bounds__(256) void k_nn_small(const double *__restrict__ V1, int64_t ldv1, int m1,
                                                  const double *__restrict__ V2, int64_t ldv2, int m, int D,
                                                  const double *__restrict__ Cm, int ldc, int ne,
                                                  const double *__restrict__ base, int64_t ldb, double beta,
                                                  double alpha, double *__restrict__ out, int64_t ldo,
                                                  const double *__restrict__ V1z, double *__restrict__ outz)
{
    extern __shared__ double cs[];   // [m][NE]
    if (blockIdx.z == 1) {   // the second product of a pair launch: same C, other V1 and out
        V1 = V1z;
        out = outz;
    }
    const int e0 = blockIdx.y * NE;
    for (int t = threadIdx.x; t < m * NE; t += 256) {
        const int q = t / NE, e = e0 + t % NE;
        cs[t] = e < ne ? Cm[(int64_t)q * ldc + e] : 0.0;
    }
    __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= D) return;
    double acc[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) acc[e] = 0.0;
    nn_accum<NE>(V1, ldv1, 0, m1, 0, i, cs, acc);
    if (m1 < m) nn_accum<NE>(V2, ldv2, m1, m, m1, i, cs, acc);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        if (e0 + e < ne) {
            double r = alpha * acc[e];
            if (base) r += beta * base[(int64_t)(e0 + e) * ldb + i];
            out[(int64_t)(e0 + e) * ldo + i] = r;
        }
    }
}

// out and base may be the same rows (in-place update of one element by one
// thread); out must not overlap the rows read from V1 or V2.
// With V1z and outz (and no second panel), one launch also forms
// outz = beta * base + alpha * V1z C with the same C (the pair of rotations).
// Slice width: 16 outputs per thread from D = 32768 on (the inputs are then
// read ceil(ne / 16) times), 8 from 16384, else 4 (more workgroups for small D).
hipError_t launch_nn(const double *V1, int64_t ldv1, int m1, const double *V2, int64_t ldv2, int m, int D,
                     const double *C, int ldc, int ne, const double *base, int64_t ldb, double beta, double alpha,
                     double *out, int64_t ldo, hipStream_t st, const double *V1z, double *outz)
{
    if (ne <= 0 || D <= 0) return hipSuccess;
    if (m1 < 0 || m1 > m || (m1 < m && V2 == nullptr)) return hipErrorInvalidValue;
    if ((V1z == nullptr) != (outz == nullptr) || (V1z && (m1 != m || base))) return hipErrorInvalidValue;
    const int NE = D >= 32768 ? 16 : (D >= 16384 ? 8 : 4);
    const dim3 g((D + 255) / 256, (ne + NE - 1) / NE, V1z ? 2 : 1), bl(256);
    const size_t shm = sizeof(double) * NE * (size_t)(m > 0 ? m : 1);
    if (NE == 16)
        hipLaunchKernelGGL(k_nn_small<16>, g, bl, shm, st, V1, ldv1, m1, V2, ldv2, m, D, C, ldc, ne, base, ldb, beta,
                           alpha, out, ldo, V1z, outz);
    else if (NE == 8)
        hipLaunchKernelGGL(k_nn_small<8>, g, bl, shm, st, V1, ldv1, m1, V2, ldv2, m, D, C, ldc, ne, base, ldb, beta,
                           alpha, out, ldo, V1z, outz);
    else
        hipLaunchKernelGGL(k_nn_small<4>, g, bl, shm, st, V1, ldv1, m1, V2, ldv2, m, D, C, ldc, ne, base, ldb, beta,
                           alpha, out, ldo, V1z, outz);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K10: residuals R = AX - X theta and their squared norms per chunk
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ AX, const double *__restrict__ X,
                                                  int64_t ld, int D, const double *__restrict__ theta, int k,
                                                  double *__restrict__ R, double *__restrict__ part)
{
    const int e = blockIdx.y, ch = blockIdx.x;
    const int i0 = ch * TN_CHUNK, i1 = min(D, i0 + TN_CHUNK);
    const double th = theta[e];
    double s = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
        const double r = AX[(int64_t)e * ld + i] - th * X[(int64_t)e * ld + i];
        R[(int64_t)e * ld + i] = r;
        s = fma(r, r, s);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)ch * k + e] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_norm_reduce(const double *__restrict__ part, int nch, int k, double *__restrict__ out)
{
    const int e = threadIdx.x;
    if (e >= k) return;
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += part[(int64_t)c * k + e];
    out[e] = sqrt(s);
}

hipError_t launch_residual(const double *AX, const double *X, int64_t ld, int D, const double *theta, int k,
                           double *R, double *part, double *norms, hipStream_t st)
{
    const int nch = (D + TN_CHUNK - 1) / TN_CHUNK;
    hipLaunchKernelGGL(k_residual, dim3(nch, k), dim3(256), 0, st, AX, X, ld, D, theta, k, R, part);
    hipLaunchKernelGGL(k_norm_reduce, dim3(1), dim3(64), 0, st, part, nch, k, norms);
    return hipGetLastError();
}

// diagonal (Jacobi) correction t = r / (theta - H_ii), |den| floored at 1e-8
// with its sign kept; sel.e[c] picks the residual row of output c
__global__ void k_jacobi_correct(const double *__restrict__ R, int64_t ld, int D,
                                 const double *__restrict__ diag, const double *__restrict__ theta, DavSel sel,
                                 int nsel, double *__restrict__ T, int64_t ldt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= D || c >= nsel) return;
    const int e = sel.e[c];
    double den = theta[e] - diag[i];
    if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
    T[(int64_t)c * ldt + i] = R[(int64_t)e * ld + i] / den;
}

hipError_t launch_jacobi_correct(const double *R, int64_t ld, int D, const double *diag, const double *theta,
                                 const DavSel &sel, int nsel, double *T, int64_t ldt, hipStream_t st)
{
    if (nsel <= 0) return hipSuccess;
    if (nsel > 32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jacobi_correct, dim3((D + 255) / 256, nsel), dim3(256), 0, st, R, ld, D, diag, theta,
                       sel, nsel, T, ldt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cholesky QR of a projected block with column pivoting (one wave).
// The block is T' = T - V S with S = V^T T (m x b, row q = V column q); its
// Gram matrix is taken as G - S^T S with G = T^T T (b x b, b <= 32), which
// equals T'^T T' up to S^T (V^T V - I) S. Columns are picked greedily by the
// largest remaining Schur-complement diagonal and kept while it exceeds rel^2
// times the reference squared norm of that column (ref[j * ref_stride] if
// given, else the projected Gram diagonal). With R the Cholesky factor of the
// kept columns in pivot order and B = P R^-1 (b x b, column c < rank), the
// output is the (m + b) x b matrix M = [-S B; B], so that [V | T] M = T' B is
// an orthonormal basis of the kept directions; columns c >= rank are zero.
// ---------------------------------------------------------------------------
constexpr int PCH_MAX = 32, PCH_M = 96;

struct PchI2 {
    int x, y;
};

template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ double pch_dpp(double v)
{
    PchI2 a = __builtin_bit_cast(PchI2, v);
    a.x = __builtin_amdgcn_update_dpp(0, a.x, CTRL, ROW_MASK, BANK_MASK, true);
    a.y = __builtin_amdgcn_update_dpp(0, a.y, CTRL, ROW_MASK, BANK_MASK, true);
    return __builtin_bit_cast(double, a);
}

__device__ __forceinline__ double pch_rl(double v, int lane)
{
    PchI2 a = __builtin_bit_cast(PchI2, v);
    a.x = __builtin_amdgcn_readlane(a.x, lane);
    a.y = __builtin_amdgcn_readlane(a.y, lane);
    return __builtin_bit_cast(double, a);
}

// maximum over the 64 lanes of values >= 0 (lanes without a DPP source read
// 0): within rows of 16 by row shifts, then across rows by row broadcasts;
// the result collects in lane 63 and is read from there
__device__ __forceinline__ double pch_wmax(double v)
{
    double s = fmax(v, pch_dpp<0x111, 0xf, 0xf>(v));
    s = fmax(s, pch_dpp<0x112, 0xf, 0xf>(v));
    s = fmax(s, pch_dpp<0x113, 0xf, 0xf>(v));
    s = fmax(s, pch_dpp<0x114, 0xf, 0xe>(s));
    s = fmax(s, pch_dpp<0x118, 0xf, 0xc>(s));
    s = fmax(s, pch_dpp<0x142, 0xa, 0xf>(s));
    s = fmax(s, pch_dpp<0x143, 0xc, 0xf>(s));
    return pch_rl(s, 63);
}

__global__ __launch_bounds__(256) void k_pchol(const double *__restrict__ G, int ldg, int b,
                                               const double *__restrict__ S, int lds, int m,
                                               const double *__restrict__ ref, int ref_stride, double rel,
                                               double *__restrict__ Cout, int ldc, int32_t *__restrict__ rank_out)
{
    __shared__ double A[PCH_MAX][PCH_MAX + 1];    // lane l of wave 0 owns column l; column PCH_MAX is padding
    __shared__ double Ss[PCH_M][PCH_MAX + 1];
    __shared__ double Rq[PCH_MAX][PCH_MAX + 1];   // row i of R by original column
    __shared__ double R[PCH_MAX][PCH_MAX + 1];    // R in pivot order
    __shared__ double Ri[PCH_MAX][PCH_MAX + 1];   // its inverse
    __shared__ double Bq[PCH_MAX][PCH_MAX + 1];   // B by original column
    __shared__ double rdg[PCH_MAX];               // 1 / R[i][i]
    __shared__ int piv[PCH_MAX];
    __shared__ int rank_sh;
    const int t = threadIdx.x;
    for (int e = t; e < m * b; e += 256) Ss[e / b][e % b] = S[(int64_t)(e / b) * lds + e % b];
    for (int e = t; e < b * b; e += 256) {
        const int i = e / b, j = e % b;
        A[i][j] = 0.5 * (G[(int64_t)i * ldg + j] + G[(int64_t)j * ldg + i]);
    }
    for (int e = t; e < PCH_MAX * PCH_MAX; e += 256) {
        Rq[e / PCH_MAX][e % PCH_MAX] = 0.0;
        Bq[e / PCH_MAX][e % PCH_MAX] = 0.0;
    }
    __syncthreads();
    // A -= S^T S in four interleaved partial sums, combined in a fixed order:
    // the same operations for (i, j) and (j, i), so A stays exactly symmetric
    for (int e = t; e < b * b; e += 256) {
        const int i = e / b, j = e % b;
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        int q = 0;
        for (; q + 3 < m; q += 4)
#pragma unroll
            for (int u = 0; u < 4; ++u) s4[u] = fma(Ss[q + u][i], Ss[q + u][j], s4[u]);
        for (; q < m; ++q) s4[0] = fma(Ss[q][i], Ss[q][j], s4[0]);
        A[i][j] -= (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    __syncthreads();
    if (t < 64) {
        // pivoted Cholesky in wave 0 alone (no barrier inside). Every value that
        // another lane reads (key through DPP, the R row through lane reads) is
        // formed by selects with the whole wave active; only stores are masked.
        const bool mine = t < b;
        const int tc = mine ? t : PCH_MAX;   // own column, or the padding column
        const double refd = mine ? rel * rel * (ref ? ref[(int64_t)t * ref_stride] : A[t][t]) : 0.0;
        bool used = !mine;
        int r = b;
        for (int i = 0; i < b; ++i) {
            // pivot: the largest admissible remaining diagonal (ties: lowest column)
            const double d = A[mine ? t : 0][mine ? t : 0];
            const bool cand = !used && d > refd && d > 0.0;
            const double key = cand ? d : 0.0;
            const double mx = pch_wmax(key);
            if (!(mx > 0.0)) {
                r = i;
                break;
            }
            const int p = __ffsll((unsigned long long)__ballot(key == mx)) - 1;
            const double rp = sqrt(mx);
            const double quo = A[p][tc] / rp;
            const double rl = used ? 0.0 : (t == p ? rp : quo);
            used = used || t == p;
            if (mine) Rq[i][t] = rl;
            if (t == 0) piv[i] = p;
            // Schur complement on the columns still free: lane l updates its
            // column, four rows loaded before any is stored
            const unsigned long long freem = __ballot(!used);
            int q = 0;
            for (; q + 3 < b; q += 4) {
                double a4[4], r4[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a4[u] = A[q + u][tc];
                    r4[u] = pch_rl(rl, q + u);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool upd = !used && ((freem >> (q + u)) & 1ull);
                    A[q + u][tc] = upd ? fma(-r4[u], rl, a4[u]) : a4[u];
                }
            }
            for (; q < b; ++q) {
                const double a1 = A[q][tc], r1 = pch_rl(rl, q);
                const bool upd = !used && ((freem >> q) & 1ull);
                A[q][tc] = upd ? fma(-r1, rl, a1) : a1;
            }
        }
        if (t == 0) rank_sh = r;
    }
    __syncthreads();
    const int r = rank_sh;
    for (int e = t; e < r * r; e += 256) {
        const int i = e / r, j = e % r;
        R[i][j] = (j >= i) ? Rq[i][piv[j]] : 0.0;
    }
    if (t < r) rdg[t] = 1.0 / Rq[t][piv[t]];
    __syncthreads();
    // inverse of R, column c per thread (back substitution with the reciprocal
    // diagonal)
    if (t < r) {
        const int c = t;
        for (int i = c; i >= 0; --i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int j = i + 1; j <= c; ++j) s -= R[i][j] * Ri[j][c];
            Ri[i][c] = s * rdg[i];
        }
    }
    __syncthreads();
    // B[perm[j]][c] = (R^-1)[j][c]: upper triangular, only j <= c was formed
    for (int e = t; e < r * r; e += 256) {
        const int j = e / r, c = e % r;
        Bq[piv[j]][c] = j <= c ? Ri[j][c] : 0.0;
    }
    __syncthreads();
    // M = [-S B; B]
    for (int e = t; e < (m + b) * b; e += 256) {
        const int q = e / b, c = e % b;
        double v;
        if (q < m) {
            v = 0.0;
            for (int j = 0; j < b; ++j) v = fma(-Ss[q][j], Bq[j][c], v);
        } else {
            v = Bq[q - m][c];
        }
        Cout[(int64_t)q * ldc + c] = v;
    }
    if (t == 0) *rank_out = r;
}

hipError_t launch_pchol(const double *G, int ldg, int b, const double *S, int lds, int m, const double *ref,
                        int ref_stride, double rel, double *C, int ldc, int32_t *rank, hipStream_t st)
{
    if (b <= 0 || b > PCH_MAX || m < 0 || m > PCH_M || (m > 0 && S == nullptr)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pchol, dim3(1), dim3(256), 0, st, G, ldg, b, S, lds, m, ref, ref_stride, rel, C, ldc, rank);
    return hipGetLastError();
}

// G = diag(theta) on its leading m x m block (the projected matrix in the
// Ritz basis after a rotation or a thick restart)
__global__ void k_g_ritz(double *G, int ldg, int m, const double *__restrict__ theta)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * m) return;
    const int r = t / m, c = t % m;
    G[(int64_t)r * ldg + c] = (r == c) ? theta[r] : 0.0;
}

hipError_t launch_g_ritz(double *G, int ldg, int m, const double *theta, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_g_ritz, dim3((m * m + 255) / 256), dim3(256), 0, st, G, ldg, m, theta);
    return hipGetLastError();
}

// G[a][b] symmetric fill of a new column block from computed rows
// G0[r][c] = H[idx[r]][idx[c]], r, c < ns: a principal submatrix of H
__global__ void k_gather_principal(const double *__restrict__ H, int64_t ld, const int32_t *__restrict__ idx, int ns,
                                   double *__restrict__ G, int ldg)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns * ns) return;
    const int r = t / ns, c = t % ns;
    G[(int64_t)r * ldg + c] = H[(int64_t)idx[r] * ld + idx[c]];
}

hipError_t launch_gather_principal(const double *H, int64_t ld, const int32_t *idx, int ns, double *G, int ldg,
                                   hipStream_t st)
{
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_principal, dim3((ns * ns + 255) / 256), dim3(256), 0, st, H, ld, idx, ns, G, ldg);
    return hipGetLastError();
}

// V[c][idx[r]] = Y[r][c] for r < ns, c < b (the rest of V's rows already zero)
__global__ void k_seed_scatter(double *V, int64_t ldv, const int32_t *__restrict__ idx, const double *__restrict__ Y,
                               int ldy, int ns, int b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns * b) return;
    const int r = t / b, c = t % b;
    V[(int64_t)c * ldv + idx[r]] = Y[(int64_t)r * ldy + c];
}

hipError_t launch_seed_scatter(double *V, int64_t ldv, const int32_t *idx, const double *Y, int ldy, int ns, int b,
                               hipStream_t st)
{
    if (ns <= 0 || b <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seed_scatter, dim3((ns * b + 255) / 256), dim3(256), 0, st, V, ldv, idx, Y, ldy, ns, b);
    return hipGetLastError();
}

__global__ void k_unit_vectors(double *V, int64_t ldv, int D, const int32_t *idx, int b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i < D && c < b) V[(int64_t)c * ldv + i] = (i == idx[c]) ? 1.0 : 0.0;
}

hipError_t launch_unit_vectors(double *V, int64_t ldv, int D, const int32_t *idx, int b, hipStream_t st)
{
    if (b <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unit_vectors, dim3((D + 255) / 256, b), dim3(256), 0, st, V, ldv, D, idx, b);
    return hipGetLastError();
}

}  // namespace cch
