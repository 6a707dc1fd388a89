// A mat-vec for L2-heavy matrices (Sec. 2.2: the off-diagonal pure-L2 class
// is the sparse one): W = H V with H split at Dc, the first L2 row, into
//   [ Hcc  Hcl ]   dense continuum rows and columns, read from the dense
//   [ Hlc  Hll ]   matrix; Hll (classes 2 and 8) as CSR,
// so that a block of b <= 16 vectors costs the continuum panels plus the
// non-zeros of the L2 block instead of the whole dense matrix.
//   W[:, c <  Dc] = sum over all rows of H[row][c] V[row]       (panel A)
//   W[:, c >= Dc] = sum over rows < Dc of H[row][c] V[row]      (panel B)
//                 + sum over the non-zeros of L2 row c - Dc     (CSR part)
// Every sum has a fixed order, so the result does not depend on timing.
#include <algorithm>

#include "ccham_internal.h"

namespace cch {

// ---------------------------------------------------------------------------
// CSR of the L2 block from the dense matrix (both triangles present)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_l2_nnz(const double *__restrict__ H, int64_t ld, int Dc, int nl2,
                                                int64_t *__restrict__ cnt)
{
    __shared__ int red[256];
    const int r = blockIdx.x;
    const double *row = H + (int64_t)(Dc + r) * ld + Dc;
    int c = 0;
    for (int j = threadIdx.x; j < nl2; j += 256) c += row[j] != 0.0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[r] = red[0];
}

// the non-zeros of L2 row r in column order, from offset off[r]
__global__ __launch_bounds__(256) void k_l2_fill(const double *__restrict__ H, int64_t ld, int Dc, int nl2,
                                                 const int64_t *__restrict__ off, int32_t *__restrict__ col,
                                                 double *__restrict__ val)
{
    __shared__ int wsum[4];
    const int r = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double *row = H + (int64_t)(Dc + r) * ld + Dc;
    int64_t base = off[r];
    for (int j0 = 0; j0 < nl2; j0 += 256) {
        const int j = j0 + threadIdx.x;
        const double v = j < nl2 ? row[j] : 0.0;
        const bool nz = v != 0.0;
        const unsigned long long m = __ballot(nz);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wv] = __popcll(m);
        __syncthreads();
        int woff = 0;
        for (int w = 0; w < wv; ++w) woff += wsum[w];
        const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (nz) {
            col[base + woff + before] = j;
            val[base + woff + before] = v;
        }
        base += tot;
        __syncthreads();   // wsum is written again by the next tile
    }
}

hipError_t launch_l2_csr_count(const double *H, int64_t ld, int Dc, int nl2, int64_t *cnt, hipStream_t st)
{
    if (nl2 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_l2_nnz, dim3(nl2), dim3(256), 0, st, H, ld, Dc, nl2, cnt);
    return hipGetLastError();
}

hipError_t launch_l2_csr_fill(const double *H, int64_t ld, int Dc, int nl2, const int64_t *off, int32_t *col,
                              double *val, hipStream_t st)
{
    if (nl2 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_l2_fill, dim3(nl2), dim3(256), 0, st, H, ld, Dc, nl2, off, col, val);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Panel mat-vec on FP64 MFMA 16x16x4: Wp[split][q][c - c0] = sum over the
// rows of the split (inside [r0, r1)) of H[row][c] V[q][row], c in [c0, c1).
// One wave owns 64 columns (four 16-column strips sharing the V fragment);
// the B operand is 4 rows x 16 columns of H, the A operand 16 vectors x the
// same 4 rows (zero rows for q >= b).
// ---------------------------------------------------------------------------
typedef double px4 __attribute__((ext_vector_type(4)));
constexpr int PN_U = 8;   // 4-row MFMA steps per register block

__global__ __launch_bounds__(256) void k_panel_mfma(const double *__restrict__ H, int64_t ld, int hc0, int r0, int r1,
                                                    int c0, int c1, const double *__restrict__ V, int64_t ldv, int b,
                                                    int rps, double *__restrict__ Wp)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cb0 = c0 + (blockIdx.x * 4 + wv) * 64;
    const int q = lane & 15, kq = lane >> 4;
    const int rb = r0 + blockIdx.y * rps, re = min(r1, rb + rps);
    const bool qok = q < b;
    const double *vrow = V + (int64_t)(qok ? q : 0) * ldv;
    const double *hcol[4];
    bool colok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = cb0 + 16 * t + q;
        colok[t] = c < c1;
        hcol[t] = H + (colok[t] ? c - hc0 : 0);   // column c of the matrix is column c - hc0 of H
    }
    px4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (px4){0.0, 0.0, 0.0, 0.0};
    for (int k0 = rb; k0 < re; k0 += 4 * PN_U) {
        double bv[PN_U][4], av[PN_U];
#pragma unroll
        for (int u = 0; u < PN_U; ++u) {
            const int row = k0 + 4 * u + kq;
            const bool ok = row < re;
            av[u] = (ok && qok) ? vrow[row] : 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                bv[u][t] = (ok && colok[t]) ? __builtin_nontemporal_load(hcol[t] + (int64_t)row * ld) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PN_U; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u][t], acc[t], 0, 0, 0);
    }
    // item v of lane l: vector l/16 + 4 v, column l % 16 of the strip
    const int nc = c1 - c0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = cb0 + 16 * t + q;
        if (colok[t]) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int qq = kq + 4 * v;
                if (qq < b) Wp[((int64_t)blockIdx.y * 16 + qq) * nc + (c - c0)] = acc[t][v];
            }
        }
    }
}

// W[q][c] = sum of the splits in order, c in [c0, c1)
__global__ void k_panel_reduce(const double *__restrict__ Wp, int ns, int c0, int c1, int b, double *__restrict__ W,
                               int64_t ldw)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x, qq = blockIdx.y;
    const int nc = c1 - c0;
    if (i >= nc || qq >= b) return;
    double s = 0.0;
    for (int k = 0; k < ns; ++k) s += Wp[((int64_t)k * 16 + qq) * nc + i];
    W[(int64_t)qq * ldw + c0 + i] = s;
}

// VT[i][q] = V[q][i] (0 for q >= b), i < D: the vectors of one row in one
// aligned 128-byte line for the gathers of the sparse product
__global__ void k_vt16(const double *__restrict__ V, int64_t ldv, int D, int b, double *__restrict__ VT)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= D) return;
#pragma unroll
    for (int q = 0; q < 16; ++q) VT[(int64_t)i * 16 + q] = q < b ? V[(int64_t)q * ldv + i] : 0.0;
}

// W[q][Dc + r] (+)= sum over the non-zeros (j, v) of L2 row r of v VT[Dc + j][q]
// (added to panel B's sums when there are continuum rows, else assigned):
// one wave per row, lanes over the non-zeros, a fixed-order tree across lanes
__global__ __launch_bounds__(256) void k_l2_spmm(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                 const double *__restrict__ val, int Dc, int nl2,
                                                 const double *__restrict__ VT, int b, double *__restrict__ W,
                                                 int64_t ldw, int accumulate)
{
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nl2) return;   // the whole wave
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    const px4 *vl = reinterpret_cast<const px4 *>(VT + (int64_t)Dc * 16);
    for (int64_t e = off[r] + lane; e < off[r + 1]; e += 64) {
        const double v = val[e];
        const px4 *x = vl + (int64_t)col[e] * 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const px4 y = x[u];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[4 * u + t] = fma(v, y[t], acc[4 * u + t]);
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        double s = acc[q];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        acc[q] = s;
    }
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (q < b) W[(int64_t)q * ldw + Dc + r] = accumulate ? W[(int64_t)q * ldw + Dc + r] + acc[q] : acc[q];
}

// splits of a panel: enough waves to cover HBM latency (about 4096), at most 64
static int panel_splits(int rows, int cols)
{
    const int waves = std::max(1, (cols + 63) / 64);
    int ks = (4096 + waves - 1) / waves;
    ks = std::max(1, std::min(ks, 64));
    return std::min(ks, std::max(1, (rows + 4 * PN_U - 1) / (4 * PN_U)));
}

// doubles of scratch that launch_matvec_l2csr needs
int64_t l2csr_scratch(int D, int Dc)
{
    const int64_t a = (int64_t)panel_splits(D, Dc) * 16 * std::max(Dc, 1);
    const int64_t b = (int64_t)panel_splits(Dc, D - Dc) * 16 * std::max(D - Dc, 1);
    return a + b + (int64_t)16 * D;   // panel partials, then the transposed block
}

static hipError_t panel(const double *H, int64_t ld, int hc0, int r0, int r1, int c0, int c1, const double *V,
                        int64_t ldv, int b, double *W, int64_t ldw, double *Wp, hipStream_t st)
{
    if (r1 <= r0 || c1 <= c0) return hipSuccess;
    const int ns = panel_splits(r1 - r0, c1 - c0);
    int rps = (r1 - r0 + ns - 1) / ns;
    rps = (rps + 4 * PN_U - 1) / (4 * PN_U) * (4 * PN_U);
    const int nsu = (r1 - r0 + rps - 1) / rps;
    hipLaunchKernelGGL(k_panel_mfma, dim3((c1 - c0 + 255) / 256, nsu), dim3(256), 0, st, H, ld, hc0, r0, r1, c0, c1, V,
                       ldv, b, rps, Wp);
    hipLaunchKernelGGL(k_panel_reduce, dim3((c1 - c0 + 255) / 256, b), dim3(256), 0, st, Wp, nsu, c0, c1, b, W, ldw);
    return hipGetLastError();
}

// P: rows 0..D-1, columns < Dc (leading dimension ldp); R: rows < Dc, the
// matrix's column c >= Dc at R column c - rc0 (leading dimension ldr). The
// dense matrix passes itself for both (rc0 = 0); a sparse-L2 matrix its two
// panels (rc0 = Dc).
hipError_t launch_matvec_l2csr(const double *P, int64_t ldp, const double *R, int64_t ldr, int rc0, int D, int Dc,
                               const int64_t *off, const int32_t *col, const double *val, const double *V,
                               int64_t ldv, int b, double *W, int64_t ldw, double *Wp, hipStream_t st)
{
    if (D <= 0 || b <= 0) return hipSuccess;
    if (Dc < 0 || Dc > D) return hipErrorInvalidValue;
    const int nl2 = D - Dc;
    double *WpA = Wp, *WpB = Wp + (int64_t)panel_splits(D, Dc) * 16 * std::max(Dc, 1);
    double *VT = WpB + (int64_t)panel_splits(Dc, D - Dc) * 16 * std::max(D - Dc, 1);   // 128-byte aligned
    for (int q0 = 0; q0 < b; q0 += 16) {
        const int bb = std::min(16, b - q0);
        const double *Vq = V + (int64_t)q0 * ldv;
        double *Wq = W + (int64_t)q0 * ldw;
        hipError_t e = panel(P, ldp, 0, 0, D, 0, Dc, Vq, ldv, bb, Wq, ldw, WpA, st);   // columns < Dc, all rows
        if (e == hipSuccess) e = panel(R, ldr, rc0, 0, Dc, Dc, D, Vq, ldv, bb, Wq, ldw, WpB, st);   // rows < Dc
        if (e != hipSuccess) return e;
        if (nl2 > 0) {
            hipLaunchKernelGGL(k_vt16, dim3((D + 255) / 256), dim3(256), 0, st, Vq, ldv, D, bb, VT);
            hipLaunchKernelGGL(k_l2_spmm, dim3((nl2 + 3) / 4), dim3(256), 0, st, off, col, val, Dc, nl2, VT, bb, Wq,
                               ldw, Dc > 0 ? 1 : 0);
        }
    }
    return hipGetLastError();
}

}  // namespace cch
