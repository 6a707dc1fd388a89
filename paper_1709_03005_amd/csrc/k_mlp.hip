// Learned Davidson preconditioner: a 3-layer perceptron (4 -> 128 -> 128 -> 1,
// ReLU) maps per-row features of a Ritz pair to g, and the correction of row
// i becomes t_i = exp(clamp(g_i, -4, 4)) * r_i / (theta - H_ii), i.e. a learned
// per-row rescaling of the diagonal (Jacobi) step, which stays the fallback.
//
// Precision: FP32 master weights and Adam moments; the 128 x 128 layer and
// its two backward products run on v_mfma_f32_16x16x32_bf16 (BF16 operands,
// FP32 accumulation); the 4 -> 128 and 128 -> 1 layers in FP32.
//
// Training loss over rows r with weights w_r, Jacobi step tj_r and target
// correction e_r (the exact eigenvector error):
//     L = sum_r w_r (exp(g_r) tj_r - e_r)^2.
// Gradients are accumulated per workgroup (row tiles in a fixed order) and
// reduced in a fixed order: training steps are deterministic.
//
// MFMA bf16 16x16x32 lanes: A[l%16][8(l/16)+e], B[8(l/16)+e][l%16];
// result item v of lane l is D[4(l/16)+v][l%16].
#include "ccham_internal.h"

namespace cch {

constexpr int MLP_IN = 4, MLP_H = 128, MLP_TILE = 64;
// parameter blob layout (FP32): W1[128][4], b1[128], W2[128][128], b2[128], w3[128], b3
constexpr int P_W1 = 0, P_B1 = P_W1 + MLP_H * MLP_IN, P_W2 = P_B1 + MLP_H, P_B2 = P_W2 + MLP_H * MLP_H,
              P_W3 = P_B2 + MLP_H, P_B3 = P_W3 + MLP_H, P_TOTAL = P_B3 + 1;
constexpr float G_CLAMP = 4.0f;

typedef float fx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

int mlp_num_params() { return P_TOTAL; }

// BF16 copies of W2 (row-major [j][k]) and its transpose ([k][j])
__global__ void k_mlp_pack(const float *__restrict__ w, __bf16 *__restrict__ w2, __bf16 *__restrict__ w2t)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= MLP_H * MLP_H) return;
    const int j = t / MLP_H, k = t % MLP_H;
    const float v = w[P_W2 + t];
    w2[j * MLP_H + k] = (__bf16)v;
    w2t[k * MLP_H + j] = (__bf16)v;
}

hipError_t launch_mlp_pack(const float *w, __bf16 *w2, __bf16 *w2t, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3((MLP_H * MLP_H + 255) / 256), dim3(256), 0, st, w, w2, w2t);
    return hipGetLastError();
}

struct MlpShared {
    float x[MLP_TILE][MLP_IN];
    __attribute__((aligned(16))) __bf16 h1[MLP_TILE][MLP_H + 8];     // [r][k]
    __attribute__((aligned(16))) __bf16 h1t[MLP_H][MLP_TILE + 8];    // [k][r]
    float z2[MLP_TILE][MLP_H + 1];                                   // pre-activation of layer 2
    __attribute__((aligned(16))) __bf16 d2[MLP_TILE][MLP_H + 8];     // dL/dz2 [r][j]
    __attribute__((aligned(16))) __bf16 d2t[MLP_H][MLP_TILE + 8];    // [j][r]
    float d1[MLP_TILE][MLP_H + 1];                                   // dL/dz1
    float g[MLP_TILE], dg[MLP_TILE];
    float gW1[MLP_H * MLP_IN], gb1[MLP_H], gb2[MLP_H], gW3[MLP_H];
    float loss[MLP_TILE];
};

// Rows [0, n) in tiles of 64, tile t handled by workgroup t % grid (fixed).
// TRAIN: X, tj, e, wr -> partial gradients part[blockIdx][P_TOTAL] and partial
// losses lpart[blockIdx]; else X -> gout.
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp_main(const float *__restrict__ w, const __bf16 *__restrict__ w2,
                                                  const __bf16 *__restrict__ w2t, const float *__restrict__ X,
                                                  int64_t n, float *__restrict__ gout, const float *__restrict__ tj,
                                                  const float *__restrict__ ev, const float *__restrict__ wr,
                                                  float *__restrict__ part, double *__restrict__ lpart)
{
    __shared__ MlpShared s;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // dW2 rows j in [32 wv, 32 wv + 32): 2 x 8 MFMA tiles held across row tiles
    fx4 gw2[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) gw2[a][b] = (fx4){0.f, 0.f, 0.f, 0.f};
    if (TRAIN) {
        for (int i = tid; i < MLP_H * MLP_IN; i += 256) s.gW1[i] = 0.f;
        for (int i = tid; i < MLP_H; i += 256) {
            s.gb1[i] = 0.f;
            s.gb2[i] = 0.f;
            s.gW3[i] = 0.f;
        }
    }
    float gb3 = 0.f;
    double lsum = 0.0;
    const int64_t ntiles = (n + MLP_TILE - 1) / MLP_TILE;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * MLP_TILE;
        __syncthreads();
        for (int i = tid; i < MLP_TILE * MLP_IN; i += 256) {
            const int r = i / MLP_IN, f = i % MLP_IN;
            s.x[r][f] = (r0 + r < n) ? X[(r0 + r) * MLP_IN + f] : 0.f;
        }
        __syncthreads();
        // layer 1 (FP32): h1 = relu(W1 x + b1)
        for (int i = tid; i < MLP_TILE * MLP_H; i += 256) {
            const int r = i / MLP_H, j = i % MLP_H;
            float z = w[P_B1 + j];
#pragma unroll
            for (int f = 0; f < MLP_IN; ++f) z = fmaf(w[P_W1 + j * MLP_IN + f], s.x[r][f], z);
            const float h = z > 0.f ? z : 0.f;
            s.h1[r][j] = (__bf16)h;
            s.h1t[j][r] = (__bf16)h;
        }
        __syncthreads();
        // layer 2 (BF16 MFMA): z2[r][j] = sum_k h1[r][k] W2[j][k] + b2[j]; wave: rows 16 wv..+16
        {
            fx4 acc[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[b] = (fx4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k0 = 0; k0 < MLP_H; k0 += 32) {
                const int kk = k0 + 8 * (lane >> 4);
                const bf16x8 a = *(const bf16x8 *)&s.h1[16 * wv + (lane & 15)][kk];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const bf16x8 bb = *(const bf16x8 *)&w2[(16 * b + (lane & 15)) * MLP_H + kk];
                    acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[b], 0, 0, 0);
                }
            }
#pragma unroll
            for (int b = 0; b < 8; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * wv + 4 * (lane >> 4) + v, j = 16 * b + (lane & 15);
                    s.z2[r][j] = acc[b][v] + w[P_B2 + j];
                }
        }
        __syncthreads();
        // layer 3 (FP32): g = w3 . relu(z2) + b3; four threads per row
        {
            const int r = tid >> 2, q = tid & 3;
            float p = 0.f;
            for (int j = q; j < MLP_H; j += 4) {
                const float h = s.z2[r][j] > 0.f ? s.z2[r][j] : 0.f;
                p = fmaf(w[P_W3 + j], h, p);
            }
            p += __shfl_xor(p, 1, 64);
            p += __shfl_xor(p, 2, 64);
            if (q == 0) s.g[r] = p + w[P_B3];
        }
        __syncthreads();
        if (!TRAIN) {
            for (int r = tid; r < MLP_TILE; r += 256)
                if (r0 + r < n) gout[r0 + r] = s.g[r];
            continue;
        }
        // loss and dL/dg
        for (int r = tid; r < MLP_TILE; r += 256) {
            float dg = 0.f, lr = 0.f;
            if (r0 + r < n) {
                const float g = s.g[r];
                const float gc = fminf(fmaxf(g, -G_CLAMP), G_CLAMP);
                const float y = expf(gc) * tj[r0 + r];
                const float d = y - ev[r0 + r];
                lr = wr[r0 + r] * d * d;
                dg = (g > -G_CLAMP && g < G_CLAMP) ? 2.f * wr[r0 + r] * d * y : 0.f;
            }
            s.dg[r] = dg;
            s.loss[r] = lr;
        }
        __syncthreads();
        if (tid == 0)
            for (int r = 0; r < MLP_TILE; ++r) {
                lsum += (double)s.loss[r];
                gb3 += s.dg[r];
            }
        // dW3, db2 and dz2 = dg w3 relu'(z2)
        for (int j = tid; j < MLP_H; j += 256) {
            float a3 = 0.f, a2 = 0.f;
            const float w3j = w[P_W3 + j];
            for (int r = 0; r < MLP_TILE; ++r) {
                const float z = s.z2[r][j];
                const float h = z > 0.f ? z : 0.f;
                a3 = fmaf(s.dg[r], h, a3);
                const float d = z > 0.f ? s.dg[r] * w3j : 0.f;
                a2 += d;
                s.d2[r][j] = (__bf16)d;
                s.d2t[j][r] = (__bf16)d;
            }
            s.gW3[j] += a3;
            s.gb2[j] += a2;
        }
        __syncthreads();
        // dW2[j][k] += sum_r d2[r][j] h1[r][k]: wave rows j in 32 wv..+32, K = 64 rows
#pragma unroll
        for (int r0k = 0; r0k < MLP_TILE; r0k += 32) {
            const int rr = r0k + 8 * (lane >> 4);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const bf16x8 av = *(const bf16x8 *)&s.d2t[32 * wv + 16 * a + (lane & 15)][rr];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const bf16x8 bv = *(const bf16x8 *)&s.h1t[16 * b + (lane & 15)][rr];
                    gw2[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, gw2[a][b], 0, 0, 0);
                }
            }
        }
        // dh1[r][k] = sum_j d2[r][j] W2[j][k]; wave rows 16 wv..+16
        {
            fx4 acc[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[b] = (fx4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int j0 = 0; j0 < MLP_H; j0 += 32) {
                const int jj = j0 + 8 * (lane >> 4);
                const bf16x8 a = *(const bf16x8 *)&s.d2[16 * wv + (lane & 15)][jj];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const bf16x8 bb = *(const bf16x8 *)&w2t[(16 * b + (lane & 15)) * MLP_H + jj];
                    acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[b], 0, 0, 0);
                }
            }
#pragma unroll
            for (int b = 0; b < 8; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * wv + 4 * (lane >> 4) + v, k = 16 * b + (lane & 15);
                    const float h = (float)s.h1[r][k];
                    s.d1[r][k] = h > 0.f ? acc[b][v] : 0.f;
                }
        }
        __syncthreads();
        // dW1, db1
        for (int i = tid; i < MLP_H * (MLP_IN + 1); i += 256) {
            const int j = i / (MLP_IN + 1), f = i % (MLP_IN + 1);
            float a = 0.f;
            for (int r = 0; r < MLP_TILE; ++r) a = fmaf(s.d1[r][j], f < MLP_IN ? s.x[r][f] : 1.f, a);
            if (f < MLP_IN) s.gW1[j * MLP_IN + f] += a;
            else s.gb1[j] += a;
        }
    }
    if (!TRAIN) return;
    __syncthreads();
    float *pp = part + (int64_t)blockIdx.x * P_TOTAL;
    for (int i = tid; i < MLP_H * MLP_IN; i += 256) pp[P_W1 + i] = s.gW1[i];
    for (int i = tid; i < MLP_H; i += 256) {
        pp[P_B1 + i] = s.gb1[i];
        pp[P_B2 + i] = s.gb2[i];
        pp[P_W3 + i] = s.gW3[i];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 32 * wv + 16 * a + 4 * (lane >> 4) + v, k = 16 * b + (lane & 15);
                pp[P_W2 + j * MLP_H + k] = gw2[a][b][v];
            }
    if (tid == 0) {
        pp[P_B3] = gb3;
        lpart[blockIdx.x] = lsum;
    }
}

__global__ void k_mlp_reduce(const float *__restrict__ part, int nblk, float *__restrict__ grad,
                             const double *__restrict__ lpart, double *__restrict__ loss)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P_TOTAL) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * P_TOTAL + i];
        grad[i] = (float)s;
    }
    if (i == 0 && loss) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += lpart[b];
        *loss = s;
    }
}

// Adam (FP32): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; w -= lr mhat/(sqrt(vhat)+eps)
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float b1, float b2, float eps, int step)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P_TOTAL) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.f - powf(b1, (float)step)), vh = vi / (1.f - powf(b2, (float)step));
    w[i] -= lr * mh / (sqrtf(vh) + eps);
}

int mlp_grid(int64_t n)
{
    const int64_t tiles = (n + MLP_TILE - 1) / MLP_TILE;
    return (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), 1024);
}

hipError_t launch_mlp_forward(const float *w, const __bf16 *w2, const __bf16 *w2t, const float *X, int64_t n,
                              float *g, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_mlp_main<false>), dim3(mlp_grid(n)), dim3(256), 0, st, w, w2, w2t, X, n, g,
                       (const float *)nullptr, (const float *)nullptr, (const float *)nullptr, (float *)nullptr,
                       (double *)nullptr);
    return hipGetLastError();
}

// gradient (and loss) of the training loss; part: mlp_grid(n) * P_TOTAL floats
hipError_t launch_mlp_grad(const float *w, const __bf16 *w2, const __bf16 *w2t, const float *X, const float *tj,
                           const float *ev, const float *wr, int64_t n, float *part, double *lpart, float *grad,
                           double *loss, hipStream_t st)
{
    const int grid = mlp_grid(n);
    hipLaunchKernelGGL((k_mlp_main<true>), dim3(grid), dim3(256), 0, st, w, w2, w2t, X, n, (float *)nullptr, tj, ev,
                       wr, part, lpart);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((P_TOTAL + 255) / 256), dim3(256), 0, st, part, grid, grad, lpart, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *w, float *m, float *v, const float *g, float lr, int step, hipStream_t st)
{
    hipLaunchKernelGGL(k_adam, dim3((P_TOTAL + 255) / 256), dim3(256), 0, st, w, m, v, g, lr, 0.9f, 0.999f, 1e-8f,
                       step);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Davidson glue
// ---------------------------------------------------------------------------
// features of row i for Ritz pair e = sel[c]: asinh(d), asinh(rho),
// asinh(rho/|d|), [i is an L2 row], with d = theta_e - H_ii (floored at 1e-8)
// and rho the off-diagonal 2-norm of row i
__device__ __forceinline__ void mlp_features(double th, double hii, double rho, int is_l2, float *f)
{
    double d = th - hii;
    if (fabs(d) < 1e-8) d = d < 0.0 ? -1e-8 : 1e-8;
    f[0] = (float)asinh(d);
    f[1] = (float)asinh(rho);
    f[2] = (float)asinh(rho / fabs(d));
    f[3] = (float)is_l2;
}

__global__ void k_mlp_dav_features(const double *__restrict__ diag, const double *__restrict__ rho, int D, int Dc,
                                   const double *__restrict__ theta, DavSel sel, int nsel, float *__restrict__ X)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= D || c >= nsel) return;
    float f[MLP_IN];
    mlp_features(theta[sel.e[c]], diag[i], rho[i], i >= Dc, f);
    for (int q = 0; q < MLP_IN; ++q) X[((int64_t)c * D + i) * MLP_IN + q] = f[q];
}

// t = exp(clamp(g)) r / den; a non-finite value falls back to the Jacobi step
__global__ void k_mlp_dav_correct(const double *__restrict__ R, int64_t ld, int D, const double *__restrict__ diag,
                                  const double *__restrict__ theta, DavSel sel, int nsel, const float *__restrict__ g, double *__restrict__ T, int64_t ldt,
                                  int32_t *__restrict__ nfallback)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= D || c >= nsel) return;
    const int e = sel.e[c];
    double den = theta[e] - diag[i];
    if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
    const double tj = R[(int64_t)e * ld + i] / den;
    const float gi = g[(int64_t)c * D + i];
    double t = tj * exp((double)fminf(fmaxf(gi, -G_CLAMP), G_CLAMP));
    if (!isfinite(t) || !isfinite(gi)) {
        t = tj;
        atomicAdd(nfallback, 1);
    }
    T[(int64_t)c * ldt + i] = t;
}

// off-diagonal 2-norm of every row of H
__global__ __launch_bounds__(256) void k_row_norms(const double *__restrict__ H, int64_t ld, int D,
                                                   double *__restrict__ rho)
{
    const int i = blockIdx.x;
    double s = 0.0;
    for (int j = threadIdx.x; j < D; j += 256) {
        const double v = j == i ? 0.0 : H[(int64_t)i * ld + j];
        s = fma(v, v, s);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) rho[i] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

hipError_t launch_row_norms(const double *H, int64_t ld, int D, double *rho, hipStream_t st)
{
    if (D <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_norms, dim3(D), dim3(256), 0, st, H, ld, D, rho);
    return hipGetLastError();
}

hipError_t launch_mlp_dav(const float *w, const __bf16 *w2, const __bf16 *w2t, const double *R, int64_t ld, int D,
                          int Dc, const double *diag, const double *rho, const double *theta, const DavSel &sel,
                          int nsel, float *X, float *g, double *T, int64_t ldt, int32_t *nfallback, hipStream_t st)
{
    if (nsel <= 0) return hipSuccess;
    if (nsel > 32) return hipErrorInvalidValue;
    const dim3 gr((D + 255) / 256, nsel);
    hipLaunchKernelGGL(k_mlp_dav_features, gr, dim3(256), 0, st, diag, rho, D, Dc, theta, sel, nsel, X);
    hipError_t e = launch_mlp_forward(w, w2, w2t, X, (int64_t)D * nsel, g, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_dav_correct, gr, dim3(256), 0, st, R, ld, D, diag, theta, sel, nsel, g, T, ldt,
                       nfallback);
    return hipGetLastError();
}

}  // namespace cch

namespace cch {
// features of every row for one Ritz value (training data)
__global__ void k_mlp_features_theta(const double *__restrict__ diag, const double *__restrict__ rho, int D, int Dc,
                                     double theta, float *__restrict__ X)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= D) return;
    float f[MLP_IN];
    mlp_features(theta, diag[i], rho[i], i >= Dc, f);
    for (int q = 0; q < MLP_IN; ++q) X[(int64_t)i * MLP_IN + q] = f[q];
}

hipError_t launch_mlp_features_theta(const double *diag, const double *rho, int D, int Dc, double theta, float *X,
                                     hipStream_t st)
{
    if (D <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_features_theta, dim3((D + 255) / 256), dim3(256), 0, st, diag, rho, D, Dc, theta, X);
    return hipGetLastError();
}
}  // namespace cch
