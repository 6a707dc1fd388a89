// Excitation scan over determinant pairs (Sec. 2.1, Slater's rules on
// bitstrings): every ket of a row is XORed with the row's bra and popcounted;
// pairs within a double substitution are compacted, in ket order, with their
// holes/particles packed into four 16-bit fields and the sign from masks.
// One workgroup per bra row; a count pass sizes the lists at plan time, the
// emit pass (same scan) writes them during the build. Integer work, bit-exact.
#include "ccham_internal.h"

namespace cch {

constexpr int SCAN_THREADS = 256;

template <int W, int MODE, bool EMIT>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan(const uint64_t *__restrict__ A, int nA,
                                                       const uint64_t *__restrict__ B, int nB,
                                                       int top, const int64_t *__restrict__ row_off,
                                                       int64_t *__restrict__ row_cnt, PairList out)
{
    const int x = blockIdx.x;
    if (x >= nA) return;
    uint64_t a[W];
#pragma unroll
    for (int w = 0; w < W; ++w) a[w] = A[(size_t)x * W + w];
    const int ylim = (MODE == SCAN_LL) ? x + 1 : nB;
    __shared__ int wave_tot[SCAN_THREADS / 64];
    __shared__ int64_t base_sh;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t base = EMIT ? row_off[x] : 0;
    int64_t cnt = 0;
    for (int y0 = 0; y0 < ylim; y0 += SCAN_THREADS) {
        const int y = y0 + threadIdx.x;
        int deg = 3, h[2] = {-1, -1}, p[2] = {-1, -1}, s = 1, pt = -1;
        if (y < ylim) {
            uint64_t b[W];
#pragma unroll
            for (int w = 0; w < W; ++w) b[w] = B[(size_t)y * W + w];
            if (MODE == SCAN_LT)
                deg = excite_cont_l2<W>(b, a, top, h, &pt, &s);   // bra = det y + continuum, ket = L2 x
            else
                deg = excite<W>(a, b, h, p, &s);
        }
        const bool conn = deg <= 2;
        if (!EMIT) {
            cnt += conn;
            continue;
        }
        const uint64_t bal = __ballot(conn);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wave_tot[wv] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < SCAN_THREADS / 64; ++k) {
            woff += (k < wv) ? wave_tot[k] : 0;
            tot += wave_tot[k];
        }
        if (conn) {
            const int64_t pos = base + woff + before;
            out.x[pos] = x;
            out.y[pos] = y;
            out.deg[pos] = (int8_t)deg;
            out.phase[pos] = (int8_t)s;
            uint64_t lab;
            if (MODE == SCAN_LT)
                lab = pack_label(deg == 2 ? pt : CCH_NOLAB, h[0], deg == 2 ? h[1] : CCH_NOLAB, CCH_NOLAB);
            else
                lab = pack_label(deg >= 1 ? p[0] : CCH_NOLAB, deg >= 1 ? h[0] : CCH_NOLAB,
                                 deg >= 2 ? p[1] : CCH_NOLAB, deg >= 2 ? h[1] : CCH_NOLAB);
            out.label[pos] = lab;
        }
        base += tot;
        __syncthreads();
    }
    if (!EMIT) {
        // block reduction of the per-thread counts
        __shared__ int64_t red[SCAN_THREADS];
        red[threadIdx.x] = cnt;
        __syncthreads();
        for (int o = SCAN_THREADS / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) row_cnt[x] = red[0];
    }
    (void)base_sh;
}

template <int W, int MODE>
static hipError_t scan_w(const uint64_t *A, int nA, const uint64_t *B, int nB, int top,
                         const int64_t *row_off, int64_t *row_cnt, PairList out, hipStream_t st)
{
    if (nA <= 0) return hipSuccess;
    if (row_off)
        hipLaunchKernelGGL((k_scan<W, MODE, true>), dim3(nA), dim3(SCAN_THREADS), 0, st, A, nA, B,
                           nB, top, row_off, row_cnt, out);
    else
        hipLaunchKernelGGL((k_scan<W, MODE, false>), dim3(nA), dim3(SCAN_THREADS), 0, st, A, nA, B,
                           nB, top, row_off, row_cnt, out);
    return hipGetLastError();
}

template <int MODE>
static hipError_t scan_mode(int W, const uint64_t *A, int nA, const uint64_t *B, int nB, int top,
                            const int64_t *row_off, int64_t *row_cnt, PairList out, hipStream_t st)
{
    switch (W) {
    case 1: return scan_w<1, MODE>(A, nA, B, nB, top, row_off, row_cnt, out, st);
    case 2: return scan_w<2, MODE>(A, nA, B, nB, top, row_off, row_cnt, out, st);
    case 3: return scan_w<3, MODE>(A, nA, B, nB, top, row_off, row_cnt, out, st);
    case 4: return scan_w<4, MODE>(A, nA, B, nB, top, row_off, row_cnt, out, st);
    }
    return hipErrorInvalidValue;
}

// mode SCAN_TT/SCAN_LL/SCAN_LT; row_off == nullptr: count pass into row_cnt,
// else emit pass writing pairs from row_off[x].
hipError_t launch_scan(int mode, int W, const uint64_t *A, int nA, const uint64_t *B, int nB, int top,
                       const int64_t *row_off, int64_t *row_cnt, PairList out, hipStream_t st)
{
    switch (mode) {
    case SCAN_TT: return scan_mode<SCAN_TT>(W, A, nA, B, nB, top, row_off, row_cnt, out, st);
    case SCAN_LL: return scan_mode<SCAN_LL>(W, A, nA, B, nB, top, row_off, row_cnt, out, st);
    case SCAN_LT: return scan_mode<SCAN_LT>(W, A, nA, B, nB, top, row_off, row_cnt, out, st);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// exclusive prefix sum of int64 counts, one workgroup (n up to a few 1e5)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_exscan(const int64_t *__restrict__ in, int64_t *__restrict__ out,
                                                 int n, int64_t *__restrict__ total)
{
    __shared__ int64_t buf[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < n; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int64_t v = i < n ? in[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int64_t t = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) out[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

hipError_t launch_exclusive_scan(const int64_t *in, int64_t *out, int n, int64_t *total, hipStream_t st)
{
    hipLaunchKernelGGL(k_exscan, dim3(1), dim3(1024), 0, st, in, out, n, total);
    return hipGetLastError();
}

}  // namespace cch
