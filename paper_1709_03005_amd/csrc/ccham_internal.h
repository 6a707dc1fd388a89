// Internal declarations shared by the ccham kernels and the host runtime.
// Device helpers here implement Slater's rules on bitstring determinants
// (Sec. 2.1 of the MPI-SCATCI paper: XOR + popcount for the excitation
// degree, masks counting the occupied spin-orbitals between the differing
// ones for the sign), written for 64-bit words on gfx950.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define CCH_MAXW 4          // up to 256 target spin-orbitals per determinant
#define CCH_NOLAB 0xFFFFu

namespace cch {

// ---------------------------------------------------------------------------
// bit helpers (no shift by 64 anywhere: an index that is a multiple of 64 is
// the case the paper singles out for wrong masks)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t lowmask(int x)   // bits [0, x), x clamped to [0, 64]
{
    return x >= 64 ? ~0ull : (x <= 0 ? 0ull : ((1ull << x) - 1ull));
}

template <int W>
__device__ __forceinline__ int count_between(const uint64_t *d, int lo, int hi)
{
    // set bits of d strictly between spin-orbitals lo < hi
    int c = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int b = 64 * w;
        uint64_t m = lowmask(hi - b) & ~lowmask(lo + 1 - b);
        c += __popcll(d[w] & m);
    }
    return c;
}

template <int W>
__device__ __forceinline__ int first_bits(const uint64_t *x, int *out, int maxn)
{
    // ascending indices of the set bits of x (at most maxn)
    int n = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint64_t v = x[w];
        while (v && n < maxn) {
            out[n++] = 64 * w + (int)__builtin_ctzll(v);
            v &= v - 1;
        }
    }
    return n;
}

// the two lowest set bits of x, ascending (-1 where absent), without loops
// or branches: each word offers its lowest bit and the bit after it, and the
// first two offers found in word order are kept (the excitation scan runs
// this for every determinant pair, with lanes of one wave on different pairs)
template <int W>
__device__ __forceinline__ void low_two(const uint64_t *x, int *b0, int *b1)
{
    int f0 = -1, f1 = -1;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint64_t v = x[w], rest = v & (v - 1ull);
        const int t0 = v ? 64 * w + (int)__builtin_ctzll(v) : -1;
        const int t1 = rest ? 64 * w + (int)__builtin_ctzll(rest) : -1;
        f1 = f0 < 0 ? t1 : (f1 < 0 ? t0 : f1);
        f0 = f0 < 0 ? t0 : f0;
    }
    *b0 = f0;
    *b1 = f1;
}

__device__ __forceinline__ uint64_t pack_label(int f0, int f1, int f2, int f3)
{
    return (uint64_t)(uint16_t)f0 | ((uint64_t)(uint16_t)f1 << 16) |
           ((uint64_t)(uint16_t)f2 << 32) | ((uint64_t)(uint16_t)f3 << 48);
}

__device__ __forceinline__ int lab_field(uint64_t lab, int f) { return (int)((lab >> (16 * f)) & 0xFFFFu); }

// Excitation of bra A from ket B, equal electron counts. Returns the degree
// (0..2) or 3 when more than a double substitution apart. Holes = B & ~A,
// particles = A & ~B, ascending, paired in order; sign of
// A = s a+_p2 a_h2 a+_p1 a_h1 B.
template <int W>
__device__ __forceinline__ int excite(const uint64_t *A, const uint64_t *B, int *h, int *p, int *sign)
{
    int x = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) x += __popcll(A[w] ^ B[w]);
    if (x > 4) return 3;
    const int deg = x >> 1;
    if (deg == 0) { *sign = 1; return 0; }
    uint64_t hb[W], pb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { hb[w] = B[w] & ~A[w]; pb[w] = A[w] & ~B[w]; }
    low_two<W>(hb, &h[0], &h[1]);
    low_two<W>(pb, &p[0], &p[1]);
    int c = count_between<W>(B, min(h[0], p[0]), max(h[0], p[0]));
    if (deg == 2) {
        uint64_t B2[W];
#pragma unroll
        for (int w = 0; w < W; ++w) B2[w] = B[w];
        B2[h[0] >> 6] ^= 1ull << (h[0] & 63);
        B2[p[0] >> 6] ^= 1ull << (p[0] & 63);
        c += count_between<W>(B2, min(h[1], p[1]), max(h[1], p[1]));
    }
    *sign = (c & 1) ? -1 : 1;
    return deg;
}

// Continuum function (target det D of N electrons plus the alpha continuum
// electron above every target spin-orbital, index `top` = 2 n_o) as bra,
// against an L2 det L (N+1 target electrons) as ket. Returns the degree of
// the (N+1)-electron pair (1..2) or 3. h[0..deg) = holes (in L), pt = the
// target particle (in D) for degree 2.
template <int W>
__device__ __forceinline__ int excite_cont_l2(const uint64_t *D, const uint64_t *L, int top, int *h,
                                              int *pt, int *sign)
{
    int x = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) x += __popcll(D[w] ^ L[w]);
    if (x > 3 || !(x & 1)) return 3;
    const int deg = (x + 1) >> 1;   // 1 or 2
    uint64_t hb[W], pb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) { hb[w] = L[w] & ~D[w]; pb[w] = D[w] & ~L[w]; }
    low_two<W>(hb, &h[0], &h[1]);
    int c;
    if (deg == 1) {
        *pt = -1;
        c = count_between<W>(L, h[0], top);
    } else {
        int unused;
        low_two<W>(pb, pt, &unused);
        c = count_between<W>(L, min(h[0], *pt), max(h[0], *pt));
        uint64_t L2[W];
#pragma unroll
        for (int w = 0; w < W; ++w) L2[w] = L[w];
        L2[h[0] >> 6] ^= 1ull << (h[0] & 63);
        L2[*pt >> 6] ^= 1ull << (*pt & 63);
        c += count_between<W>(L2, h[1], top);
    }
    *sign = (c & 1) ? -1 : 1;
    return deg;
}

// ---------------------------------------------------------------------------
// integrals over target orbitals
// ---------------------------------------------------------------------------
struct TgtInts {
    const double *h;      // full one-electron matrix [n_orb][n_orb]
    const double *tttt;   // [n_o]^4
    int n_o, n_orb;
    double e_core;
};

__device__ __forceinline__ double g4(const TgtInts &I, int P, int Q, int R, int S)
{
    return I.tttt[(((size_t)P * I.n_o + Q) * I.n_o + R) * I.n_o + S];
}

// <A|H|B> for target-only determinants connected by degree 0..2, from the
// excitation (holes h, particles p, sign s). The degree-1 sum runs over all
// of B: its k = h term cancels exactly.
template <int W>
__device__ double sc_value(const TgtInts &I, const uint64_t *A, const uint64_t *B, int deg,
                           const int *h, const int *p, int s)
{
    if (deg == 0) {
        int occ[64];
        uint64_t t[W];
#pragma unroll
        for (int w = 0; w < W; ++w) t[w] = A[w];
        const int n = first_bits<W>(t, occ, 64);
        double e = I.e_core, e2 = 0.0;
        for (int a = 0; a < n; ++a) {
            const int ka = occ[a], Pa = ka >> 1;
            e += I.h[(size_t)Pa * I.n_orb + Pa];
            for (int b = 0; b < a; ++b) {
                const int kb = occ[b], Pb = kb >> 1;
                double v = g4(I, Pa, Pa, Pb, Pb);
                if ((ka & 1) == (kb & 1)) v -= g4(I, Pa, Pb, Pb, Pa);
                e2 += v;
            }
        }
        return e + e2;
    }
    if (deg == 1) {
        if ((h[0] & 1) != (p[0] & 1)) return 0.0;
        const int P = p[0] >> 1, H = h[0] >> 1, sp = p[0] & 1;
        double v = I.h[(size_t)P * I.n_orb + H];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            uint64_t x = B[w];
            while (x) {
                const int k = 64 * w + (int)__builtin_ctzll(x);
                x &= x - 1;
                const int K = k >> 1;
                v += g4(I, P, H, K, K);
                if ((k & 1) == sp) v -= g4(I, P, K, K, H);
            }
        }
        return s * v;
    }
    // degree 2
    double v = 0.0;
    if ((p[0] & 1) == (h[0] & 1) && (p[1] & 1) == (h[1] & 1))
        v += g4(I, p[0] >> 1, h[0] >> 1, p[1] >> 1, h[1] >> 1);
    if ((p[0] & 1) == (h[1] & 1) && (p[1] & 1) == (h[0] & 1))
        v -= g4(I, p[0] >> 1, h[1] >> 1, p[1] >> 1, h[0] >> 1);
    return s * v;
}

// ---------------------------------------------------------------------------
// pair lists
// ---------------------------------------------------------------------------
struct PairList {
    int32_t *x, *y;      // bra index, ket index
    int8_t *deg;
    int8_t *phase;
    uint64_t *label;
};

enum ScanMode { SCAN_TT = 0, SCAN_LL = 1, SCAN_LT = 2 };

// the symmetry-packed two-continuum integrals, for one relayout launch: record
// of the target pair (P, Q) at rec[P * n_o + Q]; inside it, the (tt|cc) rows
// of this launch start at boffJ (row length ncb), the (tc|tc) block of the
// second symmetry's irrep at boffK (row length nca_full, rows from column jr0)
struct PackedCC {
    const int64_t *rec;
    int64_t boffJ, boffK;
    int jr0, nca_full;
};

// work vectors of the Householder tridiagonalisation (length n each): wp =
// the current column after the panel's corrections, p = tau_j A_j v_j; the
// diagonal d, the off-diagonal e and the reflector scalars tau of T
struct TrdVec {
    double *wp, *p;
    double *d, *e, *tau;
};

// columns per panel of the blocked tridiagonalisation
constexpr int TRD_NB = 32;
// rows per workgroup of the column kernel, and the stride of its partial sums
constexpr int TRD_CR = 256, TRD_PS = 2 * TRD_NB + 8;
constexpr int TRD_PT = 2 * TRD_NB;   // doubles per row of PVt
// trailing blocks of at least TRD_TILE_MIN rows are multiplied from their
// lower triangle in TRD_TT x TRD_TT tiles (below that the row pass reads
// whole rows)
constexpr int TRD_TT = 128, TRD_TILE_MIN = 3072;
constexpr int TRD_SR = 32;   // rows per workgroup of the tiled pass's row sums
struct TrdPanel {
    double *PV, *PW;   // 2 TRD_NB rows each, ldp doubles a row (the panel update's operands)
    int64_t ldp;
    double *PVt;       // PV by matrix row: PVt[r][d] = PV[d][r], 2 TRD_NB doubles a row
    double *part1;     // column kernel: TRD_PS partial sums per workgroup
    double *part2;     // row pass: one partial sum per workgroup
    double *rowp, *colp;   // tiled pass: [tile column][n] row sums, [tile row][n] column sums
    double *z;             // tiled pass: z[d] of its reflector (2 TRD_NB)
};

// tiles per side of the tiled pass over m trailing rows
__host__ __device__ inline int trd_tiles(int m) { return (m + TRD_TT - 1) / TRD_TT; }

// doubles of the panel buffers for dimension n with rows of ldp doubles
inline size_t trd_panel_doubles(int n, int64_t ldp)
{
    const size_t T = (size_t)trd_tiles(n);
    return (size_t)2 * TRD_NB * n + (size_t)4 * TRD_NB * ldp + (size_t)((n + TRD_CR - 1) / TRD_CR) * TRD_PS +
           (size_t)(n + 3) / 4 + 2 * T * (size_t)n + 2 * TRD_NB;
}

// a matrix whose L2 block (classes 2 and 8) is held as CSR: P[r][c] for
// c < Dc (every row), R[r][c - Dc] for r < Dc <= c, and the L2 block's rows
// as CSR (columns relative to Dc, ascending)
// class 4 of one target symmetry (k_class4.hip)
struct Class4Args {
    const uint64_t *tdets;   // target dets of the symmetry [M][W]
    const int8_t *cspin;     // continuum spin per target det (0 alpha, 1 beta); nullptr: alpha
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

// one (instance, symmetry) block of the persistent class-4 launch
struct C4Task {
    Class4Args a;
    int n_l2, jtiles;
    int64_t first;   // first global work item of this block
};

// continuum orbitals per class-4 workgroup (the j block of one L2 row)
constexpr int C4_JB = 512;

struct SparseMat {
    const double *P;
    int64_t ldp;
    const double *R;
    int64_t ldr;
    const int64_t *off;
    const int32_t *col;
    const double *val;
    int64_t Dc;
};

}  // namespace cch

// ---------------------------------------------------------------------------
// kernel launchers (host side, defined in the .hip files)
// ---------------------------------------------------------------------------
namespace cch {
// the Ritz pairs whose corrections a Davidson step forms (output c uses pair
// e[c]), passed to the kernels by value
struct DavSel {
    int32_t e[32];
};

struct GemmDesc;
hipError_t launch_scan(int mode, int W, const uint64_t *A, int nA, const uint64_t *B, int nB,
                       int top, const int64_t *row_off, int64_t *row_cnt, PairList out,
                       hipStream_t st);
hipError_t launch_exclusive_scan(const int64_t *in, int64_t *out, int n, int64_t *total,
                                 hipStream_t st);
hipError_t launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t st);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t st);
}  // namespace cch
