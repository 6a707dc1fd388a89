/*
 * CPU oracle for the contracted close-coupling Hamiltonian.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do. It is deliberately plain and slow.
 *
 * What it computes, straight from the definitions:
 *   - the Hamiltonian of the (N+1)-electron problem (Sec. 2, Eq. 3),
 *       H = sum_pq h_pq a+_p a_q + 1/2 sum_pqrs (pq|rs) a+_p a+_r a_s a_q + E_core,
 *     between single determinants, by the Slater-Condon rules. The excitation
 *     (holes, particles, sign) is found by applying creation and annihilation
 *     operators to explicit ordered occupation lists (no bit masks);
 *   - the CI-contracted matrix (Sec. 2, Eqs. 4 and 5): for continuum rows
 *     (i,n,j) and columns (i',n',j'),
 *       Ht = sum_m sum_m' c_imn c_i'm'n' <eta_im u_ij | H | eta_i'm' u_i'j'>,
 *     for continuum rows against L2 columns Ht = sum_m c_imn <eta_im u_ij|H|chi_l>,
 *     and the pure L2 elements <chi_l|H|chi_l'> with no contraction (Sec. 2.2,
 *     classes 2 and 8).
 *
 * Conventions (fixed by the library's interface; the paper leaves them open):
 *   - spin-orbital k = 2*orbital + spin, alpha = 0; determinants are ascending
 *     products a+_k1 a+_k2 ... |0>, k1 < k2 < ...;
 *   - the continuum electron is the highest-indexed spin-orbital of a
 *     continuum function: u_j = 2*(n_o + j) + sigma, sigma its spin (0 alpha,
 *     1 beta; given per target determinant, alpha unless stated);
 *   - the only shortcut taken: a pair whose target parts differ in more than
 *     two spin-orbitals is skipped, since its (N+1)-electron determinants then
 *     differ in more than two as well and the Slater-Condon element is zero.
 *
 * Each element's sum is accumulated with Neumaier compensation, and the sum of
 * the absolute values of its terms plus the number of terms are returned for
 * the tolerance rule of the parity tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXE 128   /* electrons per determinant */

typedef struct {
    int32_t n_o, n_cont;
    const double *h;     /* [n_orb][n_orb] */
    const double *tttt;  /* [n_o]^4            (pq|rs)   */
    const double *tttc;  /* [n_o][n_o][n_o][nc] (pq|rj)  */
    const double *ttcc;  /* [n_o][n_o][nc][nc]  (pq|jj') */
    const double *tctc;  /* [n_o][nc][n_o][nc]  (pj|qj') */
    double e_core;
    /* symmetry-packed ttcc / tctc (pk_rec != NULL): record pk_rec[P * n_o + Q]
     * holds, for each continuum irrep ca, the block of n_c[ca] x n_c[ca ^ x]
     * values (x = irrep(P) ^ irrep(Q)) at offset pk_blk[x * n_irrep + ca];
     * values outside the blocks are zero by symmetry */
    const int64_t *pk_rec;
    const int64_t *pk_blk;
    int32_t n_irrep;
    const int32_t *t_irrep;   /* [n_o] */
    const int32_t *c_irrep;   /* [nc] */
    const int32_t *c_local;   /* [nc] index inside its irrep */
    const int32_t *c_count;   /* [n_irrep] */
} orc_ints;

/* (P Q | a b) of the packed layout, P, Q target, a, b continuum (local j) */
static double packed_cc(const orc_ints *I, const double *arr, int P, int Q, int a, int b)
{
    const int x = I->t_irrep[P] ^ I->t_irrep[Q], ca = I->c_irrep[a];
    if ((ca ^ I->c_irrep[b]) != x) return 0.0;
    return arr[I->pk_rec[(size_t)P * I->n_o + Q] + I->pk_blk[x * I->n_irrep + ca] +
               (int64_t)I->c_local[a] * I->c_count[ca ^ x] + I->c_local[b]];
}

typedef struct {
    orc_ints ints;
    int32_t n_elec;        /* N, target electrons */
    int32_t n_words;
    int32_t n_sym;
    int32_t n_l2;
    int32_t total_irrep;
    const int32_t *cont_start;   /* [n_irrep+1] first continuum index j of each irrep */
    const int32_t *sym_irrep;    /* [n_sym] */
    const int32_t *sym_ndet;     /* [n_sym] */
    const int32_t *sym_nstate;   /* [n_sym] */
    const uint64_t *const *sym_dets; /* [n_sym] -> [ndet][n_words] */
    const double *const *sym_ci;     /* [n_sym] -> [ndet][nstate] */
    const uint64_t *l2_dets;         /* [n_l2][n_words] */
    /* continuum spin per target determinant (0 alpha, 1 beta) of each
     * symmetry; NULL (or a NULL entry): alpha throughout */
    const int8_t *const *sym_cspin;
} orc_inst;

/* ------------------------------------------------------------------------ */
/* integrals                                                                */
/* ------------------------------------------------------------------------ */

/* Spatial (pq|rs) for global orbital indices (targets first, then continuum),
 * real orbitals, 8-fold symmetry; at most two continuum indices. */
static double X(const orc_ints *I, int p, int q, int r, int s)
{
    const int no = I->n_o, nc = I->n_cont;
    int cp = p >= no, cq = q >= no, cr = r >= no, cs = s >= no;
    int ncnt = cp + cq + cr + cs;
    if (ncnt == 0)
        return I->tttt[(((size_t)p * no + q) * no + r) * no + s];
    if (ncnt == 1) {
        if (cp || cq) { int t0 = p, t1 = q; p = r; q = s; r = t0; s = t1; }
        /* now the continuum index is r or s */
        if (r >= no) { int t = r; r = s; s = t; }
        return I->tttc[(((size_t)p * no + q) * no + r) * nc + (s - no)];
    }
    if (ncnt == 2) {
        if ((cp && cq) || (cr && cs)) {       /* (tt|cc) */
            if (cp) { int t0 = p, t1 = q; p = r; q = s; r = t0; s = t1; }
            if (I->pk_rec) return packed_cc(I, I->ttcc, p, q, r - no, s - no);
            return I->ttcc[(((size_t)p * no + q) * nc + (r - no)) * nc + (s - no)];
        }
        /* one continuum index in each pair: (tc|tc) */
        if (cp) { int t = p; p = q; q = t; }
        if (cr) { int t = r; r = s; s = t; }
        if (I->pk_rec) return packed_cc(I, I->tctc, p, r, q - no, s - no);
        return I->tctc[(((size_t)p * nc + (q - no)) * no + r) * nc + (s - no)];
    }
    return NAN;   /* never needed: at most one continuum electron */
}

static double h1(const orc_ints *I, int p, int q)
{
    size_t n = (size_t)I->n_o + I->n_cont;
    return I->h[(size_t)p * n + q];
}

/* spin-orbital two-electron integral (ab|cd) with spin deltas */
static double Xs(const orc_ints *I, int a, int b, int c, int d)
{
    if ((a & 1) != (b & 1) || (c & 1) != (d & 1)) return 0.0;
    return X(I, a >> 1, b >> 1, c >> 1, d >> 1);
}

static double hs(const orc_ints *I, int a, int b)
{
    if ((a & 1) != (b & 1)) return 0.0;
    return h1(I, a >> 1, b >> 1);
}

/* ------------------------------------------------------------------------ */
/* explicit operator application on ordered occupation lists                */
/* ------------------------------------------------------------------------ */

/* a_k on the ordered product of list L: sign (-1)^(position of k), k removed.
 * Returns 0 if k is empty. */
static int op_annihilate(int *L, int *n, int k)
{
    for (int i = 0; i < *n; ++i) {
        if (L[i] == k) {
            memmove(L + i, L + i + 1, sizeof(int) * (size_t)(*n - i - 1));
            --*n;
            return (i & 1) ? -1 : 1;
        }
    }
    return 0;
}

/* a+_k: k is put in front of the product, then carried to its ordered place
 * by transpositions, each giving a factor -1. Returns 0 if k is occupied. */
static int op_create(int *L, int *n, int k)
{
    int sign = 1;
    for (int i = 0; i < *n; ++i)
        if (L[i] == k) return 0;
    memmove(L + 1, L, sizeof(int) * (size_t)(*n));
    L[0] = k;
    ++*n;
    for (int i = 0; i + 1 < *n && L[i] > L[i + 1]; ++i) {
        int t = L[i]; L[i] = L[i + 1]; L[i + 1] = t;
        sign = -sign;
    }
    return sign;
}

/* Excitation of bra A from ket B (both ascending, n electrons each).
 * holes = B \ A, particles = A \ B, both ascending; degree = their count.
 * For degree <= 2 the sign s with A = s a+_p2 a_h2 a+_p1 a_h1 B is found by
 * applying those operators to B. Returns the degree (3 for anything above 2). */
static int excitation(const int *A, const int *B, int n, int *holes, int *parts, int *sign)
{
    int nh = 0, np = 0;
    for (int i = 0; i < n; ++i) {
        int in = 0;
        for (int j = 0; j < n; ++j) if (A[j] == B[i]) { in = 1; break; }
        if (!in) { if (nh >= 3) return 3; holes[nh++] = B[i]; }
    }
    for (int i = 0; i < n; ++i) {
        int in = 0;
        for (int j = 0; j < n; ++j) if (B[j] == A[i]) { in = 1; break; }
        if (!in) { if (np >= 3) return 3; parts[np++] = A[i]; }
    }
    if (nh != np) return 3;
    if (nh > 2) return 3;
    int L[MAXE], m = n, s = 1;
    memcpy(L, B, sizeof(int) * (size_t)n);
    for (int e = 0; e < nh; ++e) {
        s *= op_annihilate(L, &m, holes[e]);
        s *= op_create(L, &m, parts[e]);
    }
    /* the result must be the ordered list A */
    for (int i = 0; i < n; ++i)
        if (L[i] != A[i]) return -1;
    *sign = s;
    return nh;
}

/* Slater-Condon element <A|H|B> between n-electron determinants (ascending
 * spin-orbital lists). Also returns sum |terms| and the number of terms. */
static double slater_condon(const orc_ints *I, const int *A, const int *B, int n,
                            double *abss, int *nterm)
{
    int holes[3], parts[3], s = 0;
    int deg = excitation(A, B, n, holes, parts, &s);
    double v = 0.0, a = 0.0;
    int cnt = 0;
    if (deg == 0) {
        for (int i = 0; i < n; ++i) {
            double t = hs(I, A[i], A[i]);
            v += t; a += fabs(t); ++cnt;
        }
        /* k = l terms cancel exactly and are left out */
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                if (i == j) continue;
                double t = 0.5 * (Xs(I, A[i], A[i], A[j], A[j]) - Xs(I, A[i], A[j], A[j], A[i]));
                v += t; a += fabs(t); ++cnt;
            }
        v += I->e_core; a += fabs(I->e_core); ++cnt;
    } else if (deg == 1) {
        int p = parts[0], h = holes[0];
        double t = hs(I, p, h);
        v += t; a += fabs(t); ++cnt;
        for (int i = 0; i < n; ++i) {
            int k = B[i];
            if (k == h) continue;
            double t1 = Xs(I, p, h, k, k), t2 = -Xs(I, p, k, k, h);
            v += t1 + t2; a += fabs(t1) + fabs(t2); cnt += 2;
        }
        v *= s;
    } else if (deg == 2) {
        double t1 = Xs(I, parts[0], holes[0], parts[1], holes[1]);
        double t2 = -Xs(I, parts[0], holes[1], parts[1], holes[0]);
        v = s * (t1 + t2); a = fabs(t1) + fabs(t2); cnt = 2;
    }
    if (abss) *abss = a;
    if (nterm) *nterm = cnt;
    return v;
}

/* ------------------------------------------------------------------------ */
/* determinants                                                             */
/* ------------------------------------------------------------------------ */

/* occupation list of a bitstring determinant: bit k of word k/64 set means
 * spin-orbital k is occupied; bits are tested one at a time */
static int det_occ(const uint64_t *d, int n_words, int *occ)
{
    int n = 0;
    for (int k = 0; k < 64 * n_words; ++k)
        if ((d[k / 64] >> (k % 64)) & 1u) occ[n++] = k;
    return n;
}

/* number of spin-orbitals of A missing from B */
static int n_missing(const int *A, int na, const int *B, int nb)
{
    int c = 0;
    for (int i = 0; i < na; ++i) {
        int in = 0;
        for (int j = 0; j < nb; ++j) if (B[j] == A[i]) { in = 1; break; }
        c += !in;
    }
    return c;
}

typedef struct { double s, c, a; int n; } acc_t;   /* Neumaier sum */

static inline void acc_add(acc_t *x, double t, double ab, int n)
{
    double s = x->s + t;
    if (fabs(x->s) >= fabs(t)) x->c += (x->s - s) + t;
    else x->c += (t - s) + x->s;
    x->s = s;
    x->a += ab;
    x->n += n;
}

/* ------------------------------------------------------------------------ */
/* row/column layout of the contracted matrix                               */
/* ------------------------------------------------------------------------ */

static int n_cont_of(const orc_inst *I, int sym)
{
    int a = I->sym_irrep[sym] ^ I->total_irrep;
    return I->cont_start[a + 1] - I->cont_start[a];
}

static int64_t sym_row0(const orc_inst *I, int sym)
{
    int64_t r = 0;
    for (int s = 0; s < sym; ++s) r += (int64_t)I->sym_nstate[s] * n_cont_of(I, s);
    return r;
}

int64_t orc_dim(const orc_inst *I)
{
    return sym_row0(I, I->n_sym) + I->n_l2;
}

/* what a row of the contracted matrix is: continuum (sym, state n, j) or L2 l */
typedef struct { int is_l2, sym, n, j, l; } rowid;

static rowid decode_row(const orc_inst *I, int64_t r)
{
    rowid id = {0, 0, 0, 0, 0};
    for (int s = 0; s < I->n_sym; ++s) {
        int64_t sz = (int64_t)I->sym_nstate[s] * n_cont_of(I, s);
        if (r < sz) {
            int nc = n_cont_of(I, s);
            int a = I->sym_irrep[s] ^ I->total_irrep;
            id.sym = s;
            id.n = (int)(r / nc);
            id.j = I->cont_start[a] + (int)(r % nc);
            return id;
        }
        r -= sz;
    }
    id.is_l2 = 1;
    id.l = (int)r;
    return id;
}

/* continuum spin of target determinant m of a symmetry (0 alpha, 1 beta) */
static int cspin(const orc_inst *I, int sym, int m)
{
    return (I->sym_cspin && I->sym_cspin[sym]) ? I->sym_cspin[sym][m] : 0;
}

/* continuum function |eta_im u_j sigma_m>: target occupation plus the
 * spin-orbital 2(n_o+j) + sigma_m, last */
static int cont_occ(const orc_inst *I, int sym, int m, int j, int *occ)
{
    int n = det_occ(I->sym_dets[sym] + (size_t)m * I->n_words, I->n_words, occ);
    occ[n++] = 2 * (I->ints.n_o + j) + cspin(I, sym, m);
    return n;
}

/* ------------------------------------------------------------------------ */
/* single element by definition (Eqs. 4, 5 and the pure L2 element)         */
/* ------------------------------------------------------------------------ */

static void element(const orc_inst *I, int64_t r, int64_t c, acc_t *out)
{
    rowid R = decode_row(I, r), C = decode_row(I, c);
    int A[MAXE], B[MAXE];
    acc_t acc = {0, 0, 0, 0};
    if (R.is_l2 && C.is_l2) {
        int na = det_occ(I->l2_dets + (size_t)R.l * I->n_words, I->n_words, A);
        int nb = det_occ(I->l2_dets + (size_t)C.l * I->n_words, I->n_words, B);
        if (na == nb) {
            double ab; int nt;
            double v = slater_condon(&I->ints, A, B, na, &ab, &nt);
            acc_add(&acc, v, ab, nt);
        }
        *out = acc;
        return;
    }
    if (R.is_l2) { rowid t = R; R = C; C = t; }   /* continuum row first */
    const double *cr = I->sym_ci[R.sym];
    int Sr = I->sym_nstate[R.sym];
    if (C.is_l2) {
        /* Eq. 5: sum over target determinants of the row's symmetry */
        int nb = det_occ(I->l2_dets + (size_t)C.l * I->n_words, I->n_words, B);
        for (int m = 0; m < I->sym_ndet[R.sym]; ++m) {
            int na = cont_occ(I, R.sym, m, R.j, A);
            if (na != nb) continue;
            if (n_missing(A, na - 1, B, nb) > 1) continue;   /* > 2 differences */
            double ab; int nt;
            double v = slater_condon(&I->ints, A, B, na, &ab, &nt);
            double w = cr[(size_t)m * Sr + R.n];
            acc_add(&acc, w * v, fabs(w) * ab, nt);
        }
        *out = acc;
        return;
    }
    /* Eq. 4: double sum over target determinants */
    const double *cc = I->sym_ci[C.sym];
    int Sc = I->sym_nstate[C.sym];
    for (int m = 0; m < I->sym_ndet[R.sym]; ++m) {
        int na = cont_occ(I, R.sym, m, R.j, A);
        for (int m2 = 0; m2 < I->sym_ndet[C.sym]; ++m2) {
            int nb = cont_occ(I, C.sym, m2, C.j, B);
            if (na != nb) continue;
            if (n_missing(A, na - 1, B, nb - 1) > 2) continue;
            double ab; int nt;
            double v = slater_condon(&I->ints, A, B, na, &ab, &nt);
            double w = cr[(size_t)m * Sr + R.n] * cc[(size_t)m2 * Sc + C.n];
            acc_add(&acc, w * v, fabs(w) * ab, nt);
        }
    }
    *out = acc;
}

/* Sampled elements: val/abs/cnt may be NULL except val. Same sums as
 * element() above (same order of m, m'), with the occupation lists and the
 * target-pair connectivity of each symmetry pair computed once per call. */
typedef struct { int64_t *off; int32_t *m2; } conn_t;

void orc_elements(const orc_inst *I, int64_t n, const int64_t *rows, const int64_t *cols,
                  double *val, double *abss, int32_t *cnt)
{
    const int W = I->n_words, N = I->n_elec, ns = I->n_sym;
    /* occupation lists of the target determinants of every symmetry */
    int **occ = (int **)malloc(sizeof(int *) * (size_t)(ns > 0 ? ns : 1));
    for (int s = 0; s < ns; ++s) {
        occ[s] = (int *)malloc(sizeof(int) * (size_t)I->sym_ndet[s] * (N > 0 ? N : 1));
        for (int m = 0; m < I->sym_ndet[s]; ++m) det_occ(I->sym_dets[s] + (size_t)m * W, W, occ[s] + (size_t)m * N);
    }
    /* which continuum symmetry pairs are needed */
    conn_t *cn = (conn_t *)calloc((size_t)(ns * ns > 0 ? ns * ns : 1), sizeof(conn_t));
    for (int64_t e = 0; e < n; ++e) {
        rowid R = decode_row(I, rows[e]), C = decode_row(I, cols[e]);
        if (!R.is_l2 && !C.is_l2) cn[R.sym * ns + C.sym].off = (int64_t *)1;
    }
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            conn_t *c = &cn[a * ns + b];
            if (!c->off) continue;
            const int Ma = I->sym_ndet[a], Mb = I->sym_ndet[b];
            c->off = (int64_t *)calloc((size_t)Ma + 1, sizeof(int64_t));
            int64_t *cntr = (int64_t *)calloc((size_t)Ma, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
            for (int m = 0; m < Ma; ++m) {
                int64_t k = 0;
                for (int m2 = 0; m2 < Mb; ++m2)
                    k += n_missing(occ[a] + (size_t)m * N, N, occ[b] + (size_t)m2 * N, N) <= 2;
                cntr[m] = k;
            }
            for (int m = 0; m < Ma; ++m) c->off[m + 1] = c->off[m] + cntr[m];
            c->m2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c->off[Ma] > 0 ? c->off[Ma] : 1));
#pragma omp parallel for schedule(dynamic, 16)
            for (int m = 0; m < Ma; ++m) {
                int64_t k = c->off[m];
                for (int m2 = 0; m2 < Mb; ++m2)
                    if (n_missing(occ[a] + (size_t)m * N, N, occ[b] + (size_t)m2 * N, N) <= 2) c->m2[k++] = m2;
            }
            free(cntr);
        }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < n; ++e) {
        rowid R = decode_row(I, rows[e]), C = decode_row(I, cols[e]);
        acc_t acc = {0, 0, 0, 0};
        int A[MAXE], B[MAXE];
        if (R.is_l2 && C.is_l2) {
            element(I, rows[e], cols[e], &acc);
        } else {
            if (R.is_l2) { rowid t = R; R = C; C = t; }
            const double *cr = I->sym_ci[R.sym];
            const int Sr = I->sym_nstate[R.sym];
            const int top = 2 * (I->ints.n_o + R.j);
            if (C.is_l2) {
                int nb = det_occ(I->l2_dets + (size_t)C.l * W, W, B);
                for (int m = 0; m < I->sym_ndet[R.sym]; ++m) {
                    memcpy(A, occ[R.sym] + (size_t)m * N, sizeof(int) * (size_t)N);
                    A[N] = top + cspin(I, R.sym, m);
                    if (N + 1 != nb) continue;
                    if (n_missing(A, N, B, nb) > 1) continue;
                    double ab; int nt;
                    double v = slater_condon(&I->ints, A, B, N + 1, &ab, &nt);
                    double w = cr[(size_t)m * Sr + R.n];
                    acc_add(&acc, w * v, fabs(w) * ab, nt);
                }
            } else {
                const conn_t *c = &cn[R.sym * ns + C.sym];
                const double *cc = I->sym_ci[C.sym];
                const int Sc = I->sym_nstate[C.sym];
                const int topc = 2 * (I->ints.n_o + C.j);
                for (int m = 0; m < I->sym_ndet[R.sym]; ++m) {
                    memcpy(A, occ[R.sym] + (size_t)m * N, sizeof(int) * (size_t)N);
                    A[N] = top + cspin(I, R.sym, m);
                    for (int64_t k = c->off[m]; k < c->off[m + 1]; ++k) {
                        const int m2 = c->m2[k];
                        memcpy(B, occ[C.sym] + (size_t)m2 * N, sizeof(int) * (size_t)N);
                        B[N] = topc + cspin(I, C.sym, m2);
                        double ab; int nt;
                        double v = slater_condon(&I->ints, A, B, N + 1, &ab, &nt);
                        double w = cr[(size_t)m * Sr + R.n] * cc[(size_t)m2 * Sc + C.n];
                        acc_add(&acc, w * v, fabs(w) * ab, nt);
                    }
                }
            }
        }
        val[e] = acc.s + acc.c;
        if (abss) abss[e] = acc.a;
        if (cnt) cnt[e] = acc.n;
    }
    for (int i = 0; i < ns * ns; ++i) {
        if (cn[i].off) { free(cn[i].off); free(cn[i].m2); }
    }
    free(cn);
    for (int s = 0; s < ns; ++s) free(occ[s]);
    free(occ);
}

/* ------------------------------------------------------------------------ */
/* full matrix                                                              */
/* ------------------------------------------------------------------------ */

/* Full rows of the dense D x D contracted matrix (both triangles computed
 * independently) for the listed rows; H is [nrows][D] in list order. The
 * continuum blocks are built per symmetry pair by looping the target pairs
 * (m, m') outside and j, j' inside, so each uncontracted element is formed
 * once and folded into all (n, n') at once (Eq. 4 as written). */
void orc_build_rows(const orc_inst *I, int64_t nrows, const int64_t *rows, double *H, double *Habs,
                    int32_t *Hcnt)
{
    const int64_t D = orc_dim(I);
    const int64_t Dc = sym_row0(I, I->n_sym);
    const int W = I->n_words;
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)D);
    for (int64_t r = 0; r < D; ++r) slot[r] = -1;
    for (int64_t i = 0; i < nrows; ++i) slot[rows[i]] = i;
    acc_t *acc = (acc_t *)calloc((size_t)(nrows > 0 ? nrows : 1) * (size_t)D, sizeof(acc_t));

    /* continuum x continuum */
    for (int si = 0; si < I->n_sym; ++si) {
        int ai = I->sym_irrep[si] ^ I->total_irrep, nci = n_cont_of(I, si), Si = I->sym_nstate[si];
        int64_t ri0 = sym_row0(I, si);
        int j0i = I->cont_start[ai];
        int Mi = I->sym_ndet[si];
        /* continuum orbitals jj of this symmetry with at least one listed row */
        int *jneed = (int *)malloc(sizeof(int) * (size_t)(nci > 0 ? nci : 1));
        int nj = 0;
        for (int jj = 0; jj < nci; ++jj) {
            int any = 0;
            for (int n = 0; n < Si; ++n) any |= slot[ri0 + (int64_t)n * nci + jj] >= 0;
            if (any) jneed[nj++] = jj;
        }
        if (nj == 0) { free(jneed); continue; }
        /* target pairs connected by at most a double substitution, per ket symmetry */
        int **pm = (int **)malloc(sizeof(int *) * (size_t)I->n_sym);
        int64_t *np = (int64_t *)malloc(sizeof(int64_t) * (size_t)I->n_sym);
        for (int sk = 0; sk < I->n_sym; ++sk) {
            int Mk = I->sym_ndet[sk];
            pm[sk] = (int *)malloc(sizeof(int) * 2 * ((size_t)Mi * Mk + 1));
            np[sk] = 0;
            for (int m = 0; m < Mi; ++m) {
                int A[MAXE], B[MAXE];
                int na = det_occ(I->sym_dets[si] + (size_t)m * W, W, A);
                for (int m2 = 0; m2 < Mk; ++m2) {
                    int nb = det_occ(I->sym_dets[sk] + (size_t)m2 * W, W, B);
                    if (na == nb && n_missing(A, na, B, nb) <= 2) {
                        pm[sk][2 * np[sk]] = m; pm[sk][2 * np[sk] + 1] = m2; ++np[sk];
                    }
                }
            }
        }
        const double *ci = I->sym_ci[si];
        const int ntask = nj * I->n_sym;
#pragma omp parallel for schedule(dynamic, 1)
        for (int task = 0; task < ntask; ++task) {
            const int jj = jneed[task / I->n_sym], sk = task % I->n_sym;
            int ak = I->sym_irrep[sk] ^ I->total_irrep, nck = n_cont_of(I, sk), Sk = I->sym_nstate[sk];
            int64_t rk0 = sym_row0(I, sk);
            int j0k = I->cont_start[ak];
            const double *ck = I->sym_ci[sk];
            int A[MAXE], B[MAXE];
            for (int64_t e = 0; e < np[sk]; ++e) {
                int m = pm[sk][2 * e], m2 = pm[sk][2 * e + 1];
                int na = cont_occ(I, si, m, j0i + jj, A);
                for (int jk = 0; jk < nck; ++jk) {
                    cont_occ(I, sk, m2, j0k + jk, B);
                    double ab; int nt;
                    double v = slater_condon(&I->ints, A, B, na, &ab, &nt);
                    if (nt == 0) continue;
                    for (int n = 0; n < Si; ++n) {
                        int64_t sl = slot[ri0 + (int64_t)n * nci + jj];
                        if (sl < 0) continue;
                        double wn = ci[(size_t)m * Si + n];
                        acc_t *row = acc + (size_t)sl * D;
                        for (int n2 = 0; n2 < Sk; ++n2) {
                            int64_t c = rk0 + (int64_t)n2 * nck + jk;
                            double w = wn * ck[(size_t)m2 * Sk + n2];
                            acc_add(row + c, w * v, fabs(w) * ab, nt);
                        }
                    }
                }
            }
        }
        for (int sk = 0; sk < I->n_sym; ++sk) free(pm[sk]);
        free(pm); free(np); free(jneed);
    }

    /* continuum x L2 (Eq. 5) and L2 x continuum (its transpose, computed again) */
#pragma omp parallel for schedule(dynamic, 4)
    for (int l = 0; l < I->n_l2; ++l) {
        int A[MAXE], B[MAXE];
        int nb = det_occ(I->l2_dets + (size_t)l * W, W, B);
        int64_t rl = Dc + l;
        int64_t sll = slot[rl];
        for (int si = 0; si < I->n_sym; ++si) {
            int ai = I->sym_irrep[si] ^ I->total_irrep, nci = n_cont_of(I, si), Si = I->sym_nstate[si];
            int64_t ri0 = sym_row0(I, si);
            const double *ci = I->sym_ci[si];
            for (int m = 0; m < I->sym_ndet[si]; ++m) {
                int na0 = det_occ(I->sym_dets[si] + (size_t)m * W, W, A);
                if (na0 + 1 != nb || n_missing(A, na0, B, nb) > 1) continue;
                for (int jj = 0; jj < nci; ++jj) {
                    int need = sll >= 0;
                    for (int n = 0; n < Si && !need; ++n) need = slot[ri0 + (int64_t)n * nci + jj] >= 0;
                    if (!need) continue;
                    int na = cont_occ(I, si, m, I->cont_start[ai] + jj, A);
                    double ab1, ab2; int nt1, nt2;
                    double v1 = slater_condon(&I->ints, A, B, na, &ab1, &nt1);   /* <cont|H|l> */
                    double v2 = slater_condon(&I->ints, B, A, na, &ab2, &nt2);   /* <l|H|cont> */
                    for (int n = 0; n < Si; ++n) {
                        int64_t r = ri0 + (int64_t)n * nci + jj;
                        double w = ci[(size_t)m * Si + n];
                        if (slot[r] >= 0)
                            acc_add(acc + (size_t)slot[r] * D + rl, w * v1, fabs(w) * ab1, nt1);
                        if (sll >= 0)
                            acc_add(acc + (size_t)sll * D + r, w * v2, fabs(w) * ab2, nt2);
                    }
                }
            }
        }
    }

    /* L2 x L2 (classes 2 and 8): no contraction */
#pragma omp parallel for schedule(dynamic, 4)
    for (int l = 0; l < I->n_l2; ++l) {
        int64_t sll = slot[Dc + l];
        if (sll < 0) continue;
        int A[MAXE], B[MAXE];
        int na = det_occ(I->l2_dets + (size_t)l * W, W, A);
        for (int l2 = 0; l2 < I->n_l2; ++l2) {
            int nb = det_occ(I->l2_dets + (size_t)l2 * W, W, B);
            if (na != nb || n_missing(A, na, B, nb) > 2) continue;
            double ab; int nt;
            double v = slater_condon(&I->ints, A, B, na, &ab, &nt);
            acc_add(acc + (size_t)sll * D + Dc + l2, v, ab, nt);
        }
    }

    for (int64_t i = 0; i < nrows * D; ++i) {
        H[i] = acc[i].s + acc[i].c;
        if (Habs) Habs[i] = acc[i].a;
        if (Hcnt) Hcnt[i] = acc[i].n;
    }
    free(acc);
    free(slot);
}

/* rows [r0, r1) */
void orc_build(const orc_inst *I, int64_t r0, int64_t r1, double *H, double *Habs, int32_t *Hcnt)
{
    const int64_t D = orc_dim(I);
    if (r1 > D) r1 = D;
    int64_t n = r1 > r0 ? r1 - r0 : 0;
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) rows[i] = r0 + i;
    orc_build_rows(I, n, rows, H, Habs, Hcnt);
    free(rows);
}

/* ------------------------------------------------------------------------ */
/* determinant-pair artefacts for the bit-exact excitation checks           */
/* ------------------------------------------------------------------------ */

#define NOLAB 0xFFFFull

/* packed label: four 16-bit spin-orbital fields (p1, h1, p2, h2), unused 0xFFFF */
static uint64_t pack4(int f0, int f1, int f2, int f3)
{
    return ((uint64_t)(uint16_t)f0) | ((uint64_t)(uint16_t)f1 << 16) |
           ((uint64_t)(uint16_t)f2 << 32) | ((uint64_t)(uint16_t)f3 << 48);
}

/* Excitation analysis of bra dets a[] against ket dets b[] (same electron
 * count): for every pair (x, y) with degree <= 2, in row-major order (only
 * y <= x when `lower`), emit x, y, degree, packed label and sign.
 * Returns the number of connected pairs (writes at most cap). */
int64_t orc_pairs(const uint64_t *a, int na_det, const uint64_t *b, int nb_det, int n_words,
                  int lower, int64_t cap, int32_t *ox, int32_t *oy, int8_t *odeg,
                  uint64_t *olab, int8_t *ophase)
{
    int64_t cnt = 0;
    for (int x = 0; x < na_det; ++x) {
        int A[MAXE], B[MAXE];
        int na = det_occ(a + (size_t)x * n_words, n_words, A);
        int ylim = lower ? x + 1 : nb_det;
        for (int y = 0; y < ylim; ++y) {
            int nb = det_occ(b + (size_t)y * n_words, n_words, B);
            if (na != nb) continue;
            int holes[3], parts[3], s = 0;
            int deg = excitation(A, B, na, holes, parts, &s);
            if (deg < 0 || deg > 2) continue;
            if (cnt < cap) {
                ox[cnt] = x; oy[cnt] = y; odeg[cnt] = (int8_t)deg;
                ophase[cnt] = (int8_t)(deg == 0 ? 1 : s);
                olab[cnt] = pack4(deg >= 1 ? parts[0] : NOLAB, deg >= 1 ? holes[0] : NOLAB,
                                  deg >= 2 ? parts[1] : NOLAB, deg >= 2 ? holes[1] : NOLAB);
            }
            ++cnt;
        }
    }
    return cnt;
}

/* Continuum-L2 artefacts: bra = target det D_y with a continuum electron
 * above every target spin-orbital, ket = L2 det chi_x. For every pair with
 * at most a double substitution emit x, y, degree of the (N+1)-electron pair,
 * the packed target label (target particle, hole 1, hole 2, 0xFFFF) and the
 * sign of <D_y u|H|chi_x>. n_spin_orb is 2*n_o (the continuum slot index). */
int64_t orc_pairs_l2tgt(const uint64_t *l2, int n_l2, const uint64_t *tg, int n_tg, int n_words,
                        int n_spin_orb, int64_t cap, int32_t *ox, int32_t *oy, int8_t *odeg,
                        uint64_t *olab, int8_t *ophase)
{
    int64_t cnt = 0;
    for (int x = 0; x < n_l2; ++x) {
        int A[MAXE], B[MAXE];
        int nb = det_occ(l2 + (size_t)x * n_words, n_words, B);
        for (int y = 0; y < n_tg; ++y) {
            int na = det_occ(tg + (size_t)y * n_words, n_words, A);
            if (na + 1 != nb) continue;
            A[na++] = n_spin_orb;     /* continuum electron, highest index */
            int holes[3], parts[3], s = 0;
            int deg = excitation(A, B, na, holes, parts, &s);
            if (deg < 0 || deg > 2) continue;
            if (cnt < cap) {
                int pt = NOLAB;
                for (int e = 0; e < deg; ++e) if (parts[e] != n_spin_orb) pt = parts[e];
                ox[cnt] = x; oy[cnt] = y; odeg[cnt] = (int8_t)deg; ophase[cnt] = (int8_t)s;
                olab[cnt] = pack4(pt, holes[0], deg >= 2 ? holes[1] : NOLAB, NOLAB);
            }
            ++cnt;
        }
    }
    return cnt;
}

/* Slater-Condon elements for explicit pairs of occupation lists (ascending,
 * n electrons each), over the global spin-orbital index space. */
void orc_sc_lists(const orc_ints *I, int n, int64_t npair, const int32_t *A, const int32_t *B,
                  double *out, double *abss)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < npair; ++e) {
        double ab; int nt;
        out[e] = slater_condon(I, A + (size_t)e * n, B + (size_t)e * n, n, &ab, &nt);
        if (abss) abss[e] = ab;
    }
}

/* the excitation of a single pair, for the unit checks */
int orc_excitation(const int32_t *A, const int32_t *B, int n, int32_t *holes, int32_t *parts,
                   int32_t *sign)
{
    int h[3], p[3], s = 0;
    int deg = excitation(A, B, n, h, p, &s);
    for (int i = 0; i < 3 && i < (deg > 0 ? deg : 0) && deg <= 2; ++i) { holes[i] = h[i]; parts[i] = p[i]; }
    *sign = s;
    return deg;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads the oracle's parallel loops use from now on (n >= 1); harness
 * control for timing, no effect on any value. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
