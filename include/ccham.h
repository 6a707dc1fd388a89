/*
 * ccham: CI-contracted close-coupling scattering Hamiltonian on one MI355X.
 *
 * The library builds the contracted Hamiltonian of the close-coupling
 * expansion (Al-Refaie & Tennyson, MPI-SCATCI, Sec. 2, Eqs. 1-5) from
 * integrals, orbital and determinant lists and target CI vectors, and finds
 * its lowest eigenpairs with a block Davidson solver (the paper's Sec. 3.2
 * names Davidson among its diagonalisers).
 *
 * Basis and conventions
 *   - Orbitals: n_o target orbitals (global indices 0..n_o-1), then the
 *     continuum orbitals grouped by irrep (global n_o + j, j = 0..n_cont-1).
 *     Irreps form an abelian group whose product is XOR.
 *   - Spin-orbital k = 2*orbital + spin (alpha = 0). A determinant is a
 *     bitstring over the 2*n_o target spin-orbitals, bit k%64 of word k/64,
 *     read as the ascending product a+_k1 a+_k2 ... |0>.
 *   - A continuum function |eta_im u_j> (Eq. 1, first sum) appends the alpha
 *     continuum spin-orbital 2*(n_o + j) after all target electrons; j runs
 *     over the continuum orbitals whose irrep is irrep(i) XOR total_irrep.
 *   - Rows/columns of the contracted matrix: target symmetries in the order
 *     they were added, within each (state n, continuum j) with j fastest, then
 *     the L2 functions chi_l in input order (Eq. 1, second sum).
 *   - The matrix is real symmetric (Sec. 2.2: only the lower triangle is
 *     evaluated); the library stores it densely with both triangles.
 *
 * Error behaviour: every call returns a cch_status; no exception or abort
 * crosses the interface. cch_last_error() describes the last failure of a
 * context. Inputs are copied during the call and stay owned by the caller.
 * A pointer argument is a host pointer unless `flags & CCH_MEM_DEVICE`, in
 * which case it is a device pointer on the context's device. Device work is
 * ordered on the context's HIP stream; cch_sync() waits for it.
 * One context must not be used from two threads at once.
 */
#ifndef CCHAM_H
#define CCHAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cch_status;

#define CCH_OK 0
#define CCH_E_INVALID_ARG (-1)   /* null pointer, negative size, bad option */
#define CCH_E_STATE (-2)         /* call made in the wrong order */
#define CCH_E_INPUT (-3)         /* malformed determinant list or CI vectors */
#define CCH_E_LIMIT (-4)         /* orbital index above the 16-bit label range */
#define CCH_E_OOM (-5)           /* device allocation failed or over budget */
#define CCH_E_HIP (-6)           /* a HIP runtime call failed */
#define CCH_E_NOT_CONVERGED (-7) /* Davidson hit max_iter; best pairs returned */

#define CCH_MEM_HOST 0
#define CCH_MEM_DEVICE 1
#define CCH_DAV_RESIDUALS 2   /* cch_davidson: evecs holds 2k rows, residuals after the vectors */
#define CCH_DAV_SPARSE_L2 4   /* cch_davidson: the L2 block (classes 2 and 8) as CSR in the mat-vec */

/* cch_dav_opts.restart. A restart rebuilds a full basis from Ritz vectors of
 * the last Rayleigh-Ritz step (Sec. 3.2's Davidson):
 *   CCH_RESTART_THICK  the lowest 2k Ritz vectors;
 *   CCH_RESTART_PREV   the lowest kr = min(4k, mmax - 2k) Ritz vectors plus, for
 *                      each wanted pair, the part of its Ritz vector of the
 *                      iteration before that lies outside the kept ones
 *                      (orthonormalised; parts below 1e-8 are dropped), so the
 *                      direction in which each pair was moving survives the
 *                      restart; the thick restart when kr < 2k;
 *   CCH_RESTART_AUTO   (0) CCH_RESTART_PREV from a basis of 96 vectors on (the
 *                      default from D = 20000), CCH_RESTART_THICK below. */
#define CCH_RESTART_AUTO 0
#define CCH_RESTART_THICK 1
#define CCH_RESTART_PREV 2
#define CCH_LOWER 8           /* cch_get_matrix: only the lower triangle (Sec. 2.2) is required */

/* cch_plan_opts.flags */
#define CCH_PLAN_SPARSE_L2 1  /* classes 2 and 8 built and stored as CSR, never dense (see cch_plan) */

/* precision of the CI-contraction / expansion GEMMs (cch_plan_opts) */
#define CCH_PREC_FP64 0
#define CCH_PREC_FP32 1
#define CCH_PREC_SPLIT_BF16 2

/* Davidson preconditioners */
#define CCH_PRECOND_JACOBI 0
#define CCH_PRECOND_MLP 1

/* cch_subspace_eig methods */
#define CCH_EIG_AUTO 0
#define CCH_EIG_JACOBI 1

/* which determinant-pair list cch_get_labels returns */
#define CCH_PAIRS_TARGET 0   /* target x target, one symmetry pair */
#define CCH_PAIRS_L2 1       /* L2 x L2, lower triangle */
#define CCH_PAIRS_L2_TARGET 2 /* L2 x target dets of one symmetry */

typedef struct cch_ctx cch_ctx;

typedef struct {
    int32_t precision;      /* CCH_PREC_* for the expansion GEMMs */
    int32_t split_slices;   /* slices per operand for CCH_PREC_SPLIT_BF16 (2..8) */
    int32_t autotune;       /* 1: time candidate tile shapes on the device */
    int32_t flags;          /* CCH_PLAN_* (0: the whole matrix stored dense) */
    int64_t max_device_bytes; /* 0: no limit. Else the plan's device memory stays
                                 within it: in FP64 mode the integral rows of the
                                 expansion product are laid out and multiplied in
                                 passes over the continuum orbitals, as many per
                                 pass as fit (same result, bit for bit; the
                                 relayout time then counts in phase 3);
                                 CCH_E_OOM when the rest alone, or one orbital
                                 per pass, does not fit, or in FP32 / split-BF16
                                 mode when the whole plan does not */
} cch_plan_opts;

typedef struct {
    int32_t k;              /* eigenpairs wanted (lowest) */
    int32_t max_iter;       /* Davidson iterations */
    int32_t max_subspace;   /* basis size before a thick restart (0: max(8k, 64), or 96
                               from D = 20000 on; at most 96 and D) */
    int32_t precond;        /* CCH_PRECOND_* */
    double tol;             /* converged when ||H x - theta x||_2 <= tol, ||x|| = 1 */
    int32_t block;          /* Ritz pairs given a correction each iteration, k..16
                               (0: k); pairs k..block-1 are guards: corrected
                               while any wanted pair is unconverged, never
                               tested for convergence */
    int32_t restart;        /* CCH_RESTART_*: what a restart keeps when the
                               basis is full */
} cch_dav_opts;

typedef struct {
    int32_t iterations;
    int32_t matvecs;        /* columns multiplied by H */
    int32_t converged;      /* number of converged pairs */
    int32_t fallbacks;      /* MLP corrections replaced by the Jacobi step */
    double max_residual;
    double seconds;         /* wall time of the solve */
    double matvec_ms;       /* device time of the H V launches (HIP events) */
    int32_t matvec_launches;
    int32_t rr_fallbacks;   /* Rayleigh-Ritz solves rerun by cyclic Jacobi */
    double rr_ms;           /* device time of the Rayleigh-Ritz launches (HIP events) */
    double rr_flops;        /* sum over those solves of (10/3) m^3 */
    int32_t rr_calls;       /* Rayleigh-Ritz solves */
    int32_t dropped;        /* correction directions dropped by the rank test
                               (nearly inside the basis); each iteration with a
                               drop repeats its Rayleigh-Ritz step */
    int32_t restarts;       /* restarts of the basis */
    int32_t prev_kept;      /* directions from previous Ritz vectors kept over
                               all restarts (CCH_RESTART_PREV) */
} cch_dav_info;

/* Library version string (static storage). */
const char *cch_version(void);

/* Measured FP64 issue rates of HIP device `device` on `hip_stream` (NULL = the
 * null stream), in TFLOP/s: rates[0] the 16x16x4 FP64 MFMA, rates[1] the
 * four-block 4x4x4 FP64 MFMA, rates[2] the FP64 vector FMA, each from
 * register-only loops with independent accumulator chains over 2048
 * workgroups (best of two timed launches after a warm-up). A calibration for
 * the roofline figures of the FP64 kernels (the published FP64 peak of the
 * MI355X is 78.6 TFLOP/s for both units); no context needed. rates[3] host
 * array. CCH_E_INVALID_ARG for NULL rates, CCH_E_HIP / CCH_E_OOM from the
 * runtime. Synchronous. */
cch_status cch_probe_fp64(int32_t device, void *hip_stream, double *rates);

/* Create a context on HIP device `device`, ordering work on `hip_stream`
 * (a hipStream_t; NULL = the null stream). *out receives the context. */
cch_status cch_create(cch_ctx **out, int32_t device, void *hip_stream);
/* Free every device buffer the context owns. NULL is accepted. */
cch_status cch_destroy(cch_ctx *ctx);
/* Message of the last failed call on ctx (or of a failed create if NULL). */
const char *cch_last_error(const cch_ctx *ctx);
/* Wait for all work queued on the context's stream. */
cch_status cch_sync(cch_ctx *ctx);

/* Orbitals (Eq. 1: target orbitals, continuum orbitals u_ij per symmetry).
 * tgt_irrep[n_o]: irrep of each target orbital (< n_irrep); n_c_per_irrep
 * [n_irrep]: continuum orbitals of each irrep, stored irrep-major after the
 * target orbitals; total_irrep: irrep of the (N+1)-electron functions.
 * n_o + sum(n_c) must fit the 16-bit orbital fields of the packed labels
 * (Sec. 2.1): CCH_E_LIMIT otherwise. Host pointers. */
cch_status cch_set_orbitals(cch_ctx *ctx, int32_t n_o, const uint8_t *tgt_irrep,
                            int32_t n_irrep, const int32_t *n_c_per_irrep,
                            int32_t total_irrep);

/* Integrals (Sec. 2.1: the integral function X maps labels to precomputed
 * one- and two-electron arrays), real orbitals, chemists' notation, row-major,
 * symmetry zeros explicit. Only classes with at most two continuum indices
 * exist for functions with at most one continuum electron:
 *   h    [n_orb][n_orb]            h_pq            (n_orb = n_o + n_cont)
 *   tttt [n_o][n_o][n_o][n_o]      (pq|rs)
 *   tttc [n_o][n_o][n_o][n_cont]   (pq|r j)
 *   ttcc [n_o][n_o][n_cont][n_cont] (pq|j j')
 *   tctc [n_o][n_cont][n_o][n_cont] (p j|q j')
 * e_core is added to every diagonal element. Requires cch_set_orbitals. */
cch_status cch_set_integrals(cch_ctx *ctx, const double *h, const double *tttt,
                             const double *tttc, const double *ttcc, const double *tctc,
                             double e_core, int32_t flags);

/* The same integrals with (tt|cc) and (tc|tc) in a symmetry-packed layout
 * (Sec. 3.3: the integrals dominate memory; values that symmetry forbids are
 * not stored). For the target pair (P, Q), with x = irrep(P) XOR irrep(Q),
 * one record holds a block for each continuum irrep ca in increasing order:
 * the n_c[ca] x n_c[ca XOR x] values (P Q | j j') (ttcc) or (P j | Q j')
 * (tctc), row-major, j of irrep ca and j' of irrep ca XOR x (indices local to
 * their irreps). Records follow in pair order P * n_o + Q, so each array
 * holds sum over (P, Q) of sum over ca of n_c[ca] n_c[ca XOR x] values (for
 * four irreps of equal size a quarter of the dense array). h, tttt and tttc,
 * the rest of the arguments and the errors are those of cch_set_integrals;
 * the matrix built is the same as from the dense arrays, bit for bit. */
cch_status cch_set_integrals_packed(cch_ctx *ctx, const double *h, const double *tttt,
                                    const double *tttc, const double *ttcc, const double *tctc,
                                    double e_core, int32_t flags);

/* One target symmetry (Eq. 2): n_det determinants of n_words words each
 * (n_words = ceil(2 n_o / 64)), every one with N electrons, N/2 of each
 * spin, irrep `irrep`, all distinct; CI vectors ci[n_det][n_states]
 * (row-major, c_imn). N is fixed by the first symmetry. *sym_id receives the
 * symmetry's index. CCH_E_INPUT for a malformed list. */
cch_status cch_add_target_symmetry(cch_ctx *ctx, int32_t irrep, int32_t n_det,
                                   int32_t n_words, const uint64_t *dets,
                                   int32_t n_states, const double *ci, int32_t flags,
                                   int32_t *sym_id);

/* One target symmetry whose continuum functions carry a continuum electron of
 * either spin (Eq. 1 with spin-coupled channels; the CSF-driven build of
 * Sec. 2 couples e.g. triplet target states with the continuum electron to
 * doublets: sqrt(2/3) |T, 1> u_beta - sqrt(1/3) |T, 0> u_alpha). As
 * cch_add_target_symmetry, with cont_spin[n_det] the continuum spin of each
 * determinant's function (0 alpha, 1 beta): a continuum function is
 * sum_m c_imn |D_m u_j sigma_m>. The total M_S stays +1/2, so a determinant
 * with a beta continuum electron has N/2 + 1 alpha and N/2 - 1 beta
 * electrons, one with an alpha continuum electron N/2 of each. Pairs of
 * determinants with different continuum spins couple through the exchange
 * integrals (P j'|j Q) of spin-flip single substitutions; the L2 functions
 * (M_S = +1/2) are unchanged. Host pointers unless flags holds
 * CCH_MEM_DEVICE. CCH_E_INPUT for a spin other than 0 or 1 or an alpha count
 * that does not match the spin; CCH_E_INVALID_ARG for cont_spin == NULL. */
cch_status cch_add_target_symmetry_spin(cch_ctx *ctx, int32_t irrep, int32_t n_det, int32_t n_words,
                                        const uint64_t *dets, const int8_t *cont_spin, int32_t n_states,
                                        const double *ci, int32_t flags, int32_t *sym_id);

/* One target symmetry whose CSFs (Eq. 2) are fixed combinations of
 * determinants: CSF m is sum_t coef[t] |dets[t]> over the terms
 * t in [csf_start[m], csf_start[m+1]) (csf_start[0] = 0, every CSF at least
 * one term; a determinant may appear in several CSFs), each determinant an
 * ascending product of spin-orbitals as in cch_add_target_symmetry; CI vectors
 * ci[n_csf][n_states] over the CSFs. The states are rewritten over the
 * distinct determinants (in order of first appearance, coefficients summed in
 * term order) and added as by cch_add_target_symmetry, whose checks and limits
 * then apply (n_states <= distinct determinants). The continuum electron stays
 * alpha, so the (N+1)-electron functions are spin-adapted for singlet targets.
 * CCH_E_INPUT for a malformed list or a non-finite coefficient. */
cch_status cch_add_target_symmetry_csf(cch_ctx *ctx, int32_t irrep, int32_t n_csf, const int32_t *csf_start,
                                       int32_t n_words, const uint64_t *dets, const double *coef,
                                       int32_t n_states, const double *ci, int32_t flags, int32_t *sym_id);

/* The L2 functions (Eq. 1, second sum): n_l2 determinants with N+1 electrons
 * in target orbitals, N/2+1 alpha and N/2 beta, irrep total_irrep. */
cch_status cch_set_l2(cch_ctx *ctx, int32_t n_l2, int32_t n_words, const uint64_t *dets,
                      int32_t flags);

/* The L2 functions as configuration state functions (Eq. 1's second sum;
 * Sec. 2 builds the matrix from CSF lists): CSF l is
 * sum_{t = csf_start[l]}^{csf_start[l+1]-1} coef[t] |dets[t]>, each determinant
 * with N+1 electrons in target orbitals (N/2+1 alpha, N/2 beta, irrep
 * total_irrep), n_words 64-bit words each; a determinant may appear in several
 * CSFs. Replaces any earlier cch_set_l2 / cch_set_l2_csf. The matrix then has
 * n_csf L2 rows and columns: the build forms the blocks over the distinct
 * determinants (in order of first appearance) and contracts them with the
 * coefficients, which needs device memory for both matrices; classes 2, 4
 * and 8 then hold <chi_l|H|chi_l'> and the contracted class-4 rows.
 * cch_get_labels still lists determinant pairs. Not with CCH_PLAN_SPARSE_L2
 * (cch_plan fails with CCH_E_STATE) nor in a batch. Host pointers unless
 * flags holds CCH_MEM_DEVICE. CCH_E_INPUT for csf_start[0] != 0, a CSF without
 * determinants, a non-finite coefficient or a determinant that fails the
 * checks of cch_set_l2. Before cch_plan. */
cch_status cch_set_l2_csf(cch_ctx *ctx, int32_t n_csf, const int32_t *csf_start, int32_t n_words,
                          const uint64_t *dets, const double *coef, int32_t flags);

/* Target energies on the diagonal (Sec. 3.1, the option kept for classes 1,
 * 3, 5, 6 and 7): E[n] holds the n = sum of n_states energies of all target
 * states, symmetry by symmetry in the order they were added, state by state
 * within a symmetry (total energies, E_core included). With them, the terms of
 * a continuum element made of target orbitals only -- which add up to
 * delta_jj' (C_a^T H_T C_b)_nn', E_core included -- are left out, and
 * delta_ab delta_nn' delta_jj' E_an is added instead; classes 2, 4 and 8 are
 * unchanged. When the CI vectors diagonalise the target Hamiltonian and E are
 * their eigenvalues, the matrix is the one built without the option. n = 0
 * (E ignored) switches the option off. Before cch_plan, after the last target
 * symmetry (cch_plan fails with CCH_E_STATE if a symmetry was added since).
 * Host pointer unless flags holds CCH_MEM_DEVICE. CCH_E_INPUT for a count that
 * does not match the states or a non-finite energy. */
cch_status cch_set_target_energies(cch_ctx *ctx, const double *E, int64_t n, int32_t flags);

/* Plan the build (precision, tiles, memory budget). opts may be NULL for the
 * FP64 defaults. Allocates the device matrix.
 * With opts->flags & CCH_PLAN_SPARSE_L2 the L2 block (classes 2 and 8; Sec.
 * 2.2 names the off-diagonal pure-L2 class as the sparse one) is built and
 * stored as CSR of its structural non-zeros -- the L2 determinant pairs
 * within a double substitution, found by the excitation scan over all pairs,
 * both triangles, columns ascending, 12 bytes each -- and never as a dense
 * block. The rest is stored dense: the continuum columns of every row (the
 * continuum block and class 4, D x Dc) and the transpose of class 4 (Dc x
 * n_L2). Device memory is then about 8 (2 D Dc + ...) + 12 nnz bytes instead
 * of 8 D^2, so L2-heavy matrices far beyond the dense limit fit one GPU.
 * Every value equals the dense build's bit for bit. Such a context: solves
 * with the sparse L2 mat-vec (cch_davidson's CCH_DAV_SPARSE_L2 is implied);
 * serves cch_get_matrix, cch_get_elements, cch_get_block and
 * cch_get_diagonal from its parts; refuses cch_matrix_device (CCH_E_STATE)
 * and cannot join a batch. */
cch_status cch_plan(cch_ctx *ctx, const cch_plan_opts *opts);

/* Build the contracted matrix on the device (asynchronous on the stream):
 * classes 1, 3, 5, 6, 7 by CI contraction of transition densities followed by
 * expansion over (j, j') (Eq. 8 and Sec. 3.1), class 4 by the one-dimensional
 * contraction of Eq. 5, classes 2 and 8 by Slater's rules on bitstrings. */
cch_status cch_build(cch_ctx *ctx);

/* D = dimension, n_cont_rows = rows of continuum functions (before the L2). */
cch_status cch_get_dim(const cch_ctx *ctx, int64_t *D, int64_t *n_cont_rows);

/* Copy the symmetric matrix to out (row-major, leading dimension ld >= D),
 * host memory, or device memory with CCH_MEM_DEVICE. With CCH_LOWER only the
 * lower triangle (j <= i) is guaranteed to be written (the copy stops at the
 * diagonal of each row block, about half the bytes); without it every element.
 * The copy runs in row blocks of at most 1 GiB. A host copy is checked after
 * the transfer: its diagonal must equal the device's diagonal bit for bit,
 * else CCH_E_HIP (the contents of out are then undefined). Synchronous. */
cch_status cch_get_matrix(cch_ctx *ctx, double *out, int64_t ld, int32_t flags);

/* Device pointer and leading dimension of the resident matrix (owned by ctx,
 * valid until cch_destroy or the next cch_plan). */
cch_status cch_matrix_device(cch_ctx *ctx, const double **dptr, int64_t *ld);

/* Diagonal of the matrix (D values). */
cch_status cch_get_diagonal(cch_ctx *ctx, double *out, int32_t flags);

/* Sampled elements out[i] = H[rows[i]][cols[i]], i < n, of the built matrix
 * (Sec. 2.2), for matrices too large to copy whole. rows, cols and out are
 * host arrays unless flags holds CCH_MEM_DEVICE (then all three are device
 * arrays). Synchronous. CCH_E_INVALID_ARG for an index outside [0, D),
 * CCH_E_STATE before cch_build. */
cch_status cch_get_elements(cch_ctx *ctx, int64_t n, const int64_t *rows, const int64_t *cols, double *out,
                            int32_t flags);

/* One block of the matrix by the contraction classes of Sec. 2.2, row-major
 * into out (leading dimension ld >= the block width), host memory, or device
 * memory with CCH_MEM_DEVICE; elements of the block outside the class are 0.
 *   cls 1, 3, 5, 6, 7: rows of target symmetry sym_a by columns of sym_b, each
 *     indexed (n, j) -> n * n_c + j (n the state, j the coupled continuum
 *     orbital), S_a n_c(a) x S_b n_c(b). sym_a == sym_b: class 1 where the
 *     states agree (n = n'), class 3 where they differ; sym_a != sym_b coupled
 *     to the same continuum irrep: class 5 where the continuum orbitals agree
 *     (j = j', the diagonal of the local block), class 6 where they differ;
 *     different continuum irreps: class 7 (the whole block).
 *   cls 4: the L2 rows by the continuum columns of sym_a (n_L2 x S_a n_c(a));
 *     sym_b is not used.
 *   cls 2, 8: the L2 block (n_L2 x n_L2), its diagonal (2) or the rest (8);
 *     neither symmetry is used.
 * CCH_E_INVALID_ARG for a class that does not occur between the two
 * symmetries or a symmetry out of range; CCH_E_STATE before cch_build.
 * Synchronous. */
cch_status cch_get_block(cch_ctx *ctx, int32_t cls, int32_t sym_a, int32_t sym_b, double *out, int64_t ld,
                         int32_t flags);

/* Rows and columns of the block cch_get_block returns for (cls, sym_a, sym_b),
 * with the same argument checks; available after cch_plan. */
cch_status cch_block_shape(cch_ctx *ctx, int32_t cls, int32_t sym_a, int32_t sym_b, int64_t *rows, int64_t *cols);

/* Determinant-pair artefacts of the excitation scan (Sec. 2.1: XOR and
 * popcount for the degree, masks for the sign, four 16-bit orbital indices
 * per 64-bit label). For every connected pair (degree <= 2), in row-major
 * order of (x, y):
 *   CCH_PAIRS_TARGET   bra = det x of sym_a, ket = det y of sym_b; label
 *                      fields (p1, h1, p2, h2) with unused fields 0xFFFF;
 *   CCH_PAIRS_L2       bra = L2 x, ket = L2 y, y <= x; same label fields;
 *   CCH_PAIRS_L2_TARGET bra = target det y of sym_a plus the continuum
 *                      electron, ket = L2 x; fields (target particle or
 *                      0xFFFF, hole 1, hole 2 or 0xFFFF, 0xFFFF).
 * Host output arrays of capacity cap; *n receives the total count (arrays
 * untouched beyond cap). Synchronous. */
cch_status cch_get_labels(cch_ctx *ctx, int32_t which, int32_t sym_a, int32_t sym_b,
                          int32_t *x, int32_t *y, int8_t *degree, uint64_t *label,
                          int8_t *phase, int64_t cap, int64_t *n);

/* The N-electron target Hamiltonian between the determinants of target
 * symmetries sym_a (rows) and sym_b (columns): out[x][y] = <D_ax|H|D_by> over
 * target orbitals only, E_core on the diagonal (Sec. 3.1: the target-only
 * integrals, whose contraction the target-energy option replaces; Eq. 2's
 * CI vectors are eigenvectors of it when the target states are exact). The
 * values are those the build evaluated for its target pairs (zero where the
 * determinants are more than two substitutions apart). out is M_a x M_b
 * row-major with leading dimension ld >= M_b, host memory, or device memory
 * with CCH_MEM_DEVICE. After cch_build; synchronous. */
cch_status cch_target_hamiltonian(cch_ctx *ctx, int32_t sym_a, int32_t sym_b, double *out, int64_t ld,
                                  int32_t flags);

/* W = H V for b vectors of the built matrix (the product every iterative
 * diagonaliser of Sec. 3.2 is made of), in FP64 on the device. V and W hold
 * one vector per row: V[q * ldv + i], W[q * ldw + i], q < b, i < D,
 * ldv, ldw >= D; host arrays unless flags holds CCH_MEM_DEVICE (then both are
 * device arrays of the context's device and W may not overlap V). A dense
 * context reads the lower triangle of H once per 16 vectors; a context
 * planned with CCH_PLAN_SPARSE_L2 reads its continuum panels and the CSR of
 * the L2 block. The sums run in a fixed order: equal inputs give equal bits.
 * Scratch (and, for host arrays, staging) is allocated per call.
 * CCH_E_STATE before cch_build, CCH_E_INVALID_ARG for b < 0, a NULL array
 * with b > 0 or a leading dimension below D. Synchronous. */
cch_status cch_apply(cch_ctx *ctx, const double *V, int64_t ldv, int32_t b, double *W, int64_t ldw,
                     int32_t flags);

/* Lowest opts->k eigenpairs of the built matrix by block Davidson in FP64 on
 * the device. evals[k]; evecs[k][D] (row-major: eigenvector e at evecs + e*D);
 * either may be NULL. With flags & CCH_DAV_RESIDUALS, evecs has 2k rows and
 * rows k..2k-1 receive the residuals H x - theta x. With flags &
 * CCH_DAV_SPARSE_L2 the mat-vec reads the continuum rows and columns from the
 * dense matrix and the L2 block (classes 2 and 8, sparse when the L2
 * determinants are far apart) as CSR of its non-zeros, formed from the built
 * matrix on the first such solve after each build (device memory: 12 bytes
 * per non-zero, kept until cch_destroy); the eigenpairs agree with the dense
 * mat-vec's to rounding. Returns
 * CCH_E_NOT_CONVERGED (with the best pairs) when max_iter is reached.
 * Synchronous. */
cch_status cch_davidson(cch_ctx *ctx, const cch_dav_opts *opts, double *evals,
                        double *evecs, cch_dav_info *info, int32_t flags);

/* The Rayleigh-Ritz eigenproblem of cch_davidson, exposed for testing and
 * reuse: every eigenpair of a small dense symmetric matrix in FP64 on the
 * context's device and stream (the context needs no build). G is m x m,
 * 1 <= m <= 96, row-major with leading dimension ldg >= m; (G + G^T)/2 is
 * used. theta[m] receives the eigenvalues ascending; Y (m rows, leading
 * dimension ldy >= m) the orthonormal eigenvectors, eigenvector e in column
 * e (Y[q*ldy + e]). method CCH_EIG_AUTO: Householder tridiagonalisation,
 * eigenvalues by Sturm multisection, eigenvectors by twisted factorisation,
 * re-orthogonalised, with cyclic Jacobi when a check fails (*fallback, which
 * may be NULL, receives 1 then); CCH_EIG_JACOBI: cyclic Jacobi alone. Arrays
 * are host memory, or device memory with flags & CCH_MEM_DEVICE.
 * Synchronous. */
cch_status cch_subspace_eig(cch_ctx *ctx, const double *G, int32_t ldg, int32_t m,
                            double *theta, double *Y, int32_t ldy, int32_t method,
                            int32_t *fallback, int32_t flags);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments and results as cch_subspace_eig, with no device
 * allocation or free. Its staging buffers (used for host arrays) and its
 * fallback counter live in one fixed array per GPU of 148 480 bytes, held by
 * each GPU the library runs on until the process ends; m <= 96
 * (CCH_E_INVALID_ARG beyond). Every call on a GPU shares that GPU's array:
 * calls that overlap in time on one GPU (several threads, or concurrent
 * streams) race, and the caller must serialise them. Synchronous. */
cch_status cch_subspace_eig_noalloc(cch_ctx *ctx, const double *G, int32_t ldg, int32_t m,
                                    double *theta, double *Y, int32_t ldy, int32_t method,
                                    int32_t *fallback, int32_t flags);

/* Timing and work of cch_eig_all (device times from HIP events). */
typedef struct {
    double tridiag_ms;          /* Householder tridiagonalisation */
    double eigenvalues_ms;      /* multisection on Sturm counts */
    double vectors_ms;          /* twisted factorisations, cluster orthogonalisation, back-transformation */
    int32_t clusters;           /* runs of eigenvalues closer than 1e-5 ||T|| (re-orthogonalised) */
    int32_t clustered;          /* eigenvalues in those runs */
    double tridiag_bytes;       /* algorithmic bytes of the blocked reduction: the distinct (lower-triangle)
                                   elements of the trailing block, 8 B read per column and 16 B read and
                                   written per panel of 32 columns */
    double backtransform_flops; /* 2 n^3 when vectors are formed */
} cch_eig_info;

/* Every eigenpair of a dense real symmetric matrix in FP64 on the context's
 * device (Sec. 3.2: often all eigenvectors are required, and a dense
 * diagonaliser serves then). A = NULL: the built matrix (n = 0 or D; not
 * for CCH_PLAN_SPARSE_L2 contexts, CCH_E_STATE); else A is n x n row-major
 * with leading dimension lda >= n, both triangles read ((A + A^T)/2 is
 * used). w[n] receives the
 * eigenvalues ascending; V (may be NULL: eigenvalues only) receives the
 * orthonormal eigenvectors as rows, eigenvector e at V + e * ldv (ldv >= n).
 * Householder tridiagonalisation (blocked in panels of 32 columns),
 * multisection on Sturm counts, twisted factorisations with modified
 * Gram-Schmidt (and inverse iteration for vectors that collapse) inside
 * clusters of eigenvalues closer than 1e-5 ||T||, and the
 * back-transformation in blocks of 128 reflectors on FP64 MFMA. Every sum
 * runs in a fixed order: the same input gives the same bits. Work space about 3 n^2 doubles of device memory
 * (n^2 for eigenvalues only). A, w and V are host memory, or device memory
 * with CCH_MEM_DEVICE. info may be NULL. CCH_E_INPUT for a non-finite
 * matrix. Synchronous. */
cch_status cch_eig_all(cch_ctx *ctx, const double *A, int64_t lda, int32_t n, double *w, double *V, int64_t ldv,
                       int32_t flags, cch_eig_info *info);

/* Device time of the last cch_build in milliseconds (HIP events around the
 * queued work on the context's stream), and per-phase times (phases[8],
 * NULL allowed): 0 excitation scans, 1 target elements + densities,
 * 2 integral relayout, 3 expansion GEMM, 4 class 4, 5 classes 2/8,
 * 6 mirror + diagonal, 7 reserved (0). Synchronous. */
cch_status cch_build_time(cch_ctx *ctx, float *total_ms, float *phases);

/* Work counts of the planned build, for throughput and roofline figures:
 * out[0] lower-triangle elements computed (D(D+1)/2 when stored dense; with
 * CCH_PLAN_SPARSE_L2 the dense parts plus the L2 block's structural non-zeros
 * of the lower triangle), out[1] expansion GEMM flops (2 * rows * cols * K
 * summed over symmetry pairs), out[2] connected target pairs, out[3]
 * connected L2 x target pairs, out[4] relayout bytes moved (read + write),
 * out[5] class-4 outputs, out[6] L2 lower-triangle elements computed (all of
 * them dense, the structural non-zeros sparse), out[7] number of symmetry
 * pairs. */
cch_status cch_work_counts(const cch_ctx *ctx, double *out8);

/* Algorithmic work of the last build, for throughput and roofline figures;
 * out[i] for i < n (entries 13 and up are 0). Synchronous (it counts the
 * excitation lists the build produced, and the connected L2 pairs by a
 * counting pass of the excitation scan). CCH_E_STATE before cch_build.
 *   0-7  as cch_work_counts;
 *   8    connected target pairs of degree 0 or 1 (those the transition
 *        densities of Eq. 8 use);
 *   9    transition-density flops: one multiply-add (2 flops) per (n, n') row
 *        per density update; a degree-0 pair makes 1.5 N updates (every
 *        occupied spin-orbital in the spin-summed diagonal, the alpha ones in
 *        the alpha-resolved one), an alpha excitation 2, a beta one 1;
 *   10   class-4 flops (Eq. 5): 2 S n_c per connected L2 x target pair (one
 *        outer product of a CI row with an integral row over j);
 *   11   connected L2 x L2 pairs (degree <= 2), lower triangle with the
 *        diagonal: the structural non-zeros of classes 2 and 8;
 *   12   bytes of the mirror: 16 per element above the diagonal. */
cch_status cch_work_detail(cch_ctx *ctx, double *out, int32_t n);

/* Device memory held by the planned context (bytes) and the number of passes
 * the expansion product takes under cch_plan_opts.max_device_bytes (1 when
 * unsplit). Contexts planned in several passes cannot join a batch
 * (cch_batch_create returns CCH_E_STATE). Either pointer may be NULL. */
cch_status cch_plan_info(cch_ctx *ctx, int64_t *device_bytes, int32_t *expansion_passes);

/* ------------------------------------------------------------------------
 * Learned Davidson preconditioner (not in the paper): a 3-layer perceptron
 * 4 -> 128 -> 128 -> 1 (ReLU) maps per-row features of a Ritz pair (theta,
 * H_ii, off-diagonal row norm, row class) to g and the correction becomes
 * exp(clamp(g, -4, 4)) r_i / (theta - H_ii); the diagonal (Jacobi) step is the
 * fallback. Weights are an FP32 blob of cch_mlp_num_params() floats:
 * W1[128][4], b1[128], W2[128][128], b2[128], w3[128], b3. The 128 x 128 layer
 * runs on BF16 matrix cores with FP32 accumulation; training uses Adam in FP32.
 * Training rows: features X[n][4] (see cch_mlp_features), the Jacobi step tj,
 * the target correction e and a weight w per row; loss = sum w (exp(g) tj - e)^2.
 * Array arguments are host pointers unless flags & CCH_MEM_DEVICE.
 * ------------------------------------------------------------------------ */
typedef struct cch_mlp cch_mlp;

int32_t cch_mlp_num_params(void);
/* He-initialised weights from `seed`, output layer near zero (starts as Jacobi). */
cch_status cch_mlp_create(cch_mlp **out, int32_t device, void *hip_stream, uint64_t seed);
cch_status cch_mlp_destroy(cch_mlp *m);
const char *cch_mlp_last_error(const cch_mlp *m);
cch_status cch_mlp_set_weights(cch_mlp *m, const float *w, int64_t n, int32_t flags);
cch_status cch_mlp_get_weights(cch_mlp *m, float *w, int64_t n, int32_t flags);
/* g[n] = network(X[n][4]). Synchronous. */
cch_status cch_mlp_forward(cch_mlp *m, const float *X, int64_t n, float *g, int32_t flags);
/* loss and its gradient grad[num_params] (FP32) for the rows. Synchronous. */
cch_status cch_mlp_grad(cch_mlp *m, const float *X, const float *tj, const float *e, const float *w, int64_t n,
                        double *loss, float *grad, int32_t flags);
/* one Adam step (lr) on the rows; *loss = loss before the step. Synchronous. */
cch_status cch_mlp_train_step(cch_mlp *m, const float *X, const float *tj, const float *e, const float *w,
                              int64_t n, float lr, double *loss, int32_t flags);
/* Feature rows of the built matrix for one Ritz value theta: X[D][4]
 * (asinh(d), asinh(rho), asinh(rho/|d|), L2-row flag; d = theta - H_ii
 * floored at 1e-8, rho = off-diagonal row norm). Synchronous. */
cch_status cch_mlp_features(cch_ctx *ctx, double theta, float *X, int32_t flags);
/* Attach (or detach with NULL) the network used by CCH_PRECOND_MLP. */
cch_status cch_davidson_set_mlp(cch_ctx *ctx, cch_mlp *m);

/* ------------------------------------------------------------------------
 * Batched build: many instances of uneven size built together. Every context
 * must be planned with the FP64 form, on the same device. The build phases of
 * all instances are queued on one internal stream; the expansion products of
 * all (instance, symmetry pair), all class-4 rows and all L2 tiles each run as
 * one persistent launch walking a tile list, and the whole sequence is
 * captured once in a hipGraph and replayed on every cch_batch_build.
 * With CCH_BATCH_AUTOTUNE, cch_batch_create times candidate tile heights of
 * the expansion product and grid sizes of the persistent launches on the
 * device and keeps the fastest (cached per batch shape for the process).
 * Results are bit-identical to building each context alone.
 * ------------------------------------------------------------------------ */
typedef struct cch_batch cch_batch;

#define CCH_BATCH_AUTOTUNE 1

/* ctxs[n]: planned contexts (caller keeps ownership; they must outlive the
 * batch). Synchronous: waits for the contexts' streams. */
cch_status cch_batch_create(cch_batch **out, cch_ctx *const *ctxs, int32_t n, int32_t flags);
/* Build every context's matrix (graph replay); synchronous. Afterwards each
 * context is built: cch_get_matrix / cch_davidson work on it as usual. */
cch_status cch_batch_build(cch_batch *b);
/* Device time of the last cch_batch_build in ms (HIP events around the graph). */
cch_status cch_batch_time(const cch_batch *b, float *ms);
/* out[8]: expansion tile height, expansion grid, class-4 grid, L2 grid,
 * autotuned (0/1), taken from the cache (0/1), graph nodes, instances. */
cch_status cch_batch_info(const cch_batch *b, int32_t *out8);
cch_status cch_batch_destroy(cch_batch *b);
const char *cch_batch_last_error(const cch_batch *b);

#ifdef __cplusplus
}
#endif
#endif
