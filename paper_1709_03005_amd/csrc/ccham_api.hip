// Host runtime of the ccham C ABI: input validation, device upload, build
// plan (pair-list sizing, label slots, row lists), the asynchronous build
// sequence, read-out, and the block Davidson driver. See include/ccham.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/ccham.h"
#include "ccham_internal.h"

namespace cch {
// launchers defined in the kernel files
hipError_t launch_pair_values(int W, TgtInts I, const uint64_t *da, const uint64_t *db, PairList pl,
                              int64_t n, double *hv, hipStream_t st);
hipError_t launch_energy_rows(int nrows, const int32_t *rn, const int32_t *rn2, const double *E, double *HT,
                              hipStream_t st);
hipError_t launch_projection(int M, const int64_t *row_off, const int64_t *row_cnt, PairList pl,
                             const double *hv, const double *ca, int Sa, const double *cb, int Sb,
                             int nrows, const int32_t *rn, const int32_t *rn2, double *Y, double *Yo,
                             double *HT, double *O, hipStream_t st);
hipError_t launch_bucket(PairList pl, int64_t n, const int32_t *pqidx, int n_o, int n_slot, int M,
                         int32_t *key, int64_t *count, int64_t *start, int64_t *cursor, int64_t *sorted,
                         int64_t *tmp, int64_t *d0, hipStream_t st);
hipError_t launch_gamma(int W, PairList pl, const int64_t *start, const int64_t *count,
                        const int64_t *sorted, const int64_t *d0, int M0, const int32_t *slotP,
                        const int32_t *slotQ, int n_slot, const uint64_t *da, const int8_t *spa, const int8_t *spb,
                        const double *ca, int Sa, const double *cb, int Sb, int nrows, const int32_t *rn,
                        const int32_t *rn2, double *At, hipStream_t st);
hipError_t launch_relayout(const double *ttcc, const double *tctc, int n_o, int n_cont,
                           const int32_t *slotP, const int32_t *slotQ, int n_slot, int ja0, int nca,
                           int jb0, int ncb, double *B, hipStream_t st, const PackedCC *pk);
struct ExpandEpi {
    double *H;
    int64_t ld;
    int64_t row0a, row0b;
    int nca, ncb;
    int ja0, jb0;
    const int32_t *rn, *rn2;
    const double *HT, *O;
    const double *h;
    int n_o, n_orb;
};
hipError_t launch_expand_f64(const double *At, const double *B, int nrows, int N, int K, const ExpandEpi &ep,
                             hipStream_t st);
hipError_t launch_to_f32(const double *x, float *y, int64_t n, hipStream_t st);
hipError_t launch_expand_f32(const float *At, const float *B, int nrows, int N, int K, const ExpandEpi &ep,
                             hipStream_t st);
hipError_t launch_slices(const double *At, int nrows, const double *B, int K, int N, int s, int ldk,
                         double *sigA, __bf16 *SA, double *sigB, __bf16 *SB, hipStream_t st);
hipError_t launch_expand_bf16split(const __bf16 *SA, const __bf16 *SB, const double *sigA, const double *sigB,
                                   int s, int nrows, int N, int ldk, const ExpandEpi &ep, hipStream_t st);
hipError_t launch_class4(int W, const Class4Args &a, int n_l2, hipStream_t st);
struct L2Args {
    const uint64_t *dets;
    int n_l2;
    TgtInts I;
    double *H;
    int64_t ld;
    int64_t row0;
};
hipError_t launch_l2_block(int W, const L2Args &a, hipStream_t st);
hipError_t launch_l2csf_gather(const double *Hd, int64_t ldd, int Dc, int ncsf, const int32_t *start,
                               const int32_t *det, const double *coef, double *H, int64_t ld, hipStream_t st);
struct GemmTask {
    const double *At;
    const double *B;
    int nrows, N, K;
    int tiles_m, tiles_n;
    int64_t first;
    ExpandEpi ep;
};
struct L2Task {
    L2Args a;
    int64_t first;
};
int expand_tiles(int nrows, int N, int bm);
int64_t l2_tiles(int n_l2);
hipError_t launch_expand_f64_batched(const GemmTask *tasks, int ntask, int64_t total, int bm, int grid,
                                     hipStream_t st);
hipError_t launch_l2_batched(int W, const L2Task *tasks, int ntask, int64_t total, int grid, hipStream_t st);
hipError_t launch_class4_batched(int W, const C4Task *tasks, int ntask, int64_t total, int grid, hipStream_t st);
hipError_t launch_mirror(double *H, int64_t ld, int D, hipStream_t st);
hipError_t launch_scatter_pairs(const int32_t *px, const int32_t *py, const double *v, int64_t n, int transpose,
                                double *out, int64_t ldo, hipStream_t st);
hipError_t launch_pair_census(const int8_t *deg, const uint64_t *label, int64_t n, unsigned long long *out,
                              hipStream_t st);
hipError_t launch_diag(const double *H, int64_t ld, int D, double *out, hipStream_t st);
hipError_t launch_gather_elements(const double *H, int64_t ldh, const int64_t *rows, const int64_t *cols, int64_t n,
                                  double *out, hipStream_t st);
hipError_t launch_get_block(const double *H, int64_t ldh, int64_t row0, int nrows, int64_t col0, int ncols, int mode,
                            int nca, int ncb, double *out, int64_t ldo, hipStream_t st);
// Davidson
hipError_t launch_l2_csr_count(const double *H, int64_t ld, int Dc, int nl2, int64_t *cnt, hipStream_t st);
hipError_t launch_l2_csr_fill(const double *H, int64_t ld, int Dc, int nl2, const int64_t *off, int32_t *col,
                              double *val, hipStream_t st);
hipError_t launch_matvec_l2csr(const double *P, int64_t ldp, const double *R, int64_t ldr, int rc0, int D, int Dc,
                               const int64_t *off, const int32_t *col, const double *val, const double *V,
                               int64_t ldv, int b, double *W, int64_t ldw, double *Wp, hipStream_t st);
// sparse L2 block (classes 2 and 8 as CSR)
hipError_t launch_l2s_struct(int W, const uint64_t *dets, int n, const int64_t *off, int64_t *cnt, int32_t *col,
                             hipStream_t st);
hipError_t launch_l2s_values(int W, const uint64_t *dets, int n, const TgtInts &I, const int64_t *off,
                             const int32_t *col, double *val, double *diag, hipStream_t st);
hipError_t launch_transpose_c4(const double *P, int64_t ldp, int Dc, int nl2, double *R, int64_t ldr, hipStream_t st);
hipError_t launch_sparse_gather(const SparseMat &S, const int64_t *rows, const int64_t *cols, int64_t n, double *out,
                                hipStream_t st);
hipError_t launch_sparse_principal(const SparseMat &S, const int32_t *idx, int ns, double *G, int ldg, hipStream_t st);
hipError_t launch_sparse_rows(const SparseMat &S, int64_t r0, int nr, int64_t c0, int ncols, int mode, double *out,
                              int64_t ldo, hipStream_t st);
hipError_t launch_sparse_row_norms(const SparseMat &S, int D, double *rho, hipStream_t st);
// full-spectrum eigensolver
hipError_t launch_eig_gemm(int M, int N, int K, double alpha, const double *A, int64_t sai, int64_t sak,
                           const double *B, int64_t sbk, int64_t sbj, double beta, double *C, int64_t ldc,
                           hipStream_t st, double *P = nullptr, int64_t p_cap = 0, int lowq = -1);
hipError_t launch_trd_panel(double *A, int64_t lda, int n, int j0, int nbp, const TrdVec &V, const TrdPanel &P,
                            hipStream_t st);
hipError_t launch_tri_eigenvalues(const double *d, const double *e, double *e2, int n, const int32_t *bs,
                                  const int32_t *bm, const int32_t *bk, double lo, double hi, double pivmin,
                                  double *w, hipStream_t st);
hipError_t launch_tri_vectors(const double *d, const double *e, int n, const int32_t *bs, const int32_t *bm,
                              const double *w, double pivmin, double *Z, int64_t ldz, double *S, int64_t lds,
                              hipStream_t st);
hipError_t launch_cluster_mgs(double *Z, int64_t ldz, const int32_t *desc, int ncl, const int32_t *cols, const double *d,
                              const double *e, const double *w, double *S, int64_t lds, double piv, hipStream_t st);
hipError_t launch_copy_reflectors(const double *A, int64_t lda, int n, int j0, int nb, double *Vb, hipStream_t st);
hipError_t launch_larft(const double *G, const double *tau, int nb, double *T, double *X, hipStream_t st);
hipError_t launch_symmetrize(double *W, int64_t ld, int n, hipStream_t st);
hipError_t launch_transpose_sq(const double *Z, int64_t ldz, int n, double *out, int64_t ldo, hipStream_t st);
int64_t l2csr_scratch(int D, int Dc);
hipError_t launch_matvec(const double *H, int64_t ld, int D, const double *V, int64_t ldv, int b, double *W,
                         int64_t ldw, double *Wp, hipStream_t st);
int matvec_splits(int D);
int64_t matvec_scratch_doubles(int D);
int64_t tn_part_doubles();
hipError_t launch_tn(const double *X1, int64_t ldx1, int na1, const double *X2, int64_t ldx2, int na,
                     const double *Y, int64_t ldy, int nc, int D, double *part, double *out, int64_t ldo,
                     int transpose, hipStream_t st, double *outT = nullptr, int cT = 0);
hipError_t launch_nn(const double *V1, int64_t ldv1, int m1, const double *V2, int64_t ldv2, int m, int D,
                     const double *C, int ldc, int ne, const double *base, int64_t ldb, double beta, double alpha,
                     double *out, int64_t ldo, hipStream_t st, const double *V1z = nullptr,
                     double *outz = nullptr);
hipError_t launch_residual(const double *AX, const double *X, int64_t ld, int D, const double *theta, int k,
                           double *R, double *part, double *norms, hipStream_t st);
hipError_t launch_jacobi_correct(const double *R, int64_t ld, int D, const double *diag, const double *theta,
                                 const DavSel &sel, int nsel, double *T, int64_t ldt, hipStream_t st);
hipError_t launch_pchol(const double *G, int ldg, int b, const double *S, int lds, int m, const double *ref,
                        int ref_stride, double rel, double *C, int ldc, int32_t *rank, hipStream_t st);
hipError_t launch_jacobi_eig(const double *G, int ldg, int m, double *theta, double *Y, int ldy, hipStream_t st);
hipError_t launch_rr_eig(const double *G, int ldg, int m, double *theta, double *Y, int ldy, int32_t *nfallback,
                         hipStream_t st);
hipError_t launch_g_ritz(double *G, int ldg, int m, const double *theta, hipStream_t st);
hipError_t launch_unit_vectors(double *V, int64_t ldv, int D, const int32_t *idx, int b, hipStream_t st);
hipError_t launch_gather_principal(const double *H, int64_t ld, const int32_t *idx, int ns, double *G, int ldg,
                                   hipStream_t st);
hipError_t launch_seed_scatter(double *V, int64_t ldv, const int32_t *idx, const double *Y, int ldy, int ns, int b,
                               hipStream_t st);
// learned preconditioner
int mlp_num_params();
int mlp_grid(int64_t n);
hipError_t launch_mlp_pack(const float *w, __bf16 *w2, __bf16 *w2t, hipStream_t st);
hipError_t launch_mlp_forward(const float *w, const __bf16 *w2, const __bf16 *w2t, const float *X, int64_t n,
                              float *g, hipStream_t st);
hipError_t launch_mlp_grad(const float *w, const __bf16 *w2, const __bf16 *w2t, const float *X, const float *tj,
                           const float *ev, const float *wr, int64_t n, float *part, double *lpart, float *grad,
                           double *loss, hipStream_t st);
hipError_t launch_adam(float *w, float *m, float *v, const float *g, float lr, int step, hipStream_t st);
hipError_t launch_row_norms(const double *H, int64_t ld, int D, double *rho, hipStream_t st);
hipError_t launch_mlp_dav(const float *w, const __bf16 *w2, const __bf16 *w2t, const double *R, int64_t ld, int D,
                          int Dc, const double *diag, const double *rho, const double *theta, const DavSel &sel,
                          int nsel, float *X, float *g, double *T, int64_t ldt, int32_t *nfallback, hipStream_t st);
}  // namespace cch

struct cch_mlp;

using namespace cch;

namespace {

struct DevPairs {
    int64_t n = 0;
    int64_t *row_off = nullptr, *row_cnt = nullptr;
    PairList pl{};
};

struct SymInfo {
    int irrep = 0, M = 0, S = 0, nc = 0, ja0 = 0;
    int64_t row0 = 0, e_off = 0;   // first row; first of its states' target energies
    uint64_t *d_dets = nullptr;
    int8_t *d_cspin = nullptr;   // continuum spin per det (0 alpha, 1 beta); nullptr: alpha throughout
    double *d_ci = nullptr;
    std::vector<uint64_t> h_dets;
};

struct PairPlan {
    int a = 0, b = 0;
    DevPairs pr;
    int n_slot = 0, nrows = 0;
    int32_t *d_slotP = nullptr, *d_slotQ = nullptr, *d_pqidx = nullptr, *d_rn = nullptr, *d_rn2 = nullptr;
    double *d_hv = nullptr, *d_Y = nullptr, *d_Yo = nullptr, *d_HT = nullptr, *d_O = nullptr, *d_At = nullptr;
    int32_t *d_key = nullptr;
    int64_t *d_count = nullptr, *d_start = nullptr, *d_cursor = nullptr, *d_sorted = nullptr, *d_tmp = nullptr,
            *d_d0 = nullptr;
    double *d_B = nullptr;   // integral rows laid out for this pair's expansion
    int jj_chunk = 0;        // continuum orbitals (rows j) per expansion pass; < nca: passes share d_B
    // reduced-precision operands of the expansion product
    float *d_At32 = nullptr, *d_B32 = nullptr;
    double *d_sigA = nullptr, *d_sigB = nullptr;
    __bf16 *d_SA = nullptr, *d_SB = nullptr;
    int ldk = 0;
};

struct LtPlan {
    int sym = 0;
    DevPairs pr;
};

}  // namespace

constexpr int CCH_NAUX = 6;   // auxiliary streams of a build: 4 for the symmetry pairs, class 4, L2 block
constexpr int CCH_NPAIRS_ST = 4;

struct cch_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<void *> allocs;
    int64_t bytes = 0;
    // orbitals
    bool have_orb = false;
    int n_o = 0, n_irrep = 1, total_irrep = 0, n_cont = 0, n_orb = 0, W = 0;
    std::vector<uint8_t> tgt_irrep;
    std::vector<int> n_c, cont_start;
    // integrals
    bool have_ints = false;
    double *d_h = nullptr, *d_tttt = nullptr, *d_tttc = nullptr, *d_ttcc = nullptr, *d_tctc = nullptr;
    // symmetry-packed (tt|cc) / (tc|tc): record offsets per target pair (device)
    // and block offsets blk[x * n_irrep + ca] inside a record (host)
    bool packed = false;
    int64_t *d_pk_rec = nullptr;
    std::vector<int64_t> pk_blk;
    double e_core = 0.0;
    // target energies on the diagonal (all states, symmetry by symmetry)
    bool energy_mode = false;
    std::vector<double> h_tgtE;
    double *d_tgtE = nullptr;
    // determinant spaces
    int n_elec = -1;
    std::vector<SymInfo> syms;
    int n_l2 = 0;               // L2 determinants
    uint64_t *d_l2 = nullptr;
    std::vector<uint64_t> h_l2;
    // L2 functions as CSFs (cch_set_l2_csf): the build writes the matrix over
    // the L2 determinants into d_Hd (Dd x ldd); k_l2csf_gather then forms the
    // matrix over the CSFs in d_H
    int n_l2r = 0;              // L2 rows of the matrix: the CSFs, else the determinants
    bool l2csf = false;
    std::vector<int32_t> h_csf_start, h_csf_det;
    std::vector<double> h_csf_coef;
    int32_t *d_csf_start = nullptr, *d_csf_det = nullptr;
    double *d_csf_coef = nullptr;
    double *d_Hd = nullptr;
    int64_t Dd = 0, ldd = 0;
    double *d_Hb = nullptr;     // the matrix the build kernels write: d_H, or d_Hd with CSFs
    int64_t ldb = 0;
    // plan
    bool planned = false, built = false;
    cch_plan_opts opts{};
    int64_t D = 0, Dc = 0, ld = 0;
    int64_t build_gen = 0;   // builds started; a cached CSR of the L2 block belongs to one
    struct {
        int64_t gen = -1, nnz = 0, cap = 0;
        int64_t *off = nullptr;
        int32_t *col = nullptr;
        double *val = nullptr;
        bool planned = false;   // sparse plan: allocated with the plan (freed with it)
    } csr;
    double *d_H = nullptr, *d_diag = nullptr, *d_B = nullptr;
    // CCH_PLAN_SPARSE_L2: d_H holds the continuum columns of every row (leading
    // dimension ld >= Dc), d_R the transpose of class 4, csr the L2 block
    bool sparse = false;
    double *d_R = nullptr;
    int64_t ldr = 0;
    std::vector<PairPlan> pp;
    std::vector<LtPlan> lt;
    hipEvent_t ev[8] = {};
    hipEvent_t mv0 = nullptr, mv1 = nullptr, rr0 = nullptr, rr1 = nullptr;
    // auxiliary streams (default priority) over which a build phase spreads its
    // independent per-pair work; joined back into `stream` before the phase ends
    hipStream_t aux[CCH_NAUX] = {};
    hipEvent_t fork_ev = nullptr, join_ev[CCH_NAUX] = {};
    hipEvent_t c4_ev[2] = {}, l2_ev[2] = {};   // timing of the class-4 and L2 streams
    bool have_aux = false;
    bool overlapped = false;   // the last build ran class 4 and the L2 block beside the pair phases
    int64_t relayout_elems = 0;
    int expansion_passes = 1;   // > 1: the budget split the expansion into column passes
    bool b_shared = false;      // all pairs use one integral-row buffer, laid out just before each product
    bool timed = false;     // the phase events belong to the last build
    cch_mlp *mlp = nullptr; // network used by CCH_PRECOND_MLP
    bool have_events = false;
};

static thread_local std::string g_create_err;

static cch_status fail(cch_ctx *c, cch_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_err = buf;
    return code;
}

#define HIPCK(c, x)                                                                              \
    do {                                                                                         \
        hipError_t e_ = (x);                                                                     \
        if (e_ != hipSuccess) return fail((c), CCH_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

template <class T>
static cch_status dalloc(cch_ctx *c, T **p, size_t n)
{
    size_t bytes = sizeof(T) * (n ? n : 1);
    if (c->opts.max_device_bytes > 0 && c->bytes + (int64_t)bytes > c->opts.max_device_bytes)
        return fail(c, CCH_E_OOM, "device budget of %lld bytes exceeded", (long long)c->opts.max_device_bytes);
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(c, CCH_E_OOM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    c->allocs.push_back(q);
    c->bytes += (int64_t)bytes;
    *p = (T *)q;
    return CCH_OK;
}

#define TRY(x)                          \
    do {                                \
        cch_status s_ = (x);            \
        if (s_ != CCH_OK) return s_;    \
    } while (0)

static void free_plan(cch_ctx *c)
{
    // plan buffers are appended after the input buffers; free everything and
    // re-upload is avoided by keeping inputs in the first allocations
    (void)c;
}

static int popc64(uint64_t x) { return __builtin_popcountll(x); }

static cch_status copy_in(cch_ctx *c, void *dst, const void *src, size_t bytes, int32_t flags)
{
    HIPCK(c, hipMemcpyAsync(dst, src, bytes, (flags & CCH_MEM_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                            c->stream));
    return CCH_OK;
}

static cch_status host_copy(cch_ctx *c, void *dst, const void *src, size_t bytes, int32_t flags)
{
    if (flags & CCH_MEM_DEVICE) {
        HIPCK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream));
        HIPCK(c, hipStreamSynchronize(c->stream));
    } else {
        memcpy(dst, src, bytes);
    }
    return CCH_OK;
}

// context fields for the allocation-free entry point (ccham_noalloc.hip); not exported
__attribute__((visibility("hidden"))) int32_t cch_ctx_device(const cch_ctx *c) { return c->device; }
__attribute__((visibility("hidden"))) hipStream_t cch_ctx_stream(const cch_ctx *c) { return c->stream; }
__attribute__((visibility("hidden"))) cch_status cch_ctx_fail(cch_ctx *c, cch_status code, const char *msg)
{
    return fail(c, code, "%s", msg);
}

// exported functions keep the C linkage of their declarations in ccham.h

const char *cch_version(void) { return "ccham 0.1.0 (gfx950)"; }

cch_status cch_create(cch_ctx **out, int32_t device, void *hip_stream)
{
    if (!out) return fail(nullptr, CCH_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(nullptr, CCH_E_HIP, "no HIP device: %s", hipGetErrorString(e));
    if (device < 0 || device >= ndev) return fail(nullptr, CCH_E_INVALID_ARG, "device %d out of range", device);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, CCH_E_HIP, "hipSetDevice: %s", hipGetErrorString(e));
    cch_ctx *c = new (std::nothrow) cch_ctx();
    if (!c) return fail(nullptr, CCH_E_OOM, "context allocation failed");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    for (auto &ev : c->ev) {
        if (hipEventCreate(&ev) != hipSuccess) {
            delete c;
            return fail(nullptr, CCH_E_HIP, "hipEventCreate failed");
        }
    }
    if (hipEventCreate(&c->mv0) != hipSuccess || hipEventCreate(&c->mv1) != hipSuccess ||
        hipEventCreate(&c->rr0) != hipSuccess || hipEventCreate(&c->rr1) != hipSuccess) {
        delete c;
        return fail(nullptr, CCH_E_HIP, "hipEventCreate failed");
    }
    c->have_events = true;
    bool aux_ok = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < CCH_NAUX && aux_ok; ++i)
        aux_ok = hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < 2 && aux_ok; ++i)
        aux_ok = hipEventCreate(&c->c4_ev[i]) == hipSuccess && hipEventCreate(&c->l2_ev[i]) == hipSuccess;
    c->have_aux = aux_ok;   // without them every phase runs on the context stream
    c->opts.precision = CCH_PREC_FP64;
    *out = c;
    return CCH_OK;
}

cch_status cch_destroy(cch_ctx *c)
{
    if (!c) return CCH_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (void *p : c->allocs) (void)hipFree(p);
    if (!c->csr.planned) {
        (void)hipFree(c->csr.off);
        (void)hipFree(c->csr.col);
        (void)hipFree(c->csr.val);
    }
    if (c->have_events)
        for (auto &ev : c->ev) (void)hipEventDestroy(ev);
    if (c->mv0) (void)hipEventDestroy(c->mv0);
    if (c->mv1) (void)hipEventDestroy(c->mv1);
    if (c->rr0) (void)hipEventDestroy(c->rr0);
    if (c->rr1) (void)hipEventDestroy(c->rr1);
    for (int i = 0; i < CCH_NAUX; ++i) {
        if (c->aux[i]) {
            (void)hipStreamSynchronize(c->aux[i]);
            (void)hipStreamDestroy(c->aux[i]);
        }
        if (c->join_ev[i]) (void)hipEventDestroy(c->join_ev[i]);
    }
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    for (int i = 0; i < 2; ++i) {
        if (c->c4_ev[i]) (void)hipEventDestroy(c->c4_ev[i]);
        if (c->l2_ev[i]) (void)hipEventDestroy(c->l2_ev[i]);
    }
    delete c;
    return CCH_OK;
}

const char *cch_last_error(const cch_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

cch_status cch_sync(cch_ctx *c)
{
    if (!c) return CCH_E_INVALID_ARG;
    HIPCK(c, hipStreamSynchronize(c->stream));
    return CCH_OK;
}

cch_status cch_set_orbitals(cch_ctx *c, int32_t n_o, const uint8_t *tgt_irrep, int32_t n_irrep,
                            const int32_t *n_c_per_irrep, int32_t total_irrep)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (c->have_orb) return fail(c, CCH_E_STATE, "orbitals already set");
    if (n_o <= 0 || !tgt_irrep || !n_c_per_irrep) return fail(c, CCH_E_INVALID_ARG, "bad orbital arguments");
    if (n_irrep != 1 && n_irrep != 2 && n_irrep != 4 && n_irrep != 8)
        return fail(c, CCH_E_INVALID_ARG, "n_irrep must be 1, 2, 4 or 8 (abelian group, XOR product)");
    if (total_irrep < 0 || total_irrep >= n_irrep) return fail(c, CCH_E_INVALID_ARG, "bad total_irrep");
    int64_t nc = 0;
    for (int a = 0; a < n_irrep; ++a) {
        if (n_c_per_irrep[a] < 0) return fail(c, CCH_E_INVALID_ARG, "negative continuum count");
        nc += n_c_per_irrep[a];
    }
    for (int p = 0; p < n_o; ++p)
        if (tgt_irrep[p] >= n_irrep) return fail(c, CCH_E_INVALID_ARG, "target orbital %d has irrep >= n_irrep", p);
    if (2 * ((int64_t)n_o + nc) >= 0xFFFF)
        return fail(c, CCH_E_LIMIT, "%lld orbitals exceed the 16-bit label fields", (long long)(n_o + nc));
    const int W = (2 * n_o + 63) / 64;
    if (W > CCH_MAXW) return fail(c, CCH_E_LIMIT, "n_o = %d needs %d words (max %d)", n_o, W, CCH_MAXW);
    c->n_o = n_o;
    c->n_irrep = n_irrep;
    c->total_irrep = total_irrep;
    c->n_cont = (int)nc;
    c->n_orb = n_o + (int)nc;
    c->W = W;
    c->tgt_irrep.assign(tgt_irrep, tgt_irrep + n_o);
    c->n_c.assign(n_c_per_irrep, n_c_per_irrep + n_irrep);
    c->cont_start.assign(n_irrep + 1, 0);
    for (int a = 0; a < n_irrep; ++a) c->cont_start[a + 1] = c->cont_start[a] + c->n_c[a];
    c->have_orb = true;
    return CCH_OK;
}

cch_status cch_set_integrals(cch_ctx *c, const double *h, const double *tttt, const double *tttc,
                             const double *ttcc, const double *tctc, double e_core, int32_t flags)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->have_orb) return fail(c, CCH_E_STATE, "set orbitals first");
    if (c->have_ints) return fail(c, CCH_E_STATE, "integrals already set");
    if (!h || !tttt || (c->n_cont && (!tttc || !ttcc || !tctc)))
        return fail(c, CCH_E_INVALID_ARG, "integral pointer is NULL");
    if (!std::isfinite(e_core)) return fail(c, CCH_E_INPUT, "e_core is not finite");
    const size_t no = c->n_o, nc = c->n_cont, norb = c->n_orb;
    const size_t nh = norb * norb, n4 = no * no * no * no, n3c = no * no * no * nc, n2c = no * no * nc * nc;
    TRY(dalloc(c, &c->d_h, nh));
    TRY(dalloc(c, &c->d_tttt, n4));
    TRY(dalloc(c, &c->d_tttc, n3c));
    TRY(dalloc(c, &c->d_ttcc, n2c));
    TRY(dalloc(c, &c->d_tctc, n2c));
    TRY(copy_in(c, c->d_h, h, nh * 8, flags));
    TRY(copy_in(c, c->d_tttt, tttt, n4 * 8, flags));
    if (nc) {
        TRY(copy_in(c, c->d_tttc, tttc, n3c * 8, flags));
        TRY(copy_in(c, c->d_ttcc, ttcc, n2c * 8, flags));
        TRY(copy_in(c, c->d_tctc, tctc, n2c * 8, flags));
    }
    HIPCK(c, hipStreamSynchronize(c->stream));
    c->e_core = e_core;
    c->have_ints = true;
    return CCH_OK;
}

cch_status cch_set_integrals_packed(cch_ctx *c, const double *h, const double *tttt, const double *tttc,
                                    const double *ttcc, const double *tctc, double e_core, int32_t flags)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->have_orb) return fail(c, CCH_E_STATE, "set orbitals first");
    if (c->have_ints) return fail(c, CCH_E_STATE, "integrals already set");
    if (!h || !tttt || (c->n_cont && (!tttc || !ttcc || !tctc)))
        return fail(c, CCH_E_INVALID_ARG, "integral pointer is NULL");
    if (!std::isfinite(e_core)) return fail(c, CCH_E_INPUT, "e_core is not finite");
    const int ni = c->n_irrep, no = c->n_o;
    // block offsets inside a record, record sizes per x, record offsets per pair
    std::vector<int64_t> blk((size_t)ni * ni), size((size_t)ni), rec((size_t)no * no + 1, 0);
    for (int x = 0; x < ni; ++x) {
        int64_t off = 0;
        for (int ca = 0; ca < ni; ++ca) {
            blk[(size_t)x * ni + ca] = off;
            off += (int64_t)c->n_c[ca] * c->n_c[ca ^ x];
        }
        size[x] = off;
    }
    for (int P = 0; P < no; ++P)
        for (int Q = 0; Q < no; ++Q)
            rec[(size_t)P * no + Q + 1] = rec[(size_t)P * no + Q] + size[c->tgt_irrep[P] ^ c->tgt_irrep[Q]];
    const size_t npk = (size_t)rec[(size_t)no * no];
    const size_t nc = c->n_cont, norb = c->n_orb;
    const size_t nh = norb * norb, n4 = (size_t)no * no * no * no, n3c = (size_t)no * no * no * nc;
    TRY(dalloc(c, &c->d_h, nh));
    TRY(dalloc(c, &c->d_tttt, n4));
    TRY(dalloc(c, &c->d_tttc, n3c));
    TRY(dalloc(c, &c->d_ttcc, npk));
    TRY(dalloc(c, &c->d_tctc, npk));
    TRY(dalloc(c, &c->d_pk_rec, rec.size()));
    TRY(copy_in(c, c->d_h, h, nh * 8, flags));
    TRY(copy_in(c, c->d_tttt, tttt, n4 * 8, flags));
    if (nc) {
        TRY(copy_in(c, c->d_tttc, tttc, n3c * 8, flags));
        TRY(copy_in(c, c->d_ttcc, ttcc, npk * 8, flags));
        TRY(copy_in(c, c->d_tctc, tctc, npk * 8, flags));
    }
    TRY(copy_in(c, c->d_pk_rec, rec.data(), rec.size() * 8, CCH_MEM_HOST));
    HIPCK(c, hipStreamSynchronize(c->stream));
    c->pk_blk = std::move(blk);
    c->packed = true;
    c->e_core = e_core;
    c->have_ints = true;
    return CCH_OK;
}

static cch_status check_dets(cch_ctx *c, const std::vector<uint64_t> &d, int n, int nelec, int na, int irrep,
                             const char *what, const int8_t *spin = nullptr)
{
    const int W = c->W, nso = 2 * c->n_o;
    for (int i = 0; i < n; ++i) {
        int ne = 0, nal = 0, ir = 0;
        for (int w = 0; w < W; ++w) {
            uint64_t x = d[(size_t)i * W + w];
            // bits beyond the target spin-orbitals
            const int lo = 64 * w;
            if (lo + 64 > nso) {
                const int keep = nso - lo;
                const uint64_t allowed = keep <= 0 ? 0ull : (keep >= 64 ? ~0ull : ((1ull << keep) - 1ull));
                if (x & ~allowed) return fail(c, CCH_E_INPUT, "%s det %d occupies a spin-orbital >= 2 n_o", what, i);
            }
            ne += popc64(x);
            nal += popc64(x & 0x5555555555555555ull);
            while (x) {
                const int k = lo + __builtin_ctzll(x);
                x &= x - 1;
                ir ^= c->tgt_irrep[k >> 1];
            }
        }
        if (ne != nelec) return fail(c, CCH_E_INPUT, "%s det %d has %d electrons, expected %d", what, i, ne, nelec);
        const int want = na + (spin ? spin[i] : 0);   // a beta continuum electron: one more alpha in the target
        if (nal != want)
            return fail(c, CCH_E_INPUT, "%s det %d has %d alpha electrons, expected %d", what, i, nal, want);
        if (ir != irrep) return fail(c, CCH_E_INPUT, "%s det %d has irrep %d, expected %d", what, i, ir, irrep);
    }
    // distinct
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    auto lt = [&](int a, int b) {
        for (int w = W - 1; w >= 0; --w) {
            const uint64_t x = d[(size_t)a * W + w], y = d[(size_t)b * W + w];
            if (x != y) return x < y;
        }
        return false;
    };
    std::sort(idx.begin(), idx.end(), lt);
    for (int i = 1; i < n; ++i)
        if (!lt(idx[i - 1], idx[i])) return fail(c, CCH_E_INPUT, "%s dets %d and %d are equal", what, idx[i - 1], idx[i]);
    return CCH_OK;
}

static cch_status add_symmetry(cch_ctx *c, int32_t irrep, int32_t n_det, int32_t n_words, const uint64_t *dets,
                               const int8_t *cont_spin, int32_t n_states, const double *ci, int32_t flags,
                               int32_t *sym_id)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->have_orb) return fail(c, CCH_E_STATE, "set orbitals first");
    if (c->planned) return fail(c, CCH_E_STATE, "already planned");
    if (irrep < 0 || irrep >= c->n_irrep) return fail(c, CCH_E_INVALID_ARG, "bad irrep");
    if (n_det <= 0 || !dets || !ci) return fail(c, CCH_E_INVALID_ARG, "empty symmetry");
    if (n_words != c->W) return fail(c, CCH_E_INPUT, "n_words %d != %d", n_words, c->W);
    if (n_states <= 0 || n_states > n_det) return fail(c, CCH_E_INVALID_ARG, "bad n_states");
    if (n_states > 256) return fail(c, CCH_E_LIMIT, "n_states > 256");
    std::vector<uint64_t> hd((size_t)n_det * n_words);
    TRY(host_copy(c, hd.data(), dets, hd.size() * 8, flags));
    std::vector<int8_t> hs;
    bool beta = false;
    if (cont_spin) {
        hs.resize((size_t)n_det);
        TRY(host_copy(c, hs.data(), cont_spin, hs.size(), flags));
        for (int m = 0; m < n_det; ++m) {
            if (hs[m] != 0 && hs[m] != 1)
                return fail(c, CCH_E_INPUT, "continuum spin of det %d is %d (0 alpha, 1 beta)", m, (int)hs[m]);
            beta |= hs[m] == 1;
        }
    }
    int nelec = 0;
    for (int w = 0; w < n_words; ++w) nelec += popc64(hd[w]);
    if (c->n_elec < 0) {
        if (nelec % 2) return fail(c, CCH_E_INPUT, "odd electron count %d (n_alpha = n_beta = N/2 required)", nelec);
        if (nelec + 1 > 64) return fail(c, CCH_E_LIMIT, "N + 1 > 64 electrons");
    } else if (nelec != c->n_elec) {
        return fail(c, CCH_E_INPUT, "det 0 has %d electrons, expected %d", nelec, c->n_elec);
    }
    TRY(check_dets(c, hd, n_det, nelec, nelec / 2, irrep, "target", beta ? hs.data() : nullptr));
    std::vector<double> hc((size_t)n_det * n_states);
    TRY(host_copy(c, hc.data(), ci, hc.size() * 8, flags));
    for (double v : hc)
        if (!std::isfinite(v)) return fail(c, CCH_E_INPUT, "CI coefficient is not finite");
    SymInfo s;
    s.irrep = irrep;
    s.M = n_det;
    s.S = n_states;
    TRY(dalloc(c, &s.d_dets, hd.size()));
    TRY(dalloc(c, &s.d_ci, hc.size()));
    HIPCK(c, hipMemcpy(s.d_dets, hd.data(), hd.size() * 8, hipMemcpyHostToDevice));
    HIPCK(c, hipMemcpy(s.d_ci, hc.data(), hc.size() * 8, hipMemcpyHostToDevice));
    if (beta) {
        TRY(dalloc(c, &s.d_cspin, hs.size()));
        HIPCK(c, hipMemcpy(s.d_cspin, hs.data(), hs.size(), hipMemcpyHostToDevice));
    }
    s.h_dets = std::move(hd);
    c->n_elec = nelec;
    c->syms.push_back(std::move(s));
    if (sym_id) *sym_id = (int32_t)c->syms.size() - 1;
    return CCH_OK;
}

cch_status cch_add_target_symmetry(cch_ctx *c, int32_t irrep, int32_t n_det, int32_t n_words, const uint64_t *dets,
                                   int32_t n_states, const double *ci, int32_t flags, int32_t *sym_id)
{
    return add_symmetry(c, irrep, n_det, n_words, dets, nullptr, n_states, ci, flags, sym_id);
}

cch_status cch_add_target_symmetry_spin(cch_ctx *c, int32_t irrep, int32_t n_det, int32_t n_words,
                                        const uint64_t *dets, const int8_t *cont_spin, int32_t n_states,
                                        const double *ci, int32_t flags, int32_t *sym_id)
{
    if (c && !cont_spin) return fail(c, CCH_E_INVALID_ARG, "no continuum spins");
    return add_symmetry(c, irrep, n_det, n_words, dets, cont_spin, n_states, ci, flags, sym_id);
}

cch_status cch_add_target_symmetry_csf(cch_ctx *c, int32_t irrep, int32_t n_csf, const int32_t *csf_start,
                                       int32_t n_words, const uint64_t *dets, const double *coef, int32_t n_states,
                                       const double *ci, int32_t flags, int32_t *sym_id)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->have_orb) return fail(c, CCH_E_STATE, "set orbitals first");
    if (c->planned) return fail(c, CCH_E_STATE, "already planned");
    if (n_csf <= 0 || !csf_start || !dets || !coef || !ci) return fail(c, CCH_E_INVALID_ARG, "empty CSF list");
    if (n_words != c->W) return fail(c, CCH_E_INPUT, "n_words %d != %d", n_words, c->W);
    if (n_states <= 0 || n_states > n_csf) return fail(c, CCH_E_INVALID_ARG, "bad n_states");
    std::vector<int32_t> st((size_t)n_csf + 1);
    TRY(host_copy(c, st.data(), csf_start, st.size() * 4, flags));
    if (st[0] != 0) return fail(c, CCH_E_INPUT, "csf_start[0] must be 0");
    for (int m = 0; m < n_csf; ++m)
        if (st[m + 1] <= st[m]) return fail(c, CCH_E_INPUT, "CSF %d has no determinant", m);
    const int64_t nt = st[n_csf];
    std::vector<uint64_t> hd((size_t)nt * n_words);
    std::vector<double> hc((size_t)nt), hci((size_t)n_csf * n_states);
    TRY(host_copy(c, hd.data(), dets, hd.size() * 8, flags));
    TRY(host_copy(c, hc.data(), coef, hc.size() * 8, flags));
    TRY(host_copy(c, hci.data(), ci, hci.size() * 8, flags));
    for (double v : hc)
        if (!std::isfinite(v)) return fail(c, CCH_E_INPUT, "CSF coefficient is not finite");
    for (double v : hci)
        if (!std::isfinite(v)) return fail(c, CCH_E_INPUT, "CI coefficient is not finite");
    // distinct determinants in order of first appearance; each state's
    // coefficient of a determinant sums coef * ci over its terms in input order
    std::map<std::vector<uint64_t>, int> index;
    std::vector<uint64_t> ud;
    std::vector<int> term_det((size_t)nt);
    for (int64_t t = 0; t < nt; ++t) {
        std::vector<uint64_t> key(hd.begin() + t * n_words, hd.begin() + (t + 1) * n_words);
        auto it = index.find(key);
        if (it == index.end()) {
            it = index.emplace(key, (int)index.size()).first;
            ud.insert(ud.end(), key.begin(), key.end());
        }
        term_det[t] = it->second;
    }
    const int nd = (int)index.size();
    std::vector<double> C((size_t)nd * n_states, 0.0);
    for (int m = 0; m < n_csf; ++m)
        for (int64_t t = st[m]; t < st[m + 1]; ++t)
            for (int n = 0; n < n_states; ++n)
                C[(size_t)term_det[t] * n_states + n] += hc[t] * hci[(size_t)m * n_states + n];
    return cch_add_target_symmetry(c, irrep, nd, n_words, ud.data(), n_states, C.data(), CCH_MEM_HOST, sym_id);
}

cch_status cch_set_l2(cch_ctx *c, int32_t n_l2, int32_t n_words, const uint64_t *dets, int32_t flags)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->have_orb) return fail(c, CCH_E_STATE, "set orbitals first");
    if (c->n_elec < 0) return fail(c, CCH_E_STATE, "add a target symmetry first (it fixes N)");
    if (c->planned) return fail(c, CCH_E_STATE, "already planned");
    if (n_l2 < 0 || (n_l2 > 0 && !dets)) return fail(c, CCH_E_INVALID_ARG, "bad L2 arguments");
    if (n_l2 > 0 && n_words != c->W) return fail(c, CCH_E_INPUT, "n_words %d != %d", n_words, c->W);
    std::vector<uint64_t> hd((size_t)n_l2 * c->W);
    if (n_l2) TRY(host_copy(c, hd.data(), dets, hd.size() * 8, flags));
    TRY(check_dets(c, hd, n_l2, c->n_elec + 1, c->n_elec / 2 + 1, c->total_irrep, "L2"));
    TRY(dalloc(c, &c->d_l2, hd.size()));
    if (n_l2) HIPCK(c, hipMemcpy(c->d_l2, hd.data(), hd.size() * 8, hipMemcpyHostToDevice));
    c->n_l2 = n_l2;
    c->n_l2r = n_l2;
    c->l2csf = false;
    c->h_l2 = std::move(hd);
    return CCH_OK;
}

cch_status cch_set_l2_csf(cch_ctx *c, int32_t n_csf, const int32_t *csf_start, int32_t n_words, const uint64_t *dets,
                          const double *coef, int32_t flags)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->have_orb) return fail(c, CCH_E_STATE, "set orbitals first");
    if (c->n_elec < 0) return fail(c, CCH_E_STATE, "add a target symmetry first (it fixes N)");
    if (c->planned) return fail(c, CCH_E_STATE, "already planned");
    if (n_csf <= 0 || !csf_start || !dets || !coef) return fail(c, CCH_E_INVALID_ARG, "empty CSF list");
    if (n_words != c->W) return fail(c, CCH_E_INPUT, "n_words %d != %d", n_words, c->W);
    std::vector<int32_t> st((size_t)n_csf + 1);
    TRY(host_copy(c, st.data(), csf_start, st.size() * 4, flags));
    if (st[0] != 0) return fail(c, CCH_E_INPUT, "csf_start[0] must be 0");
    for (int l = 0; l < n_csf; ++l)
        if (st[l + 1] <= st[l]) return fail(c, CCH_E_INPUT, "CSF %d has no determinant", l);
    const int64_t nt = st[n_csf];
    std::vector<uint64_t> hd((size_t)nt * n_words);
    std::vector<double> hc((size_t)nt);
    TRY(host_copy(c, hd.data(), dets, hd.size() * 8, flags));
    TRY(host_copy(c, hc.data(), coef, hc.size() * 8, flags));
    for (double v : hc)
        if (!std::isfinite(v)) return fail(c, CCH_E_INPUT, "CSF coefficient is not finite");
    // distinct determinants in order of first appearance
    std::map<std::vector<uint64_t>, int> index;
    std::vector<uint64_t> ud;
    std::vector<int32_t> term_det((size_t)nt);
    for (int64_t t = 0; t < nt; ++t) {
        std::vector<uint64_t> key(hd.begin() + t * n_words, hd.begin() + (t + 1) * n_words);
        auto it = index.find(key);
        if (it == index.end()) {
            it = index.emplace(key, (int)index.size()).first;
            ud.insert(ud.end(), key.begin(), key.end());
        }
        term_det[t] = it->second;
    }
    TRY(cch_set_l2(c, (int32_t)index.size(), n_words, ud.data(), CCH_MEM_HOST));
    c->n_l2r = n_csf;
    c->l2csf = true;
    c->h_csf_start = std::move(st);
    c->h_csf_det = std::move(term_det);
    c->h_csf_coef = std::move(hc);
    return CCH_OK;
}

cch_status cch_set_target_energies(cch_ctx *c, const double *E, int64_t n, int32_t flags)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (c->planned) return fail(c, CCH_E_STATE, "already planned");
    if (n == 0) {
        c->energy_mode = false;
        c->h_tgtE.clear();
        return CCH_OK;
    }
    if (n < 0 || !E) return fail(c, CCH_E_INVALID_ARG, "bad target energies");
    int64_t states = 0;
    for (const auto &s : c->syms) states += s.S;
    if (n != states)
        return fail(c, CCH_E_INPUT, "%lld target energies for %lld target states", (long long)n, (long long)states);
    std::vector<double> h((size_t)n);
    TRY(host_copy(c, h.data(), E, h.size() * 8, flags));
    for (double v : h)
        if (!std::isfinite(v)) return fail(c, CCH_E_INPUT, "target energy is not finite");
    c->h_tgtE = std::move(h);
    c->energy_mode = true;
    return CCH_OK;
}

static cch_status alloc_pairs(cch_ctx *c, DevPairs &p, int mode, const uint64_t *A, int nA, const uint64_t *B, int nB)
{
    TRY(dalloc(c, &p.row_off, nA));
    TRY(dalloc(c, &p.row_cnt, nA));
    int64_t *d_total = nullptr;
    TRY(dalloc(c, &d_total, 1));
    HIPCK(c, launch_scan(mode, c->W, A, nA, B, nB, 2 * c->n_o, nullptr, p.row_cnt, PairList{}, c->stream));
    HIPCK(c, launch_exclusive_scan(p.row_cnt, p.row_off, nA, d_total, c->stream));
    int64_t total = 0;
    HIPCK(c, hipMemcpyAsync(&total, d_total, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    p.n = total;
    TRY(dalloc(c, &p.pl.x, total));
    TRY(dalloc(c, &p.pl.y, total));
    TRY(dalloc(c, &p.pl.deg, total));
    TRY(dalloc(c, &p.pl.phase, total));
    TRY(dalloc(c, &p.pl.label, total));
    return CCH_OK;
}

template <class T>
static cch_status upload(cch_ctx *c, T **d, const std::vector<T> &h)
{
    TRY(dalloc(c, d, h.size()));
    if (!h.empty()) HIPCK(c, hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return CCH_OK;
}

cch_status cch_plan(cch_ctx *c, const cch_plan_opts *opts)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->have_ints) return fail(c, CCH_E_STATE, "set integrals first");
    if (c->syms.empty() && c->n_l2 == 0) return fail(c, CCH_E_STATE, "no basis functions");
    if (c->planned) return fail(c, CCH_E_STATE, "already planned");
    if (opts) {
        if (opts->precision != CCH_PREC_FP64 && opts->precision != CCH_PREC_FP32 &&
            opts->precision != CCH_PREC_SPLIT_BF16)
            return fail(c, CCH_E_INVALID_ARG, "unknown precision mode %d", opts->precision);
        if (opts->precision == CCH_PREC_SPLIT_BF16 && (opts->split_slices < 1 || opts->split_slices > 8))
            return fail(c, CCH_E_INVALID_ARG, "split_slices must be 1..8");
        if (opts->max_device_bytes < 0) return fail(c, CCH_E_INVALID_ARG, "negative memory budget");
        if (opts->flags & ~CCH_PLAN_SPARSE_L2) return fail(c, CCH_E_INVALID_ARG, "unknown plan flags %d", opts->flags);
        c->opts = *opts;
    }
    HIPCK(c, hipSetDevice(c->device));
    // rows
    int64_t row = 0;
    for (auto &s : c->syms) {
        const int a = s.irrep ^ c->total_irrep;
        s.nc = c->n_c[a];
        s.ja0 = c->cont_start[a];
        s.row0 = row;
        row += (int64_t)s.S * s.nc;
    }
    c->Dc = row;
    c->D = row + c->n_l2r;
    if (c->energy_mode) {
        int64_t off = 0;
        for (auto &s : c->syms) {
            s.e_off = off;
            off += s.S;
        }
        if (off != (int64_t)c->h_tgtE.size())
            return fail(c, CCH_E_STATE, "target energies cover %zu states, the symmetries hold %lld",
                        c->h_tgtE.size(), (long long)off);
        TRY(upload(c, &c->d_tgtE, c->h_tgtE));
    }
    if (c->D <= 0) return fail(c, CCH_E_STATE, "empty matrix");
    if (c->D > 2000000000LL) return fail(c, CCH_E_LIMIT, "dimension too large");
    c->sparse = (c->opts.flags & CCH_PLAN_SPARSE_L2) != 0;
    if (c->sparse && c->l2csf)
        return fail(c, CCH_E_STATE, "L2 functions given as CSFs need the dense L2 block (no CCH_PLAN_SPARSE_L2)");
    // dense: D x D; sparse L2 block: d_H keeps only the continuum columns
    c->ld = c->sparse ? std::max<int64_t>(32, (c->Dc + 31) / 32 * 32) : (c->D + 31) / 32 * 32;
    // symmetry pairs a >= b
    int64_t maxB = 0;
    for (int a = 0; a < (int)c->syms.size(); ++a) {
        for (int b = 0; b <= a; ++b) {
            PairPlan p;
            p.a = a;
            p.b = b;
            SymInfo &sa = c->syms[a], &sb = c->syms[b];
            TRY(alloc_pairs(c, p.pr, SCAN_TT, sa.d_dets, sa.M, sb.d_dets, sb.M));
            // label slots (P, Q) allowed by symmetry
            const int want = sa.irrep ^ sb.irrep;
            std::vector<int32_t> sP, sQ, pq((size_t)c->n_o * c->n_o, -1);
            for (int P = 0; P < c->n_o; ++P)
                for (int Q = 0; Q < c->n_o; ++Q)
                    if ((c->tgt_irrep[P] ^ c->tgt_irrep[Q]) == want) {
                        pq[(size_t)P * c->n_o + Q] = (int32_t)sP.size();
                        sP.push_back(P);
                        sQ.push_back(Q);
                    }
            p.n_slot = (int)sP.size();
            std::vector<int32_t> rn, rn2;
            for (int n = 0; n < sa.S; ++n)
                for (int n2 = 0; n2 < (a == b ? n + 1 : sb.S); ++n2) {
                    rn.push_back(n);
                    rn2.push_back(n2);
                }
            p.nrows = (int)rn.size();
            TRY(upload(c, &p.d_slotP, sP));
            TRY(upload(c, &p.d_slotQ, sQ));
            TRY(upload(c, &p.d_pqidx, pq));
            TRY(upload(c, &p.d_rn, rn));
            TRY(upload(c, &p.d_rn2, rn2));
            TRY(dalloc(c, &p.d_hv, p.pr.n));
            TRY(dalloc(c, &p.d_Y, (size_t)sa.M * sb.S));
            TRY(dalloc(c, &p.d_Yo, (size_t)sa.M * sb.S));
            TRY(dalloc(c, &p.d_HT, p.nrows));
            TRY(dalloc(c, &p.d_O, p.nrows));
            TRY(dalloc(c, &p.d_At, (size_t)2 * p.n_slot * p.nrows));
            TRY(dalloc(c, &p.d_key, p.pr.n));
            TRY(dalloc(c, &p.d_count, p.n_slot + 1));
            TRY(dalloc(c, &p.d_start, p.n_slot + 1));
            TRY(dalloc(c, &p.d_cursor, p.n_slot + 1));
            TRY(dalloc(c, &p.d_sorted, p.pr.n));
            TRY(dalloc(c, &p.d_tmp, p.pr.n));
            TRY(dalloc(c, &p.d_d0, sa.M));
            // FP64 integral rows are placed after everything else (below), where a
            // memory budget may split them into passes; the reduced-precision
            // operands are derived from a full copy
            if (c->opts.precision != CCH_PREC_FP64) TRY(dalloc(c, &p.d_B, (size_t)2 * p.n_slot * sa.nc * sb.nc));
            p.jj_chunk = sa.nc;
            maxB += (int64_t)2 * p.n_slot * sa.nc * sb.nc;
            {
                const size_t K = (size_t)2 * p.n_slot, N = (size_t)sa.nc * sb.nc;
                if (c->opts.precision == CCH_PREC_FP32) {
                    TRY(dalloc(c, &p.d_At32, K * p.nrows));
                    TRY(dalloc(c, &p.d_B32, K * N));
                } else if (c->opts.precision == CCH_PREC_SPLIT_BF16) {
                    const int sl = c->opts.split_slices;
                    p.ldk = (int)((K + 63) / 64 * 64);
                    if (p.ldk == 0) p.ldk = 64;
                    TRY(dalloc(c, &p.d_sigA, p.nrows));
                    TRY(dalloc(c, &p.d_sigB, N));
                    TRY(dalloc(c, &p.d_SA, (size_t)sl * p.nrows * p.ldk));
                    TRY(dalloc(c, &p.d_SB, (size_t)sl * N * p.ldk));
                }
            }
            c->pp.push_back(p);
        }
    }
    // L2 x target pairs per symmetry
    for (int s = 0; s < (int)c->syms.size() && c->n_l2 > 0; ++s) {
        LtPlan L;
        L.sym = s;
        TRY(alloc_pairs(c, L.pr, SCAN_LT, c->d_l2, c->n_l2, c->syms[s].d_dets, c->syms[s].M));
        c->lt.push_back(L);
    }
    c->relayout_elems = maxB;
    TRY(dalloc(c, &c->d_H, (size_t)c->D * c->ld));
    TRY(dalloc(c, &c->d_diag, c->D));
    c->d_Hb = c->d_H;
    c->ldb = c->ld;
    if (c->l2csf) {
        c->Dd = c->Dc + c->n_l2;
        c->ldd = (c->Dd + 31) / 32 * 32;
        TRY(dalloc(c, &c->d_Hd, (size_t)c->Dd * c->ldd));
        TRY(upload(c, &c->d_csf_start, c->h_csf_start));
        TRY(upload(c, &c->d_csf_det, c->h_csf_det));
        TRY(upload(c, &c->d_csf_coef, c->h_csf_coef));
        c->d_Hb = c->d_Hd;
        c->ldb = c->ldd;
    }
    if (c->sparse) {
        // transpose of class 4, and the L2 block's CSR sized by a counting pass
        // of the excitation scan over all L2 pairs (the columns are listed by
        // the build)
        c->ldr = std::max<int64_t>(32, ((int64_t)c->n_l2 + 31) / 32 * 32);
        TRY(dalloc(c, &c->d_R, (size_t)std::max<int64_t>(c->Dc, 1) * c->ldr));
        TRY(dalloc(c, &c->csr.off, (size_t)c->n_l2 + 1));
        int64_t *cnt = nullptr;
        TRY(dalloc(c, &cnt, std::max(c->n_l2, 1)));
        int64_t nnz = 0;
        if (c->n_l2 > 0) {
            HIPCK(c, launch_l2s_struct(c->W, c->d_l2, c->n_l2, nullptr, cnt, nullptr, c->stream));
            HIPCK(c, launch_exclusive_scan(cnt, c->csr.off, c->n_l2, c->csr.off + c->n_l2, c->stream));
            HIPCK(c, hipMemcpyAsync(&nnz, c->csr.off + c->n_l2, 8, hipMemcpyDeviceToHost, c->stream));
            HIPCK(c, hipStreamSynchronize(c->stream));
        }
        TRY(dalloc(c, &c->csr.col, std::max<int64_t>(nnz, 1)));
        TRY(dalloc(c, &c->csr.val, std::max<int64_t>(nnz, 1)));
        c->csr.nnz = c->csr.cap = nnz;
        c->csr.planned = true;
    }
    if (c->opts.precision == CCH_PREC_FP64) {
        const int64_t budget = c->opts.max_device_bytes;
        if (budget == 0 || c->bytes + 8 * maxB <= budget) {
            for (auto &p : c->pp)   // one pass: every pair keeps its integral rows
                TRY(dalloc(c, &p.d_B, (size_t)2 * p.n_slot * c->syms[p.a].nc * c->syms[p.b].nc));
        } else {
            // the budget left after everything else holds one shared buffer; each pair
            // relays and multiplies as many continuum rows j per pass as fit
            const int64_t left = (budget - c->bytes) / 8;
            int64_t need = 0;
            c->expansion_passes = 1;
            for (auto &p : c->pp) {
                const SymInfo &sa = c->syms[p.a], &sb = c->syms[p.b];
                const int64_t row = (int64_t)2 * p.n_slot * sb.nc;   // one j of B
                if (row == 0 || sa.nc == 0) continue;
                const int64_t fit = std::min<int64_t>(sa.nc, left / row);
                if (fit < 1)
                    return fail(c, CCH_E_OOM, "device budget of %lld bytes too small for one continuum orbital "
                                              "of the expansion", (long long)budget);
                p.jj_chunk = (int)fit;
                need = std::max(need, fit * row);
                c->expansion_passes = std::max(c->expansion_passes, (int)((sa.nc + fit - 1) / fit));
            }
            double *shared = nullptr;
            TRY(dalloc(c, &shared, (size_t)need));
            for (auto &p : c->pp) p.d_B = shared;
            c->b_shared = true;
        }
    }
    c->planned = true;
    return CCH_OK;
}

// ---------------------------------------------------------------------------
// build phases; `ev` records the phase events on the stream
// ---------------------------------------------------------------------------
#define EVREC(i)                                                 \
    do {                                                         \
        if (ev) HIPCK(c, hipEventRecord(c->ev[(i)], st));        \
    } while (0)

static Class4Args class4_args(cch_ctx *c, const LtPlan &L)
{
    const SymInfo &s = c->syms[L.sym];
    Class4Args a{};
    a.cspin = s.d_cspin;
    a.tdets = s.d_dets;
    a.ci = s.d_ci;
    a.S = s.S;
    a.h = c->d_h;
    a.tttc = c->d_tttc;
    a.n_o = c->n_o;
    a.n_orb = c->n_orb;
    a.n_cont = c->n_cont;
    a.ja0 = s.ja0;
    a.nc = s.nc;
    a.row_off = L.pr.row_off;
    a.row_cnt = L.pr.row_cnt;
    a.pl = L.pr.pl;
    a.H = c->d_Hb;
    a.ld = c->ldb;
    a.row_l2 = c->Dc;
    a.col0 = s.row0;
    a.pairs_per_chunk = std::max(1, std::min(64, 1024 / (1 + 2 * c->n_elec)));
    return a;
}

static ExpandEpi expand_epi(cch_ctx *c, const PairPlan &p)
{
    const SymInfo &sa = c->syms[p.a], &sb = c->syms[p.b];
    return ExpandEpi{c->d_Hb, c->ldb, sa.row0, sb.row0, sa.nc, sb.nc, sa.ja0, sb.ja0, p.d_rn, p.d_rn2, p.d_HT,
                     p.d_O, c->d_h, c->n_o, c->n_orb};
}

// Independent launches of one phase spread round-robin over the auxiliary
// streams: begin() makes them wait for what the stream has queued, end() makes
// the stream wait for all of them. Off (batch capture, no streams): all on st.
struct Fan {
    cch_ctx *c;
    hipStream_t st;
    bool on;
    hipError_t begin() const
    {
        if (!on) return hipSuccess;
        hipError_t e = hipEventRecord(c->fork_ev, st);
        for (int i = 0; i < CCH_NPAIRS_ST && e == hipSuccess; ++i) e = hipStreamWaitEvent(c->aux[i], c->fork_ev, 0);
        return e;
    }
    hipStream_t operator()(int i) const { return on ? c->aux[i % CCH_NPAIRS_ST] : st; }
    hipError_t end() const
    {
        if (!on) return hipSuccess;
        hipError_t e = hipSuccess;
        for (int i = 0; i < CCH_NPAIRS_ST && e == hipSuccess; ++i) {
            e = hipEventRecord(c->join_ev[i], c->aux[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, c->join_ev[i], 0);
        }
        return e;
    }
};

// where the integral rows of a symmetry pair's relayout start in the packed
// layout (continuum rows from j0 of the first symmetry's range)
static PackedCC packed_cc(const cch_ctx *c, const PairPlan &p, int j0)
{
    PackedCC pk{};
    if (!c->packed) return pk;
    const SymInfo &sa = c->syms[p.a], &sb = c->syms[p.b];
    const int ca = sa.irrep ^ c->total_irrep, cb = sb.irrep ^ c->total_irrep, x = ca ^ cb;
    pk.rec = c->d_pk_rec;
    pk.boffJ = c->pk_blk[(size_t)x * c->n_irrep + ca] + (int64_t)j0 * sb.nc;
    pk.boffK = c->pk_blk[(size_t)x * c->n_irrep + cb];
    pk.jr0 = j0;
    pk.nca_full = sa.nc;
    return pk;
}

// phases 0-2: scans, target elements and densities, relayout; every symmetry
// pair (and L2-target group) writes only its own buffers, so with `fan` they
// run on the auxiliary streams side by side
static cch_status enqueue_pre(cch_ctx *c, hipStream_t st, bool ev, bool fan, bool lt_scans = true)
{
    const TgtInts I{c->d_h, c->d_tttt, c->n_o, c->n_orb, c->e_core};
    const Fan f{c, st, fan && c->have_aux};
    EVREC(0);
    HIPCK(c, f.begin());
    int w = 0;
    for (auto &p : c->pp) {
        SymInfo &sa = c->syms[p.a], &sb = c->syms[p.b];
        HIPCK(c, launch_scan(SCAN_TT, c->W, sa.d_dets, sa.M, sb.d_dets, sb.M, 2 * c->n_o, p.pr.row_off,
                             p.pr.row_cnt, p.pr.pl, f(w++)));
    }
    for (auto &L : c->lt) {
        if (!lt_scans) break;
        SymInfo &s = c->syms[L.sym];
        HIPCK(c, launch_scan(SCAN_LT, c->W, c->d_l2, c->n_l2, s.d_dets, s.M, 2 * c->n_o, L.pr.row_off,
                             L.pr.row_cnt, L.pr.pl, f(w++)));
    }
    HIPCK(c, f.end());
    EVREC(1);
    HIPCK(c, f.begin());
    w = 0;
    for (auto &p : c->pp) {
        SymInfo &sa = c->syms[p.a], &sb = c->syms[p.b];
        const hipStream_t s = f(w++);
        HIPCK(c, launch_pair_values(c->W, I, sa.d_dets, sb.d_dets, p.pr.pl, p.pr.n, p.d_hv, s));
        HIPCK(c, launch_projection(sa.M, p.pr.row_off, p.pr.row_cnt, p.pr.pl, p.d_hv, sa.d_ci, sa.S, sb.d_ci, sb.S,
                                   p.nrows, p.d_rn, p.d_rn2, p.d_Y, p.d_Yo, p.d_HT, p.d_O, s));
        if (c->energy_mode)
            HIPCK(c, launch_energy_rows(p.nrows, p.d_rn, p.d_rn2, p.a == p.b ? c->d_tgtE + sa.e_off : nullptr,
                                        p.d_HT, s));
        HIPCK(c, launch_bucket(p.pr.pl, p.pr.n, p.d_pqidx, c->n_o, p.n_slot, sa.M, p.d_key, p.d_count, p.d_start,
                               p.d_cursor, p.d_sorted, p.d_tmp, p.d_d0, s));
        const int M0 = (sa.irrep == sb.irrep) ? sa.M : 0;
        HIPCK(c, launch_gamma(c->W, p.pr.pl, p.d_start, p.d_count, p.d_sorted, p.d_d0, M0, p.d_slotP, p.d_slotQ,
                              p.n_slot, sa.d_dets, sa.d_cspin, sb.d_cspin, sa.d_ci, sa.S, sb.d_ci, sb.S, p.nrows,
                              p.d_rn, p.d_rn2, p.d_At, s));
    }
    HIPCK(c, f.end());
    EVREC(2);
    HIPCK(c, f.begin());
    w = 0;
    for (auto &p : c->pp) {
        SymInfo &sa = c->syms[p.a], &sb = c->syms[p.b];
        if (sa.nc == 0 || sb.nc == 0) continue;
        if (c->b_shared) continue;   // one shared buffer: rows are laid out pass by pass in phase 3
        const hipStream_t s = f(w++);
        const PackedCC pk = packed_cc(c, p, 0);
        HIPCK(c, launch_relayout(c->d_ttcc, c->d_tctc, c->n_o, c->n_cont, p.d_slotP, p.d_slotQ, p.n_slot, sa.ja0,
                                 sa.nc, sb.ja0, sb.nc, p.d_B, s, c->packed ? &pk : nullptr));
        const int K = 2 * p.n_slot, N = sa.nc * sb.nc;
        if (c->opts.precision == CCH_PREC_FP32) {
            HIPCK(c, launch_to_f32(p.d_At, p.d_At32, (int64_t)K * p.nrows, s));
            HIPCK(c, launch_to_f32(p.d_B, p.d_B32, (int64_t)K * N, s));
        } else if (c->opts.precision == CCH_PREC_SPLIT_BF16) {
            HIPCK(c, launch_slices(p.d_At, p.nrows, p.d_B, K, N, c->opts.split_slices, p.ldk, p.d_sigA, p.d_SA,
                                   p.d_sigB, p.d_SB, s));
        }
    }
    HIPCK(c, f.end());
    EVREC(3);
    return CCH_OK;
}

// phase 3: expansion product per symmetry pair
static cch_status enqueue_gemm(cch_ctx *c, hipStream_t st, bool fan)
{
    // one product per pair, side by side (not with the shared integral buffer,
    // which the pairs use one after another)
    const Fan f{c, st, fan && c->have_aux && !c->b_shared};
    HIPCK(c, f.begin());
    int w = 0;
    for (auto &p : c->pp) {
        SymInfo &sa = c->syms[p.a], &sb = c->syms[p.b];
        if (sa.nc == 0 || sb.nc == 0) continue;
        const ExpandEpi ep = expand_epi(c, p);
        const int K = 2 * p.n_slot, N = sa.nc * sb.nc;
        const hipStream_t s = f(w++);
        if (c->opts.precision == CCH_PREC_FP32)
            HIPCK(c, launch_expand_f32(p.d_At32, p.d_B32, p.nrows, N, K, ep, s));
        else if (c->opts.precision == CCH_PREC_SPLIT_BF16)
            HIPCK(c, launch_expand_bf16split(p.d_SA, p.d_SB, p.d_sigA, p.d_sigB, c->opts.split_slices, p.nrows, N,
                                             p.ldk, ep, s));
        else if (!c->b_shared)
            HIPCK(c, launch_expand_f64(p.d_At, p.d_B, p.nrows, N, K, ep, s));
        else {
            // passes over ranges of j: the rows j0..j0+nj-1 of the integral layout, then
            // the product's columns (j, j') of those rows; each output keeps its sum over K
            for (int j0 = 0; j0 < sa.nc; j0 += p.jj_chunk) {
                const int nj = std::min(p.jj_chunk, sa.nc - j0);
                const PackedCC pk = packed_cc(c, p, j0);
                HIPCK(c, launch_relayout(c->d_ttcc, c->d_tctc, c->n_o, c->n_cont, p.d_slotP, p.d_slotQ, p.n_slot,
                                         sa.ja0 + j0, nj, sb.ja0, sb.nc, p.d_B, st, c->packed ? &pk : nullptr));
                ExpandEpi e2 = ep;
                e2.row0a += j0;
                e2.ja0 += j0;
                HIPCK(c, launch_expand_f64(p.d_At, p.d_B, p.nrows, nj * sb.nc, K, e2, st));
            }
        }
    }
    HIPCK(c, f.end());
    return CCH_OK;
}

static cch_status enqueue_class4(cch_ctx *c, hipStream_t st, bool fan)
{
    const Fan f{c, st, fan && c->have_aux};
    HIPCK(c, f.begin());
    int w = 0;
    for (auto &L : c->lt) HIPCK(c, launch_class4(c->W, class4_args(c, L), c->n_l2, f(w++)));
    HIPCK(c, f.end());
    return CCH_OK;
}

static cch_status enqueue_l2(cch_ctx *c, hipStream_t st)
{
    if (c->n_l2 > 0) {
        const TgtInts I{c->d_h, c->d_tttt, c->n_o, c->n_orb, c->e_core};
        if (c->sparse) {
            // column lists of the L2 rows, then the values (and the L2 part of the diagonal)
            HIPCK(c, launch_l2s_struct(c->W, c->d_l2, c->n_l2, c->csr.off, nullptr, c->csr.col, st));
            HIPCK(c, launch_l2s_values(c->W, c->d_l2, c->n_l2, I, c->csr.off, c->csr.col, c->csr.val,
                                       c->d_diag + c->Dc, st));
        } else {
            L2Args a{c->d_l2, c->n_l2, I, c->d_Hb, c->ldb, c->Dc};
            HIPCK(c, launch_l2_block(c->W, a, st));
        }
    }
    return CCH_OK;
}

static cch_status enqueue_post(cch_ctx *c, hipStream_t st)
{
    if (c->sparse) {
        // upper triangle of the continuum block, its diagonal, and the transpose of class 4
        HIPCK(c, launch_mirror(c->d_H, c->ld, (int)c->Dc, st));
        HIPCK(c, launch_diag(c->d_H, c->ld, (int)c->Dc, c->d_diag, st));
        HIPCK(c, launch_transpose_c4(c->d_H, c->ld, (int)c->Dc, c->n_l2, c->d_R, c->ldr, st));
        return CCH_OK;
    }
    if (c->l2csf)   // the matrix over the CSFs (lower triangle) from the one over the determinants
        HIPCK(c, launch_l2csf_gather(c->d_Hd, c->ldd, (int)c->Dc, c->n_l2r, c->d_csf_start, c->d_csf_det,
                                     c->d_csf_coef, c->d_H, c->ld, st));
    HIPCK(c, launch_mirror(c->d_H, c->ld, (int)c->D, st));
    HIPCK(c, launch_diag(c->d_H, c->ld, (int)c->D, c->d_diag, st));
    return CCH_OK;
}

static SparseMat sparse_mat(const cch_ctx *c)
{
    return SparseMat{c->d_H, c->ld, c->d_R, c->ldr, c->csr.off, c->csr.col, c->csr.val, c->Dc};
}

cch_status cch_build(cch_ctx *c)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->planned) return fail(c, CCH_E_STATE, "plan first");
    HIPCK(c, hipSetDevice(c->device));
    hipStream_t st = c->stream;
    const bool ev = true;
    // the streams pay from a few thousand rows on; below that the event
    // traffic of the fork and join costs more than the overlap saves
    c->overlapped = c->have_aux && c->D >= 4096;
    if (c->overlapped) {
        // class 4 (with its L2 x target scans) and the L2 block depend on no pair
        // phase and write their own blocks of H: each on a stream of its own
        // from the start, joined before the mirror
        EVREC(0);
        HIPCK(c, hipEventRecord(c->fork_ev, st));
        hipStream_t s4 = c->aux[CCH_NPAIRS_ST], sl = c->aux[CCH_NPAIRS_ST + 1];
        HIPCK(c, hipStreamWaitEvent(s4, c->fork_ev, 0));
        HIPCK(c, hipStreamWaitEvent(sl, c->fork_ev, 0));
        HIPCK(c, hipEventRecord(c->l2_ev[0], sl));
        TRY(enqueue_l2(c, sl));
        HIPCK(c, hipEventRecord(c->l2_ev[1], sl));
        HIPCK(c, hipEventRecord(c->c4_ev[0], s4));
        for (auto &L : c->lt) {
            SymInfo &s = c->syms[L.sym];
            HIPCK(c, launch_scan(SCAN_LT, c->W, c->d_l2, c->n_l2, s.d_dets, s.M, 2 * c->n_o, L.pr.row_off,
                                 L.pr.row_cnt, L.pr.pl, s4));
        }
        TRY(enqueue_class4(c, s4, false));
        HIPCK(c, hipEventRecord(c->c4_ev[1], s4));
        TRY(enqueue_pre(c, st, ev, true, false));
        TRY(enqueue_gemm(c, st, true));
        EVREC(4);
        HIPCK(c, hipEventRecord(c->join_ev[CCH_NPAIRS_ST], s4));
        HIPCK(c, hipStreamWaitEvent(st, c->join_ev[CCH_NPAIRS_ST], 0));
        EVREC(5);
        HIPCK(c, hipEventRecord(c->join_ev[CCH_NPAIRS_ST + 1], sl));
        HIPCK(c, hipStreamWaitEvent(st, c->join_ev[CCH_NPAIRS_ST + 1], 0));
        EVREC(6);
    } else {
        TRY(enqueue_pre(c, st, ev, false));
        TRY(enqueue_gemm(c, st, false));
        EVREC(4);
        TRY(enqueue_class4(c, st, false));
        EVREC(5);
        TRY(enqueue_l2(c, st));
        EVREC(6);
    }
    TRY(enqueue_post(c, st));
    EVREC(7);
    c->built = true;
    ++c->build_gen;
    if (c->sparse) c->csr.gen = c->build_gen;   // the build wrote the CSR itself
    c->timed = true;
    return CCH_OK;
}

cch_status cch_build_time(cch_ctx *c, float *total_ms, float *phases)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->built || !c->timed) return fail(c, CCH_E_STATE, "no timed build (cch_build) yet");
    HIPCK(c, hipEventSynchronize(c->ev[7]));
    if (total_ms) HIPCK(c, hipEventElapsedTime(total_ms, c->ev[0], c->ev[7]));
    if (phases) {
        for (int i = 0; i < 7; ++i) HIPCK(c, hipEventElapsedTime(&phases[i], c->ev[i], c->ev[i + 1]));
        if (c->overlapped) {   // class 4 and the L2 block on their own streams, beside phases 0-3
            HIPCK(c, hipEventElapsedTime(&phases[4], c->c4_ev[0], c->c4_ev[1]));
            HIPCK(c, hipEventElapsedTime(&phases[5], c->l2_ev[0], c->l2_ev[1]));
        }
        phases[7] = 0.0f;
    }
    return CCH_OK;
}

cch_status cch_plan_info(cch_ctx *c, int64_t *device_bytes, int32_t *expansion_passes)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->planned) return fail(c, CCH_E_STATE, "plan first");
    if (device_bytes) *device_bytes = c->bytes;
    if (expansion_passes) *expansion_passes = c->expansion_passes;
    return CCH_OK;
}

cch_status cch_work_counts(const cch_ctx *c, double *out)
{
    if (!c || !out) return CCH_E_INVALID_ARG;
    if (!c->planned) return CCH_E_STATE;
    double gemm = 0.0, tp = 0.0, ltp = 0.0, c4 = 0.0;
    for (auto &p : c->pp) {
        const SymInfo &sa = c->syms[p.a], &sb = c->syms[p.b];
        gemm += 2.0 * p.nrows * (double)sa.nc * sb.nc * (2.0 * p.n_slot);
        tp += (double)p.pr.n;
    }
    for (auto &L : c->lt) ltp += (double)L.pr.n;
    for (auto &s : c->syms) c4 += (double)c->n_l2 * s.S * s.nc;
    // lower-triangle elements: every element of the dense parts; of a sparse
    // L2 block its structural non-zeros (the CSR holds both triangles)
    const double l2_lower = c->sparse ? ((double)c->csr.nnz + c->n_l2) / 2.0
                                      : (double)c->n_l2 * (c->n_l2 + 1) / 2.0;
    out[0] = c->sparse ? (double)c->Dc * (c->Dc + 1) / 2.0 + (double)c->n_l2 * c->Dc + l2_lower
                       : (double)c->D * (c->D + 1) / 2.0;
    out[1] = gemm;
    out[2] = tp;
    out[3] = ltp;
    out[4] = 16.0 * (double)c->relayout_elems;
    out[5] = c4;
    out[6] = l2_lower;
    out[7] = (double)c->pp.size();
    return CCH_OK;
}

cch_status cch_target_hamiltonian(cch_ctx *c, int32_t sym_a, int32_t sym_b, double *out, int64_t ld, int32_t flags)
{
    if (!c || !out) return CCH_E_INVALID_ARG;
    if (!c->built) return fail(c, CCH_E_STATE, "build first");
    const int ns = (int)c->syms.size();
    if (sym_a < 0 || sym_a >= ns || sym_b < 0 || sym_b >= ns) return fail(c, CCH_E_INVALID_ARG, "bad symmetry");
    const int ma = c->syms[sym_a].M, mb = c->syms[sym_b].M;
    if (ld < mb) return fail(c, CCH_E_INVALID_ARG, "ld %lld below %d columns", (long long)ld, mb);
    // the pair list of (max, min): its values are <det of the larger index|H|det of the smaller>
    const int hi = std::max(sym_a, sym_b), lo = std::min(sym_a, sym_b);
    const PairPlan *pp = nullptr;
    for (auto &p : c->pp)
        if (p.a == hi && p.b == lo) pp = &p;
    if (!pp) return fail(c, CCH_E_STATE, "no pair list for symmetries %d, %d", hi, lo);
    HIPCK(c, hipSetDevice(c->device));
    const bool dev = flags & CCH_MEM_DEVICE;
    double *d = out;
    int64_t ldo = ld;
    if (!dev) {
        ldo = mb;
        if (hipMalloc((void **)&d, 8 * (size_t)std::max(1, ma) * std::max(1, mb)) != hipSuccess)
            return fail(c, CCH_E_OOM, "target Hamiltonian staging");
    }
    hipError_t e = hipSuccess;
    if (ldo == mb) e = launch_fill_f64(d, 0.0, (int64_t)ma * mb, c->stream);
    else
        for (int r = 0; r < ma && e == hipSuccess; ++r) e = launch_fill_f64(d + (int64_t)r * ldo, 0.0, mb, c->stream);
    if (e == hipSuccess)
        e = launch_scatter_pairs(pp->pr.pl.x, pp->pr.pl.y, pp->d_hv, pp->pr.n, sym_a < sym_b ? 1 : 0, d, ldo,
                                 c->stream);
    if (e == hipSuccess && !dev)
        e = hipMemcpy2DAsync(out, 8 * ld, d, 8 * ldo, 8 * (size_t)mb, ma, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (!dev) (void)hipFree(d);
    if (e != hipSuccess) return fail(c, CCH_E_HIP, "cch_target_hamiltonian: %s", hipGetErrorString(e));
    return CCH_OK;
}

cch_status cch_work_detail(cch_ctx *c, double *out, int32_t n)
{
    if (!c || (n > 0 && !out) || n < 0) return CCH_E_INVALID_ARG;
    if (!c->built) return fail(c, CCH_E_STATE, "build first");
    double v[16] = {};
    TRY(cch_work_counts(c, v));
    HIPCK(c, hipSetDevice(c->device));
    HIPCK(c, hipStreamSynchronize(c->stream));
    std::vector<void *> tmp;
    auto cleanup = [&]() { for (void *p : tmp) (void)hipFree(p); };
    auto galloc = [&](void **p, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(p, bytes ? bytes : 8);
        if (e == hipSuccess) tmp.push_back(*p);
        return e;
    };
    unsigned long long *cnt = nullptr;
    hipError_t e = galloc((void **)&cnt, 4 * sizeof(unsigned long long));
    double pairs01 = 0.0, gamma = 0.0;
    const double ne = c->n_elec;
    for (auto &p : c->pp) {
        if (e != hipSuccess) break;
        unsigned long long h[4] = {};
        e = launch_pair_census(p.pr.pl.deg, p.pr.pl.label, p.pr.n, cnt, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        pairs01 += (double)(h[0] + h[1] + h[2]);
        // density updates per pair: degree 0 adds every occupied spin-orbital to
        // the spin-summed diagonal and the alpha ones to the alpha-resolved one
        // (1.5 N); an alpha excitation feeds both densities (2), a beta one the
        // spin-summed density only (1); each update is one multiply-add per row
        gamma += 2.0 * p.nrows * (1.5 * ne * (double)h[0] + 2.0 * (double)h[1] + (double)h[2]);
    }
    double c4 = 0.0;
    for (auto &L : c->lt) {
        const SymInfo &s = c->syms[L.sym];
        c4 += 2.0 * s.S * (double)s.nc * (double)L.pr.n;
    }
    double l2pairs = 0.0;
    if (e == hipSuccess && c->n_l2 > 0) {
        int64_t *rc = nullptr, *ro = nullptr, *tot = nullptr, h = 0;
        e = galloc((void **)&rc, 8 * (size_t)c->n_l2);
        if (e == hipSuccess) e = galloc((void **)&ro, 8 * (size_t)c->n_l2);
        if (e == hipSuccess) e = galloc((void **)&tot, 8);
        if (e == hipSuccess)
            e = launch_scan(SCAN_LL, c->W, c->d_l2, c->n_l2, c->d_l2, c->n_l2, 2 * c->n_o, nullptr, rc, PairList{},
                            c->stream);
        if (e == hipSuccess) e = launch_exclusive_scan(rc, ro, c->n_l2, tot, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&h, tot, 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        l2pairs = (double)h;
    }
    cleanup();
    if (e != hipSuccess) return fail(c, CCH_E_HIP, "cch_work_detail: %s", hipGetErrorString(e));
    v[8] = pairs01;
    v[9] = gamma;
    v[10] = c4;
    v[11] = l2pairs;
    // mirror: 16 bytes per element above the diagonal of the dense parts (a
    // sparse L2 block also writes the transpose of class 4)
    v[12] = c->sparse ? 16.0 * (double)c->Dc * (double)(c->Dc - 1) / 2.0 + 16.0 * (double)c->Dc * c->n_l2
                      : 16.0 * (double)c->D * (double)(c->D - 1) / 2.0;
    for (int i = 0; i < n && i < 16; ++i) out[i] = v[i];
    for (int i = 16; i < n; ++i) out[i] = 0.0;
    return CCH_OK;
}

cch_status cch_get_dim(const cch_ctx *c, int64_t *D, int64_t *n_cont_rows)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (!c->planned) return CCH_E_STATE;
    if (D) *D = c->D;
    if (n_cont_rows) *n_cont_rows = c->Dc;
    return CCH_OK;
}

cch_status cch_get_matrix(cch_ctx *c, double *out, int64_t ld, int32_t flags)
{
    if (!c || !out) return CCH_E_INVALID_ARG;
    if (!c->built) return fail(c, CCH_E_STATE, "build first");
    if (ld < c->D) return fail(c, CCH_E_INVALID_ARG, "ld < D");
    const bool to_dev = flags & CCH_MEM_DEVICE, lower = flags & CCH_LOWER;
    const hipMemcpyKind kind = to_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    // row blocks of at most 1 GiB; with CCH_LOWER each block stops at its last
    // row's diagonal (the rectangle holding the block's lower-triangle part)
    const int64_t D = c->D, rows_per = std::max<int64_t>(1, (int64_t(1) << 30) / (8 * D));
    HIPCK(c, hipSetDevice(c->device));
    if (c->sparse) {
        // rows expanded from the panels and the CSR, block by block (into the
        // caller's device array, or through a staging block for host output)
        const SparseMat S = sparse_mat(c);
        double *stage = nullptr;
        if (!to_dev && hipMalloc((void **)&stage, 8 * (size_t)rows_per * D) != hipSuccess)
            return fail(c, CCH_E_OOM, "read-out staging block");
        hipError_t e = hipSuccess;
        for (int64_t r0 = 0; r0 < D && e == hipSuccess; r0 += rows_per) {
            const int64_t nr = std::min(rows_per, D - r0), width = lower ? r0 + nr : D;
            if (to_dev) {
                e = launch_sparse_rows(S, r0, (int)nr, 0, (int)width, 0, out + r0 * ld, ld, c->stream);
            } else {
                e = launch_sparse_rows(S, r0, (int)nr, 0, (int)width, 0, stage, width, c->stream);
                if (e == hipSuccess)
                    e = hipMemcpy2DAsync(out + r0 * ld, ld * 8, stage, width * 8, width * 8, nr, kind, c->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);   // the staging block is reused
            }
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        (void)hipFree(stage);
        if (e != hipSuccess) return fail(c, CCH_E_HIP, "cch_get_matrix: %s", hipGetErrorString(e));
    } else {
        for (int64_t r0 = 0; r0 < D; r0 += rows_per) {
            const int64_t nr = std::min(rows_per, D - r0), width = lower ? r0 + nr : D;
            HIPCK(c, hipMemcpy2DAsync(out + r0 * ld, ld * 8, c->d_H + r0 * c->ld, c->ld * 8, width * 8, nr, kind,
                                      c->stream));
        }
        HIPCK(c, hipStreamSynchronize(c->stream));
    }
    if (!to_dev) {
        // read-back check: the copied diagonal must equal the device diagonal
        // (a copy that silently delivered other bytes is reported, not returned)
        std::vector<double> dg((size_t)D);
        HIPCK(c, hipMemcpy(dg.data(), c->d_diag, 8 * (size_t)D, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < D; ++i) {
            const double v = out[i * ld + i];
            if (std::memcmp(&v, &dg[(size_t)i], 8) != 0)
                return fail(c, CCH_E_HIP, "read-back check failed: copied H[%lld][%lld] = %.17g, device diagonal %.17g",
                            (long long)i, (long long)i, v, dg[(size_t)i]);
        }
    }
    return CCH_OK;
}

cch_status cch_matrix_device(cch_ctx *c, const double **dptr, int64_t *ld)
{
    if (!c || !dptr || !ld) return CCH_E_INVALID_ARG;
    if (!c->planned) return fail(c, CCH_E_STATE, "plan first");
    if (c->sparse) return fail(c, CCH_E_STATE, "the L2 block is stored as CSR (CCH_PLAN_SPARSE_L2): no dense matrix");
    *dptr = c->d_H;
    *ld = c->ld;
    return CCH_OK;
}

cch_status cch_get_diagonal(cch_ctx *c, double *out, int32_t flags)
{
    if (!c || !out) return CCH_E_INVALID_ARG;
    if (!c->built) return fail(c, CCH_E_STATE, "build first");
    HIPCK(c, hipMemcpyAsync(out, c->d_diag, c->D * 8,
                            (flags & CCH_MEM_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIPCK(c, hipStreamSynchronize(c->stream));
    return CCH_OK;
}

cch_status cch_apply(cch_ctx *c, const double *V, int64_t ldv, int32_t b, double *W, int64_t ldw, int32_t flags)
{
    if (!c || b < 0 || (b > 0 && (!V || !W))) return CCH_E_INVALID_ARG;
    if (!c->built) return fail(c, CCH_E_STATE, "build first");
    const int64_t D = c->D;
    if (b == 0 || D == 0) return CCH_OK;
    if (ldv < D || ldw < D) return fail(c, CCH_E_INVALID_ARG, "leading dimensions %lld, %lld below D = %lld",
                                        (long long)ldv, (long long)ldw, (long long)D);
    const bool dev = flags & CCH_MEM_DEVICE;
    const int64_t lv = dev ? ldv : D, lw = dev ? ldw : D;
    const int64_t nscr = c->sparse ? l2csr_scratch((int)D, (int)c->Dc) : matvec_scratch_doubles((int)D);
    double *dV = dev ? const_cast<double *>(V) : nullptr, *dW = dev ? W : nullptr, *Wp = nullptr;
    hipError_t e = hipMalloc((void **)&Wp, 8 * (size_t)std::max<int64_t>(nscr, 1));
    if (e == hipSuccess && !dev) e = hipMalloc((void **)&dV, 8 * (size_t)(D * b));
    if (e == hipSuccess && !dev) e = hipMalloc((void **)&dW, 8 * (size_t)(D * b));
    if (e == hipSuccess && !dev)
        e = hipMemcpy2DAsync(dV, 8 * D, V, 8 * ldv, 8 * D, b, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = c->sparse ? launch_matvec_l2csr(c->d_H, c->ld, c->d_R, c->ldr, (int)c->Dc, (int)D, (int)c->Dc, c->csr.off,
                                            c->csr.col, c->csr.val, dV, lv, b, dW, lw, Wp, c->stream)
                      : launch_matvec(c->d_H, c->ld, (int)D, dV, lv, b, dW, lw, Wp, c->stream);
    if (e == hipSuccess && !dev)
        e = hipMemcpy2DAsync(W, 8 * ldw, dW, 8 * D, 8 * D, b, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(Wp);
    if (!dev) {
        (void)hipFree(dV);
        (void)hipFree(dW);
    }
    if (e != hipSuccess) return fail(c, CCH_E_HIP, "cch_apply: %s", hipGetErrorString(e));
    return CCH_OK;
}

cch_status cch_get_elements(cch_ctx *c, int64_t n, const int64_t *rows, const int64_t *cols, double *out,
                            int32_t flags)
{
    if (!c || n < 0 || (n > 0 && (!rows || !cols || !out))) return CCH_E_INVALID_ARG;
    if (!c->built) return fail(c, CCH_E_STATE, "build first");
    if (n == 0) return CCH_OK;
    std::vector<int64_t> hr((size_t)n), hc((size_t)n);
    TRY(host_copy(c, hr.data(), rows, hr.size() * 8, flags));
    TRY(host_copy(c, hc.data(), cols, hc.size() * 8, flags));
    for (int64_t i = 0; i < n; ++i)
        if (hr[i] < 0 || hr[i] >= c->D || hc[i] < 0 || hc[i] >= c->D)
            return fail(c, CCH_E_INVALID_ARG, "element %lld: index (%lld, %lld) outside [0, %lld)", (long long)i,
                        (long long)hr[i], (long long)hc[i], (long long)c->D);
    int64_t *d_idx = nullptr;
    double *d_out = nullptr;
    hipError_t e = hipMalloc((void **)&d_idx, 16 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc((void **)&d_out, 8 * (size_t)n);
    if (e == hipSuccess) e = hipMemcpyAsync(d_idx, hr.data(), 8 * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_idx + n, hc.data(), 8 * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = c->sparse ? launch_sparse_gather(sparse_mat(c), d_idx, d_idx + n, n, d_out, c->stream)
                      : launch_gather_elements(c->d_H, c->ld, d_idx, d_idx + n, n, d_out, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, d_out, 8 * (size_t)n,
                           (flags & CCH_MEM_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d_idx);
    (void)hipFree(d_out);
    if (e != hipSuccess) return fail(c, CCH_E_HIP, "cch_get_elements: %s", hipGetErrorString(e));
    return CCH_OK;
}

// the rectangle of a class block and its element filter (see cch_get_block)
static cch_status block_geometry(cch_ctx *c, int32_t cls, int32_t sym_a, int32_t sym_b, int64_t *row0, int64_t *nrows,
                                 int64_t *col0, int64_t *ncols, int *mode, int *nca, int *ncb)
{
    const int ns = (int)c->syms.size();
    *nca = *ncb = 0;
    if (cls == 2 || cls == 8) {
        *row0 = *col0 = c->Dc;
        *nrows = *ncols = c->n_l2r;
        *mode = cls;
        return CCH_OK;
    }
    if (sym_a < 0 || sym_a >= ns) return fail(c, CCH_E_INVALID_ARG, "symmetry %d out of range", sym_a);
    const SymInfo &sa = c->syms[sym_a];
    if (cls == 4) {
        *row0 = c->Dc;
        *nrows = c->n_l2r;
        *col0 = sa.row0;
        *ncols = (int64_t)sa.S * sa.nc;
        *mode = 0;
        return CCH_OK;
    }
    if (sym_b < 0 || sym_b >= ns) return fail(c, CCH_E_INVALID_ARG, "symmetry %d out of range", sym_b);
    const SymInfo &sb = c->syms[sym_b];
    const bool same_sym = sym_a == sym_b, same_cont = sa.ja0 == sb.ja0 && sa.nc == sb.nc;
    bool ok;
    switch (cls) {
    case 1: case 3: ok = same_sym; break;
    case 5: case 6: ok = !same_sym && same_cont; break;
    case 7: ok = !same_cont; break;
    default: return fail(c, CCH_E_INVALID_ARG, "no class %d", cls);
    }
    if (!ok) return fail(c, CCH_E_INVALID_ARG, "class %d does not occur between symmetries %d and %d", cls, sym_a, sym_b);
    *row0 = sa.row0;
    *nrows = (int64_t)sa.S * sa.nc;
    *col0 = sb.row0;
    *ncols = (int64_t)sb.S * sb.nc;
    *mode = cls == 7 ? 0 : cls;
    *nca = sa.nc;
    *ncb = sb.nc;
    return CCH_OK;
}

cch_status cch_block_shape(cch_ctx *c, int32_t cls, int32_t sym_a, int32_t sym_b, int64_t *rows, int64_t *cols)
{
    if (!c || !rows || !cols) return CCH_E_INVALID_ARG;
    if (!c->planned) return fail(c, CCH_E_STATE, "plan first");
    int64_t r0, c0;
    int mode, nca, ncb;
    TRY(block_geometry(c, cls, sym_a, sym_b, &r0, rows, &c0, cols, &mode, &nca, &ncb));
    return CCH_OK;
}

cch_status cch_get_block(cch_ctx *c, int32_t cls, int32_t sym_a, int32_t sym_b, double *out, int64_t ld, int32_t flags)
{
    if (!c || !out) return CCH_E_INVALID_ARG;
    if (!c->built) return fail(c, CCH_E_STATE, "build first");
    int64_t r0, nr, c0, nc;
    int mode, nca, ncb;
    TRY(block_geometry(c, cls, sym_a, sym_b, &r0, &nr, &c0, &nc, &mode, &nca, &ncb));
    if (ld < nc) return fail(c, CCH_E_INVALID_ARG, "ld %lld below the block width %lld", (long long)ld, (long long)nc);
    if (nr == 0 || nc == 0) return CCH_OK;
    HIPCK(c, hipSetDevice(c->device));
    if (c->sparse && (mode == 2 || mode == 8)) {
        // the L2 block from its CSR, in row blocks of at most 1 GiB
        const SparseMat S = sparse_mat(c);
        const int64_t rows_per = std::max<int64_t>(1, (int64_t(1) << 30) / (8 * nc));
        double *stage = nullptr;
        if (!(flags & CCH_MEM_DEVICE) && hipMalloc((void **)&stage, 8 * (size_t)rows_per * nc) != hipSuccess)
            return fail(c, CCH_E_OOM, "block staging");
        hipError_t e = hipSuccess;
        for (int64_t i0 = 0; i0 < nr && e == hipSuccess; i0 += rows_per) {
            const int64_t m = std::min(rows_per, nr - i0);
            if (flags & CCH_MEM_DEVICE) {
                e = launch_sparse_rows(S, r0 + i0, (int)m, c0, (int)nc, mode, out + i0 * ld, ld, c->stream);
            } else {
                e = launch_sparse_rows(S, r0 + i0, (int)m, c0, (int)nc, mode, stage, nc, c->stream);
                if (e == hipSuccess)
                    e = hipMemcpy2DAsync(out + i0 * ld, ld * 8, stage, nc * 8, nc * 8, m, hipMemcpyDeviceToHost,
                                         c->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            }
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        (void)hipFree(stage);
        if (e != hipSuccess) return fail(c, CCH_E_HIP, "cch_get_block: %s", hipGetErrorString(e));
        return CCH_OK;
    }
    if (flags & CCH_MEM_DEVICE) {
        HIPCK(c, launch_get_block(c->d_H, c->ld, r0, (int)nr, c0, (int)nc, mode, nca, ncb, out, ld, c->stream));
        HIPCK(c, hipStreamSynchronize(c->stream));
        return CCH_OK;
    }
    double *tmp = nullptr;
    if (hipMalloc((void **)&tmp, 8 * (size_t)nr * nc) != hipSuccess) return fail(c, CCH_E_OOM, "block staging");
    hipError_t e = launch_get_block(c->d_H, c->ld, r0, (int)nr, c0, (int)nc, mode, nca, ncb, tmp, nc, c->stream);
    if (e == hipSuccess) e = hipMemcpy2DAsync(out, ld * 8, tmp, nc * 8, nc * 8, nr, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(c, CCH_E_HIP, "cch_get_block: %s", hipGetErrorString(e));
    return CCH_OK;
}

cch_status cch_subspace_eig(cch_ctx *c, const double *G, int32_t ldg, int32_t m, double *theta, double *Y,
                            int32_t ldy, int32_t method, int32_t *fallback, int32_t flags)
{
    if (!c || !G || !theta || !Y) return CCH_E_INVALID_ARG;
    if (m < 1 || m > 96) return fail(c, CCH_E_INVALID_ARG, "m must lie in [1, 96]");
    if (ldg < m || ldy < m) return fail(c, CCH_E_INVALID_ARG, "leading dimension below m");
    if (method != CCH_EIG_AUTO && method != CCH_EIG_JACOBI) return fail(c, CCH_E_INVALID_ARG, "unknown method");
    HIPCK(c, hipSetDevice(c->device));
    hipStream_t st = c->stream;
    const bool dev = flags & CCH_MEM_DEVICE;
    double *dG = nullptr, *dT = nullptr, *dY = nullptr;
    int32_t *dF = nullptr;
    auto cleanup = [&]() {
        if (!dev) {
            (void)hipFree(dG);
            (void)hipFree(dT);
            (void)hipFree(dY);
        }
        (void)hipFree(dF);
    };
#define ECK(x)                                                                                  \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) {                                                                 \
            cleanup();                                                                          \
            return fail(c, CCH_E_HIP, "%s: %s", #x, hipGetErrorString(e_));                    \
        }                                                                                       \
    } while (0)
    if (dev) {
        dG = const_cast<double *>(G);
        dT = theta;
        dY = Y;
    } else {
        ECK(hipMalloc((void **)&dG, 8 * (size_t)m * ldg));
        ECK(hipMalloc((void **)&dT, 8 * (size_t)m));
        ECK(hipMalloc((void **)&dY, 8 * (size_t)m * ldy));
        ECK(hipMemcpyAsync(dG, G, 8 * (size_t)m * ldg, hipMemcpyHostToDevice, st));
    }
    ECK(hipMalloc((void **)&dF, 4));
    ECK(hipMemsetAsync(dF, 0, 4, st));
    if (method == CCH_EIG_JACOBI) ECK(launch_jacobi_eig(dG, ldg, m, dT, dY, ldy, st));
    else ECK(launch_rr_eig(dG, ldg, m, dT, dY, ldy, dF, st));
    int32_t hf = 0;
    ECK(hipMemcpyAsync(&hf, dF, 4, hipMemcpyDeviceToHost, st));
    if (!dev) {
        ECK(hipMemcpyAsync(theta, dT, 8 * (size_t)m, hipMemcpyDeviceToHost, st));
        ECK(hipMemcpyAsync(Y, dY, 8 * (size_t)m * ldy, hipMemcpyDeviceToHost, st));
    }
    ECK(hipStreamSynchronize(st));
#undef ECK
    cleanup();
    if (fallback) *fallback = hf;
    return CCH_OK;
}

cch_status cch_eig_all(cch_ctx *c, const double *A, int64_t lda, int32_t n, double *w, double *V, int64_t ldv,
                       int32_t flags, cch_eig_info *info)
{
    if (!c || !w) return CCH_E_INVALID_ARG;
    const bool own = A == nullptr;   // the built matrix
    if (own) {
        if (!c->built) return fail(c, CCH_E_STATE, "build first (or pass a matrix)");
        if (c->sparse) return fail(c, CCH_E_STATE, "the L2 block is stored as CSR (CCH_PLAN_SPARSE_L2)");
        if (n != 0 && n != c->D) return fail(c, CCH_E_INVALID_ARG, "n must be 0 or D for the built matrix");
        n = (int32_t)c->D;
    } else if (n < 1 || lda < n) {
        return fail(c, CCH_E_INVALID_ARG, "need n >= 1 and lda >= n");
    }
    if (V && ldv < n) return fail(c, CCH_E_INVALID_ARG, "ldv < n");
    HIPCK(c, hipSetDevice(c->device));
    hipStream_t st = c->stream;
    const bool dev = flags & CCH_MEM_DEVICE;
    const int64_t ld = ((int64_t)n + 31) / 32 * 32;
    const int NB = 128;   // reflectors per block of the back-transformation (at most 128: launch_larft)
    std::vector<void *> tmp;
    auto cleanup = [&]() { for (void *p : tmp) (void)hipFree(p); };
    auto al = [&](void **p, size_t bytes) -> bool {
        if (hipMalloc(p, bytes ? bytes : 8) != hipSuccess) return false;
        tmp.push_back(*p);
        return true;
    };
    double *W = nullptr, *Z = nullptr, *S = nullptr, *vec = nullptr, *Vb = nullptr, *G = nullptr, *T = nullptr,
           *w_d = nullptr, *Pk = nullptr;
    // split-K partials of the back-transformation's long products
    const int64_t p_cap = std::max<int64_t>((int64_t)16 * NB * n, (int64_t)64 * NB * NB);
    const bool want_v = V != nullptr;
    double *pan = nullptr;   // the reduction's panel buffers PV, PW and the products z
    bool ok = al((void **)&W, 8 * (size_t)n * ld) && al((void **)&vec, 8 * (size_t)10 * n + 64) &&
              al((void **)&w_d, 8 * (size_t)n) && al((void **)&pan, 8 * trd_panel_doubles(n, ld));
    if (ok && want_v)
        // S: the twisted-factorisation scratch, then two NB x n products of the back-transformation
        ok = al((void **)&Z, 8 * (size_t)n * ld) &&
             al((void **)&S, 8 * (size_t)std::max<int64_t>((int64_t)n * ld, (int64_t)2 * NB * n)) &&
             al((void **)&Vb, 8 * (size_t)n * NB) && al((void **)&G, 8 * NB * NB) && al((void **)&T, 8 * NB * NB) &&
             al((void **)&Pk, 8 * (size_t)p_cap);
    if (!ok) {
        cleanup();
        return fail(c, CCH_E_OOM, "eigensolver work space for n = %d", n);
    }
#define EGK(x)                                                                                  \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) {                                                                 \
            cleanup();                                                                          \
            return fail(c, CCH_E_HIP, "%s: %s", #x, hipGetErrorString(e_));                    \
        }                                                                                       \
    } while (0)
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
    EGK(hipEventCreate(&e0));
    EGK(hipEventCreate(&e1));
    EGK(hipEventCreate(&e2));
    EGK(hipEventCreate(&e3));
    auto evclean = [&]() {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipEventDestroy(e2);
        (void)hipEventDestroy(e3);
    };
    // the matrix into the work array, made exactly symmetric ((A + A^T) / 2)
    if (own)
        EGK(hipMemcpy2DAsync(W, 8 * ld, c->d_H, 8 * c->ld, 8 * (size_t)n, n, hipMemcpyDeviceToDevice, st));
    else
        EGK(hipMemcpy2DAsync(W, 8 * ld, A, 8 * lda, 8 * (size_t)n, n,
                             dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    EGK(launch_symmetrize(W, ld, n, st));
    EGK(hipEventRecord(e0, st));
    TrdVec tv{vec, vec + n, vec + 2 * (int64_t)n, vec + 3 * (int64_t)n, vec + 4 * (int64_t)n};
    double *e2v = vec + 8 * (int64_t)n;
    TrdPanel tp;
    tp.PVt = pan;
    tp.PV = pan + (int64_t)2 * TRD_NB * n;
    tp.PW = tp.PV + (int64_t)2 * TRD_NB * ld;
    tp.ldp = ld;
    tp.part1 = tp.PV + (int64_t)4 * TRD_NB * ld;
    tp.part2 = tp.part1 + (int64_t)((n + TRD_CR - 1) / TRD_CR) * TRD_PS;
    tp.rowp = tp.part2 + (n + 3) / 4;
    tp.colp = tp.rowp + (int64_t)trd_tiles(n) * n;
    tp.z = tp.colp + (int64_t)trd_tiles(n) * n;
    for (int j0 = 0; j0 < n; j0 += TRD_NB) EGK(launch_trd_panel(W, ld, n, j0, std::min(TRD_NB, n - j0), tv, tp, st));
    EGK(hipEventRecord(e1, st));
    // Gershgorin interval, pivot floor and the split of T into unreduced
    // blocks (off-diagonals below the rounding of their neighbours set to 0)
    std::vector<double> hd((size_t)n), he((size_t)std::max(n - 1, 1));
    EGK(hipMemcpyAsync(hd.data(), tv.d, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    if (n > 1) EGK(hipMemcpyAsync(he.data(), tv.e, 8 * (size_t)(n - 1), hipMemcpyDeviceToHost, st));
    EGK(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(hd[i]) || (i < n - 1 && !std::isfinite(he[i]))) {
            evclean();
            cleanup();
            return fail(c, CCH_E_INPUT, "non-finite tridiagonal entry (the matrix holds a non-finite value)");
        }
    for (int i = 0; i + 1 < n; ++i)
        if (std::fabs(he[i]) <= 2.220446049250313e-16 * 0.5 * (std::fabs(hd[i]) + std::fabs(hd[i + 1])))
            he[i] = 0.0;
    double lo = 1e300, hi = -1e300, emax = 0.0, tnorm = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(he[i - 1]) : 0.0) + (i < n - 1 ? std::fabs(he[i]) : 0.0);
        lo = std::min(lo, hd[i] - r);
        hi = std::max(hi, hd[i] + r);
        if (i < n - 1) emax = std::max(emax, he[i] * he[i]);
        tnorm = std::max(tnorm, std::fabs(hd[i]) + r);
    }
    const double pad = 2.0 * std::max(tnorm, 1e-300) * 1e-15 + 1e-300;
    lo -= pad;
    hi += pad;
    const double pivmin = 2.2250738585072014e-308 * std::max(1.0, emax);
    // eigenvalue slots block by block: (block start, block rows, index in the block)
    std::vector<int32_t> bs((size_t)n), bm((size_t)n), bk((size_t)n);
    int nblocks = 0;
    for (int b0 = 0; b0 < n;) {
        int b1 = b0 + 1;
        while (b1 < n && he[b1 - 1] != 0.0) ++b1;
        for (int i = b0; i < b1; ++i) {
            bs[i] = b0;
            bm[i] = b1 - b0;
            bk[i] = i - b0;
        }
        ++nblocks;
        b0 = b1;
    }
    int32_t *d_bs = nullptr, *d_bm = nullptr, *d_bk = nullptr;
    if (!al((void **)&d_bs, 4 * (size_t)n) || !al((void **)&d_bm, 4 * (size_t)n) || !al((void **)&d_bk, 4 * (size_t)n)) {
        evclean();
        cleanup();
        return fail(c, CCH_E_OOM, "eigensolver block tables");
    }
    if (n > 1) EGK(hipMemcpyAsync(tv.e, he.data(), 8 * (size_t)(n - 1), hipMemcpyHostToDevice, st));
    EGK(hipMemcpyAsync(d_bs, bs.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
    EGK(hipMemcpyAsync(d_bm, bm.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
    EGK(hipMemcpyAsync(d_bk, bk.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
    EGK(launch_tri_eigenvalues(tv.d, tv.e, e2v, n, d_bs, d_bm, d_bk, lo, hi, pivmin, vec + 9 * (int64_t)n, st));
    // ascending order over all blocks (stable: ties keep the block order)
    std::vector<double> wb((size_t)n);
    EGK(hipMemcpyAsync(wb.data(), vec + 9 * (int64_t)n, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    EGK(hipStreamSynchronize(st));
    std::vector<int> ord((size_t)n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return wb[a] < wb[b]; });
    std::vector<double> hw((size_t)n);
    std::vector<int32_t> sbs((size_t)n), sbm((size_t)n);
    for (int p = 0; p < n; ++p) {
        hw[p] = wb[ord[p]];
        sbs[p] = bs[ord[p]];
        sbm[p] = bm[ord[p]];
    }
    EGK(hipMemcpyAsync(w_d, hw.data(), 8 * (size_t)n, hipMemcpyHostToDevice, st));
    EGK(hipEventRecord(e2, st));
    int clusters = 0, clustered = 0;
    if (want_v) {
        EGK(hipMemcpyAsync(d_bs, sbs.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
        EGK(hipMemcpyAsync(d_bm, sbm.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
        EGK(launch_tri_vectors(tv.d, tv.e, n, d_bs, d_bm, w_d, pivmin, Z, ld, S, ld, st));
        // clusters: eigenvalues of one block closer than 1e-5 ||T|| to the
        // previous one of the same block, re-orthogonalised in order
        const double gap = 1e-5 * std::max(tnorm, 1e-300);
        std::map<int, std::vector<int32_t>> per_block;   // block start -> its columns, ascending
        for (int p = 0; p < n; ++p) per_block[sbs[p]].push_back(p);
        std::vector<int32_t> cl_cols;
        std::vector<std::array<int, 4>> cl;   // (offset in cl_cols, count, block start, block rows)
        for (auto &kv : per_block) {
            const std::vector<int32_t> &cols = kv.second;
            for (size_t a = 0; a < cols.size();) {
                size_t b = a + 1;
                while (b < cols.size() && hw[cols[b]] - hw[cols[b - 1]] < gap) ++b;
                if (b - a > 1) {
                    cl.push_back({(int)cl_cols.size(), (int)(b - a), kv.first, sbm[cols[a]]});
                    cl_cols.insert(cl_cols.end(), cols.begin() + a, cols.begin() + b);
                    ++clusters;
                    clustered += (int)(b - a);
                }
                a = b;
            }
        }
        if (!cl.empty()) {
            // the columns, then the descriptors (offset, count, block start, block rows)
            std::vector<int32_t> lists(cl_cols);
            for (auto &q : cl) lists.insert(lists.end(), q.begin(), q.end());
            int32_t *d_cl = nullptr;
            if (!al((void **)&d_cl, 4 * lists.size())) {
                evclean();
                cleanup();
                return fail(c, CCH_E_OOM, "eigensolver cluster lists");
            }
            EGK(hipMemcpyAsync(d_cl, lists.data(), 4 * lists.size(), hipMemcpyHostToDevice, st));
            // pivot floor of the inverse-iteration solves: the rounding of ||T||
            const double piv = 2.220446049250313e-16 * std::max(tnorm, 1e-300);
            EGK(launch_cluster_mgs(Z, ld, d_cl + cl_cols.size(), (int)cl.size(), d_cl, tv.d, tv.e, w_d, S, ld, piv,
                                   st));
        }
        // Z = Q Z_T: the blocks of reflectors from the last to the first
        const int nref = n - 1;
        const int nblk = (nref + NB - 1) / NB;
        for (int bi = nblk - 1; bi >= 0; --bi) {
            const int j0 = bi * NB, nb = std::min(NB, nref - j0), m = n - j0 - 1;
            double *Zs = Z + (int64_t)(j0 + 1) * ld;
            double *Wt = S, *W2 = S + (int64_t)NB * n;   // the twisted-factorisation scratch is free now
            EGK(launch_copy_reflectors(W, ld, n, j0, nb, Vb, st));
            EGK(launch_eig_gemm(nb, nb, m, 1.0, Vb, 1, nb, Vb, nb, 1, 0.0, G, nb, st, Pk, p_cap));
            EGK(launch_larft(G, tv.tau + j0, nb, T, Pk, st));   // (Pk is free between the products)
            EGK(launch_eig_gemm(nb, n, m, 1.0, Vb, 1, nb, Zs, ld, 1, 0.0, Wt, n, st, Pk, p_cap));
            EGK(launch_eig_gemm(nb, n, nb, 1.0, T, nb, 1, Wt, n, 1, 0.0, W2, n, st));
            EGK(launch_eig_gemm(m, n, nb, -1.0, Vb, nb, 1, W2, n, 1, 1.0, Zs, ld, st));
        }
        // rows of the output are the eigenvectors
        if (dev) {
            EGK(launch_transpose_sq(Z, ld, n, V, ldv, st));
        } else {
            EGK(launch_transpose_sq(Z, ld, n, S, ld, st));
            EGK(hipMemcpy2DAsync(V, 8 * ldv, S, 8 * ld, 8 * (size_t)n, n, hipMemcpyDeviceToHost, st));
        }
    }
    EGK(hipEventRecord(e3, st));
    EGK(hipMemcpyAsync(w, w_d, 8 * (size_t)n, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    EGK(hipStreamSynchronize(st));
    if (info) {
        float t01 = 0.0f, t12 = 0.0f, t23 = 0.0f;
        EGK(hipEventElapsedTime(&t01, e0, e1));
        EGK(hipEventElapsedTime(&t12, e1, e2));
        EGK(hipEventElapsedTime(&t23, e2, e3));
        info->tridiag_ms = t01;
        info->eigenvalues_ms = t12;
        info->vectors_ms = t23;
        info->clusters = clusters;
        info->clustered = clustered;
        // the distinct (lower-triangle) elements of the trailing block: read
        // once per column, read and written once per panel
        double tb = 0.0;
        for (int j = 0; j < n; ++j) {
            const double m = n - j - 1;
            tb += 4.0 * m * (m + 1.0);
            if (j % TRD_NB == 0 && j > 0) tb += 8.0 * (m + 1.0) * (m + 2.0);
        }
        info->tridiag_bytes = tb;
        info->backtransform_flops = want_v ? 2.0 * (double)n * n * n : 0.0;
    }
#undef EGK
    evclean();
    cleanup();
    return CCH_OK;
}

cch_status cch_get_labels(cch_ctx *c, int32_t which, int32_t sym_a, int32_t sym_b, int32_t *x, int32_t *y,
                          int8_t *degree, uint64_t *label, int8_t *phase, int64_t cap, int64_t *n)
{
    if (!c || !n) return CCH_E_INVALID_ARG;
    if (!c->have_ints && !c->have_orb) return fail(c, CCH_E_STATE, "no orbitals");
    const int ns = (int)c->syms.size();
    const uint64_t *A = nullptr, *B = nullptr;
    int nA = 0, nB = 0, mode;
    if (which == CCH_PAIRS_TARGET) {
        if (sym_a < 0 || sym_a >= ns || sym_b < 0 || sym_b >= ns) return fail(c, CCH_E_INVALID_ARG, "bad symmetry");
        A = c->syms[sym_a].d_dets; nA = c->syms[sym_a].M;
        B = c->syms[sym_b].d_dets; nB = c->syms[sym_b].M;
        mode = SCAN_TT;
    } else if (which == CCH_PAIRS_L2) {
        A = B = c->d_l2; nA = nB = c->n_l2;
        mode = SCAN_LL;
    } else if (which == CCH_PAIRS_L2_TARGET) {
        if (sym_a < 0 || sym_a >= ns) return fail(c, CCH_E_INVALID_ARG, "bad symmetry");
        A = c->d_l2; nA = c->n_l2;
        B = c->syms[sym_a].d_dets; nB = c->syms[sym_a].M;
        mode = SCAN_LT;
    } else {
        return fail(c, CCH_E_INVALID_ARG, "bad list selector");
    }
    *n = 0;
    if (nA == 0 || nB == 0) return CCH_OK;
    HIPCK(c, hipSetDevice(c->device));
    // temporary buffers, freed at the end of the call
    std::vector<void *> tmp;
    auto galloc = [&](void **p, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(p, bytes ? bytes : 8);
        if (e == hipSuccess) tmp.push_back(*p);
        return e;
    };
    auto cleanup = [&]() { for (void *p : tmp) (void)hipFree(p); };
    DevPairs P;
    int64_t *d_total = nullptr;
    hipError_t e = galloc((void **)&P.row_off, 8 * (size_t)nA);
    if (e == hipSuccess) e = galloc((void **)&P.row_cnt, 8 * (size_t)nA);
    if (e == hipSuccess) e = galloc((void **)&d_total, 8);
    if (e == hipSuccess) e = launch_scan(mode, c->W, A, nA, B, nB, 2 * c->n_o, nullptr, P.row_cnt, PairList{}, c->stream);
    if (e == hipSuccess) e = launch_exclusive_scan(P.row_cnt, P.row_off, nA, d_total, c->stream);
    int64_t total = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&total, d_total, 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = galloc((void **)&P.pl.x, 4 * (size_t)total);
    if (e == hipSuccess) e = galloc((void **)&P.pl.y, 4 * (size_t)total);
    if (e == hipSuccess) e = galloc((void **)&P.pl.deg, (size_t)total);
    if (e == hipSuccess) e = galloc((void **)&P.pl.phase, (size_t)total);
    if (e == hipSuccess) e = galloc((void **)&P.pl.label, 8 * (size_t)total);
    if (e == hipSuccess) e = launch_scan(mode, c->W, A, nA, B, nB, 2 * c->n_o, P.row_off, P.row_cnt, P.pl, c->stream);
    const int64_t m = std::min(total, cap);
    if (e == hipSuccess && m > 0) {
        if (x) e = hipMemcpyAsync(x, P.pl.x, 4 * m, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && y) e = hipMemcpyAsync(y, P.pl.y, 4 * m, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && degree) e = hipMemcpyAsync(degree, P.pl.deg, m, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && phase) e = hipMemcpyAsync(phase, P.pl.phase, m, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && label) e = hipMemcpyAsync(label, P.pl.label, 8 * m, hipMemcpyDeviceToHost, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    cleanup();
    if (e != hipSuccess) return fail(c, CCH_E_HIP, "label scan: %s", hipGetErrorString(e));
    *n = total;
    return CCH_OK;
}


// ---------------------------------------------------------------------------
// learned preconditioner object
// ---------------------------------------------------------------------------
#include <random>

struct cch_mlp {
    int device = 0;
    hipStream_t st = nullptr;
    std::string err;
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    __bf16 *w2 = nullptr, *w2t = nullptr;
    double *loss = nullptr;
    int step = 0;
    // scratch for rows (grown on demand)
    float *part = nullptr;
    double *lpart = nullptr;
    int part_blocks = 0;
    float *xin = nullptr, *tin = nullptr, *ein = nullptr, *win = nullptr, *gout = nullptr;
    int64_t cap = 0;
};

static cch_status mfail(cch_mlp *m, cch_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (m) m->err = buf;
    else g_create_err = buf;
    return code;
}

#define MCK(m, x)                                                                                \
    do {                                                                                         \
        hipError_t e_ = (x);                                                                     \
        if (e_ != hipSuccess) return mfail((m), CCH_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

int32_t cch_mlp_num_params(void) { return mlp_num_params(); }

cch_status cch_mlp_destroy(cch_mlp *m)
{
    if (!m) return CCH_OK;
    (void)hipSetDevice(m->device);
    (void)hipStreamSynchronize(m->st);
    for (void *p : {(void *)m->w, (void *)m->m, (void *)m->v, (void *)m->grad, (void *)m->w2, (void *)m->w2t,
                    (void *)m->loss, (void *)m->part, (void *)m->lpart, (void *)m->xin, (void *)m->tin,
                    (void *)m->ein, (void *)m->win, (void *)m->gout})
        if (p) (void)hipFree(p);
    delete m;
    return CCH_OK;
}

const char *cch_mlp_last_error(const cch_mlp *m) { return m ? m->err.c_str() : g_create_err.c_str(); }

cch_status cch_mlp_create(cch_mlp **out, int32_t device, void *hip_stream, uint64_t seed)
{
    if (!out) return mfail(nullptr, CCH_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t he = hipGetDeviceCount(&ndev);
    if (he != hipSuccess || ndev <= 0) return mfail(nullptr, CCH_E_HIP, "no HIP device: %s", hipGetErrorString(he));
    if (device < 0 || device >= ndev) return mfail(nullptr, CCH_E_INVALID_ARG, "device %d out of range", device);
    he = hipSetDevice(device);
    if (he != hipSuccess) return mfail(nullptr, CCH_E_HIP, "hipSetDevice(%d): %s", device, hipGetErrorString(he));
    cch_mlp *m = new (std::nothrow) cch_mlp();
    if (!m) return mfail(nullptr, CCH_E_OOM, "allocation failed");
    m->device = device;
    m->st = (hipStream_t)hip_stream;
    const int P = mlp_num_params();
    bool ok = hipMalloc(&m->w, 4 * (size_t)P) == hipSuccess && hipMalloc(&m->m, 4 * (size_t)P) == hipSuccess &&
              hipMalloc(&m->v, 4 * (size_t)P) == hipSuccess && hipMalloc(&m->grad, 4 * (size_t)P) == hipSuccess &&
              hipMalloc(&m->w2, 2 * 128 * 128) == hipSuccess && hipMalloc(&m->w2t, 2 * 128 * 128) == hipSuccess &&
              hipMalloc(&m->loss, 8) == hipSuccess;
    if (!ok) {
        cch_mlp_destroy(m);
        return mfail(nullptr, CCH_E_OOM, "MLP buffers");
    }
    // He initialisation; output layer near zero so the network starts as Jacobi
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.f, 1.f);
    std::vector<float> w(P, 0.f);
    for (int i = 0; i < 128 * 4; ++i) w[i] = nd(rng) * std::sqrt(2.f / 4.f);
    for (int i = 0; i < 128 * 128; ++i) w[128 * 4 + 128 + i] = nd(rng) * std::sqrt(2.f / 128.f);
    for (int i = 0; i < 128; ++i) w[128 * 4 + 128 + 128 * 128 + 128 + i] = nd(rng) * 1e-3f;
    std::vector<float> z(P, 0.f);
    ok = hipMemcpy(m->w, w.data(), 4 * (size_t)P, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->m, z.data(), 4 * (size_t)P, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->v, z.data(), 4 * (size_t)P, hipMemcpyHostToDevice) == hipSuccess &&
         launch_mlp_pack(m->w, m->w2, m->w2t, m->st) == hipSuccess && hipStreamSynchronize(m->st) == hipSuccess;
    if (!ok) {
        cch_mlp_destroy(m);
        return mfail(nullptr, CCH_E_HIP, "MLP initialisation");
    }
    *out = m;
    return CCH_OK;
}

cch_status cch_mlp_set_weights(cch_mlp *m, const float *w, int64_t n, int32_t flags)
{
    if (!m || !w) return CCH_E_INVALID_ARG;
    if (n != mlp_num_params()) return mfail(m, CCH_E_INVALID_ARG, "expected %d weights", mlp_num_params());
    MCK(m, hipSetDevice(m->device));
    MCK(m, hipMemcpyAsync(m->w, w, 4 * (size_t)n, (flags & CCH_MEM_DEVICE) ? hipMemcpyDeviceToDevice
                                                                            : hipMemcpyHostToDevice, m->st));
    MCK(m, launch_mlp_pack(m->w, m->w2, m->w2t, m->st));
    MCK(m, hipStreamSynchronize(m->st));
    m->step = 0;
    return CCH_OK;
}

cch_status cch_mlp_get_weights(cch_mlp *m, float *w, int64_t n, int32_t flags)
{
    if (!m || !w) return CCH_E_INVALID_ARG;
    if (n != mlp_num_params()) return mfail(m, CCH_E_INVALID_ARG, "expected %d weights", mlp_num_params());
    MCK(m, hipMemcpyAsync(w, m->w, 4 * (size_t)n, (flags & CCH_MEM_DEVICE) ? hipMemcpyDeviceToDevice
                                                                            : hipMemcpyDeviceToHost, m->st));
    MCK(m, hipStreamSynchronize(m->st));
    return CCH_OK;
}

// rows staged on the device (copied when host pointers are passed)
static cch_status mlp_rows(cch_mlp *m, int64_t n, const float *X, const float *tj, const float *e, const float *w,
                           int32_t flags, const float **dX, const float **dt, const float **de, const float **dw)
{
    if (n <= 0) return mfail(m, CCH_E_INVALID_ARG, "no rows");
    if (!(flags & CCH_MEM_DEVICE) && n > m->cap) {
        for (float *p : {m->xin, m->tin, m->ein, m->win}) if (p) (void)hipFree(p);
        m->xin = m->tin = m->ein = m->win = nullptr;
        if (hipMalloc(&m->xin, 16 * (size_t)n) != hipSuccess || hipMalloc(&m->tin, 4 * (size_t)n) != hipSuccess ||
            hipMalloc(&m->ein, 4 * (size_t)n) != hipSuccess || hipMalloc(&m->win, 4 * (size_t)n) != hipSuccess)
            return mfail(m, CCH_E_OOM, "row buffers");
        m->cap = n;
    }
    if (flags & CCH_MEM_DEVICE) {
        *dX = X; *dt = tj; *de = e; *dw = w;
        return CCH_OK;
    }
    MCK(m, hipMemcpyAsync(m->xin, X, 16 * (size_t)n, hipMemcpyHostToDevice, m->st));
    if (tj) MCK(m, hipMemcpyAsync(m->tin, tj, 4 * (size_t)n, hipMemcpyHostToDevice, m->st));
    if (e) MCK(m, hipMemcpyAsync(m->ein, e, 4 * (size_t)n, hipMemcpyHostToDevice, m->st));
    if (w) MCK(m, hipMemcpyAsync(m->win, w, 4 * (size_t)n, hipMemcpyHostToDevice, m->st));
    *dX = m->xin; *dt = m->tin; *de = m->ein; *dw = m->win;
    return CCH_OK;
}

static cch_status mlp_part(cch_mlp *m, int64_t n)
{
    const int blocks = mlp_grid(n);
    if (blocks > m->part_blocks) {
        if (m->part) (void)hipFree(m->part);
        if (m->lpart) (void)hipFree(m->lpart);
        m->part = nullptr;
        m->lpart = nullptr;
        if (hipMalloc(&m->part, 4 * (size_t)blocks * mlp_num_params()) != hipSuccess ||
            hipMalloc(&m->lpart, 8 * (size_t)blocks) != hipSuccess)
            return mfail(m, CCH_E_OOM, "gradient partials");
        m->part_blocks = blocks;
    }
    return CCH_OK;
}

cch_status cch_mlp_forward(cch_mlp *m, const float *X, int64_t n, float *g, int32_t flags)
{
    if (!m || !X || !g) return CCH_E_INVALID_ARG;
    MCK(m, hipSetDevice(m->device));
    const float *dX, *dt, *de, *dw;
    TRY(mlp_rows(m, n, X, nullptr, nullptr, nullptr, flags, &dX, &dt, &de, &dw));
    float *dg = g;
    if (!(flags & CCH_MEM_DEVICE)) {
        if (m->gout) (void)hipFree(m->gout);
        m->gout = nullptr;
        if (hipMalloc(&m->gout, 4 * (size_t)n) != hipSuccess) return mfail(m, CCH_E_OOM, "output buffer");
        dg = m->gout;
    }
    MCK(m, launch_mlp_forward(m->w, m->w2, m->w2t, dX, n, dg, m->st));
    if (!(flags & CCH_MEM_DEVICE)) MCK(m, hipMemcpyAsync(g, dg, 4 * (size_t)n, hipMemcpyDeviceToHost, m->st));
    MCK(m, hipStreamSynchronize(m->st));
    return CCH_OK;
}

cch_status cch_mlp_grad(cch_mlp *m, const float *X, const float *tj, const float *e, const float *w, int64_t n,
                        double *loss, float *grad, int32_t flags)
{
    if (!m || !X || !tj || !e || !w) return CCH_E_INVALID_ARG;
    MCK(m, hipSetDevice(m->device));
    const float *dX, *dt, *de, *dw;
    TRY(mlp_rows(m, n, X, tj, e, w, flags, &dX, &dt, &de, &dw));
    TRY(mlp_part(m, n));
    MCK(m, launch_mlp_grad(m->w, m->w2, m->w2t, dX, dt, de, dw, n, m->part, m->lpart, m->grad, m->loss, m->st));
    if (grad)
        MCK(m, hipMemcpyAsync(grad, m->grad, 4 * (size_t)mlp_num_params(),
                              (flags & CCH_MEM_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, m->st));
    if (loss) MCK(m, hipMemcpyAsync(loss, m->loss, 8, hipMemcpyDeviceToHost, m->st));
    MCK(m, hipStreamSynchronize(m->st));
    return CCH_OK;
}

cch_status cch_mlp_train_step(cch_mlp *m, const float *X, const float *tj, const float *e, const float *w,
                              int64_t n, float lr, double *loss, int32_t flags)
{
    if (!m || !X || !tj || !e || !w || !(lr > 0.f)) return CCH_E_INVALID_ARG;
    MCK(m, hipSetDevice(m->device));
    const float *dX, *dt, *de, *dw;
    TRY(mlp_rows(m, n, X, tj, e, w, flags, &dX, &dt, &de, &dw));
    TRY(mlp_part(m, n));
    MCK(m, launch_mlp_grad(m->w, m->w2, m->w2t, dX, dt, de, dw, n, m->part, m->lpart, m->grad, m->loss, m->st));
    MCK(m, launch_adam(m->w, m->m, m->v, m->grad, lr, ++m->step, m->st));
    MCK(m, launch_mlp_pack(m->w, m->w2, m->w2t, m->st));
    if (loss) MCK(m, hipMemcpyAsync(loss, m->loss, 8, hipMemcpyDeviceToHost, m->st));
    MCK(m, hipStreamSynchronize(m->st));
    return CCH_OK;
}

namespace cch {
hipError_t launch_mlp_features_theta(const double *diag, const double *rho, int D, int Dc, double theta, float *X,
                                     hipStream_t st);
}

cch_status cch_mlp_features(cch_ctx *c, double theta, float *X, int32_t flags)
{
    if (!c || !X) return CCH_E_INVALID_ARG;
    if (!c->built) return fail(c, CCH_E_STATE, "build first");
    HIPCK(c, hipSetDevice(c->device));
    const int D = (int)c->D;
    double *rho = nullptr, *th = nullptr;
    float *dX = X;
    int32_t *sel = nullptr;
    bool ok = hipMalloc(&rho, 8 * (size_t)D) == hipSuccess && hipMalloc(&th, 8) == hipSuccess &&
              hipMalloc(&sel, 4) == hipSuccess;
    if (ok && !(flags & CCH_MEM_DEVICE)) ok = hipMalloc(&dX, 16 * (size_t)D) == hipSuccess;
    const int32_t zero = 0;
    hipError_t e = ok ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipMemcpy(th, &theta, 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sel, &zero, 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = c->sparse ? launch_sparse_row_norms(sparse_mat(c), D, rho, c->stream)
                      : launch_row_norms(c->d_H, c->ld, D, rho, c->stream);
    if (e == hipSuccess) e = launch_mlp_features_theta(c->d_diag, rho, D, (int)c->Dc, theta, dX, c->stream);
    if (e == hipSuccess && !(flags & CCH_MEM_DEVICE))
        e = hipMemcpyAsync(X, dX, 16 * (size_t)D, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (rho) (void)hipFree(rho);
    if (th) (void)hipFree(th);
    if (sel) (void)hipFree(sel);
    if (dX && dX != X) (void)hipFree(dX);
    if (e != hipSuccess) return fail(c, CCH_E_HIP, "features: %s", hipGetErrorString(e));
    return CCH_OK;
}

cch_status cch_davidson_set_mlp(cch_ctx *c, cch_mlp *m)
{
    if (!c) return CCH_E_INVALID_ARG;
    if (m && m->device != c->device) return fail(c, CCH_E_INVALID_ARG, "network on another device");
    c->mlp = m;
    return CCH_OK;
}

// ---------------------------------------------------------------------------
// batched build
// ---------------------------------------------------------------------------

struct cch_batch {
    std::vector<cch_ctx *> cs;
    int device = 0;
    hipStream_t st = nullptr;
    std::string err;
    std::vector<void *> allocs;
    GemmTask *d_gemm[2] = {nullptr, nullptr};   // tile height 32 / 64
    int n_gemm = 0;
    int64_t gemm_total[2] = {0, 0};
    struct Group {
        int W;
        void *d_tasks;
        int n;
        int64_t total;
    };
    std::vector<Group> l2g, c4g;
    int bm = 64, g_gemm = 1024, g_c4 = 2048, g_l2 = 2048;
    int tuned = 0, cached = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t nodes = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float last_ms = 0.0f;
};

static std::map<std::string, std::array<int, 4>> g_tune_cache;

static cch_status bfail(cch_batch *b, cch_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    else g_create_err = buf;
    return code;
}

#define BCK(b, x)                                                                                \
    do {                                                                                         \
        hipError_t e_ = (x);                                                                     \
        if (e_ != hipSuccess) return bfail((b), CCH_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

template <class T>
static cch_status bupload(cch_batch *b, T **d, const std::vector<T> &h)
{
    void *p = nullptr;
    BCK(b, hipMalloc(&p, sizeof(T) * (h.empty() ? 1 : h.size())));
    b->allocs.push_back(p);
    if (!h.empty()) BCK(b, hipMemcpy(p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    *d = (T *)p;
    return CCH_OK;
}

static cch_status ctx_status(cch_batch *b, cch_ctx *c, cch_status rc)
{
    if (rc != CCH_OK) b->err = c->err;
    return rc;
}

static cch_status batch_gemm(cch_batch *b, int bm, int grid)
{
    const int v = bm == 32 ? 0 : 1;
    BCK(b, launch_expand_f64_batched(b->d_gemm[v], b->n_gemm, b->gemm_total[v], bm, grid, b->st));
    return CCH_OK;
}

static cch_status batch_c4(cch_batch *b, int grid)
{
    for (auto &g : b->c4g) BCK(b, launch_class4_batched(g.W, (const C4Task *)g.d_tasks, g.n, g.total, grid, b->st));
    return CCH_OK;
}

static cch_status batch_l2(cch_batch *b, int grid)
{
    for (auto &g : b->l2g) BCK(b, launch_l2_batched(g.W, (const L2Task *)g.d_tasks, g.n, g.total, grid, b->st));
    return CCH_OK;
}

static cch_status enqueue_batch(cch_batch *b)
{
    for (cch_ctx *c : b->cs) TRY(ctx_status(b, c, enqueue_pre(c, b->st, false, false)));
    TRY(batch_gemm(b, b->bm, b->g_gemm));
    TRY(batch_c4(b, b->g_c4));
    TRY(batch_l2(b, b->g_l2));
    for (cch_ctx *c : b->cs) TRY(ctx_status(b, c, enqueue_post(c, b->st)));
    return CCH_OK;
}

template <class F>
static cch_status time_it(cch_batch *b, F &&f, float *ms)
{
    BCK(b, hipEventRecord(b->e0, b->st));
    TRY(f());
    BCK(b, hipEventRecord(b->e1, b->st));
    BCK(b, hipEventSynchronize(b->e1));
    BCK(b, hipEventElapsedTime(ms, b->e0, b->e1));
    return CCH_OK;
}

cch_status cch_batch_create(cch_batch **out, cch_ctx *const *ctxs, int32_t n, int32_t flags)
{
    if (!out || !ctxs || n <= 0) return bfail(nullptr, CCH_E_INVALID_ARG, "bad batch arguments");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return bfail(nullptr, CCH_E_INVALID_ARG, "context %d is NULL", i);
        if (!ctxs[i]->planned) return bfail(nullptr, CCH_E_STATE, "context %d is not planned", i);
        if (ctxs[i]->sparse)
            return bfail(nullptr, CCH_E_STATE, "context %d stores its L2 block as CSR (CCH_PLAN_SPARSE_L2)", i);
        if (ctxs[i]->l2csf)
            return bfail(nullptr, CCH_E_STATE, "context %d has L2 functions given as CSFs", i);
        if (ctxs[i]->b_shared)
            return bfail(nullptr, CCH_E_STATE, "context %d was planned in several expansion passes", i);
        if (ctxs[i]->opts.precision != CCH_PREC_FP64)
            return bfail(nullptr, CCH_E_INVALID_ARG, "context %d: batched builds use the FP64 form", i);
        if (ctxs[i]->device != ctxs[0]->device) return bfail(nullptr, CCH_E_INVALID_ARG, "contexts on two devices");
    }
    cch_batch *b = new (std::nothrow) cch_batch();
    if (!b) return bfail(nullptr, CCH_E_OOM, "batch allocation failed");
    b->cs.assign(ctxs, ctxs + n);
    b->device = ctxs[0]->device;
    auto cleanup_fail = [&](cch_status rc) {
        g_create_err = b->err;
        cch_batch_destroy(b);
        return rc;
    };
    if (hipSetDevice(b->device) != hipSuccess || hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&b->e0) != hipSuccess || hipEventCreate(&b->e1) != hipSuccess)
        return cleanup_fail(bfail(b, CCH_E_HIP, "stream/event creation failed"));
    for (cch_ctx *c : b->cs)
        if (hipStreamSynchronize(c->stream) != hipSuccess) return cleanup_fail(bfail(b, CCH_E_HIP, "sync failed"));
    // task tables
    std::vector<GemmTask> g32, g64;
    int64_t t32 = 0, t64 = 0;
    std::map<int, std::vector<L2Task>> l2;
    std::map<int, std::vector<C4Task>> c4;
    std::map<int, int64_t> l2t, c4t;
    for (cch_ctx *c : b->cs) {
        for (auto &p : c->pp) {
            SymInfo &sa = c->syms[p.a], &sb = c->syms[p.b];
            if (sa.nc == 0 || sb.nc == 0 || p.nrows == 0) continue;
            GemmTask g{p.d_At, p.d_B, p.nrows, sa.nc * sb.nc, 2 * p.n_slot, 0, 0, 0, expand_epi(c, p)};
            g.tiles_m = (p.nrows + 31) / 32;
            g.tiles_n = expand_tiles(1, g.N, 32);
            g.first = t32;
            t32 += (int64_t)g.tiles_m * g.tiles_n;
            g32.push_back(g);
            g.tiles_m = (p.nrows + 63) / 64;
            g.first = t64;
            t64 += (int64_t)g.tiles_m * g.tiles_n;
            g64.push_back(g);
        }
        for (auto &L : c->lt) {
            const SymInfo &s = c->syms[L.sym];
            if (s.nc == 0 || c->n_l2 == 0) continue;
            C4Task k{class4_args(c, L), c->n_l2, (s.nc + C4_JB - 1) / C4_JB, c4t[c->W]};
            c4t[c->W] += (int64_t)k.n_l2 * k.jtiles;
            c4[c->W].push_back(k);
        }
        if (c->n_l2 > 0) {
            const TgtInts I{c->d_h, c->d_tttt, c->n_o, c->n_orb, c->e_core};
            L2Task t{L2Args{c->d_l2, c->n_l2, I, c->d_H, c->ld, c->Dc}, l2t[c->W]};
            l2t[c->W] += l2_tiles(c->n_l2);
            l2[c->W].push_back(t);
        }
    }
    b->n_gemm = (int)g64.size();
    b->gemm_total[0] = t32;
    b->gemm_total[1] = t64;
    cch_status rc;
    if ((rc = bupload(b, &b->d_gemm[0], g32)) != CCH_OK) return cleanup_fail(rc);
    if ((rc = bupload(b, &b->d_gemm[1], g64)) != CCH_OK) return cleanup_fail(rc);
    for (auto &kv : l2) {
        L2Task *d = nullptr;
        if ((rc = bupload(b, &d, kv.second)) != CCH_OK) return cleanup_fail(rc);
        b->l2g.push_back({kv.first, d, (int)kv.second.size(), l2t[kv.first]});
    }
    for (auto &kv : c4) {
        C4Task *d = nullptr;
        if ((rc = bupload(b, &d, kv.second)) != CCH_OK) return cleanup_fail(rc);
        b->c4g.push_back({kv.first, d, (int)kv.second.size(), c4t[kv.first]});
    }
    int cus = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, b->device) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    b->g_gemm = 4 * cus;
    b->g_c4 = 8 * cus;
    b->g_l2 = 8 * cus;
    if (flags & CCH_BATCH_AUTOTUNE) {
        int64_t c4tot = 0, l2tot = 0;
        for (auto &g : b->c4g) c4tot += g.total;
        for (auto &g : b->l2g) l2tot += g.total;
        char key[256];
        snprintf(key, sizeof key, "n%zu:g%d:%lld:%lld:c%lld:l%lld", b->cs.size(), b->n_gemm, (long long)t32,
                 (long long)t64, (long long)c4tot, (long long)l2tot);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            b->bm = it->second[0];
            b->g_gemm = it->second[1];
            b->g_c4 = it->second[2];
            b->g_l2 = it->second[3];
            b->cached = 1;
        } else {
            // inputs of the persistent phases
            for (cch_ctx *c : b->cs)
                if ((rc = ctx_status(b, c, enqueue_pre(c, b->st, false, false))) != CCH_OK) return cleanup_fail(rc);
            float best = 1e30f, ms = 0.0f;
            for (int bm : {64, 32})
                for (int mult : {1, 2, 4, 8}) {
                    if ((rc = time_it(b, [&] { return batch_gemm(b, bm, mult * cus); }, &ms)) != CCH_OK)
                        return cleanup_fail(rc);
                    if (ms < best) {
                        best = ms;
                        b->bm = bm;
                        b->g_gemm = mult * cus;
                    }
                }
            best = 1e30f;
            for (int mult : {2, 4, 8, 16}) {
                if ((rc = time_it(b, [&] { return batch_c4(b, mult * cus); }, &ms)) != CCH_OK) return cleanup_fail(rc);
                if (ms < best) {
                    best = ms;
                    b->g_c4 = mult * cus;
                }
            }
            best = 1e30f;
            for (int mult : {2, 4, 8, 16}) {
                if ((rc = time_it(b, [&] { return batch_l2(b, mult * cus); }, &ms)) != CCH_OK) return cleanup_fail(rc);
                if (ms < best) {
                    best = ms;
                    b->g_l2 = mult * cus;
                }
            }
            g_tune_cache[key] = {b->bm, b->g_gemm, b->g_c4, b->g_l2};
        }
        b->tuned = 1;
    }
    // capture the whole batched build once
    if (hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return cleanup_fail(bfail(b, CCH_E_HIP, "hipStreamBeginCapture failed"));
    rc = enqueue_batch(b);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->st, &g);
    if (rc != CCH_OK) {
        if (g) (void)hipGraphDestroy(g);
        return cleanup_fail(rc);
    }
    if (ce != hipSuccess || !g) return cleanup_fail(bfail(b, CCH_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ce)));
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
        return cleanup_fail(bfail(b, CCH_E_HIP, "hipGraphInstantiate failed"));
    (void)hipGraphGetNodes(b->graph, nullptr, &b->nodes);
    *out = b;
    return CCH_OK;
}

cch_status cch_batch_build(cch_batch *b)
{
    if (!b || !b->exec) return CCH_E_INVALID_ARG;
    BCK(b, hipSetDevice(b->device));
    for (cch_ctx *c : b->cs) BCK(b, hipStreamSynchronize(c->stream));
    BCK(b, hipEventRecord(b->e0, b->st));
    BCK(b, hipGraphLaunch(b->exec, b->st));
    BCK(b, hipEventRecord(b->e1, b->st));
    BCK(b, hipEventSynchronize(b->e1));
    BCK(b, hipEventElapsedTime(&b->last_ms, b->e0, b->e1));
    for (cch_ctx *c : b->cs) {
        c->built = true;
        ++c->build_gen;
        c->timed = false;
    }
    return CCH_OK;
}

cch_status cch_batch_time(const cch_batch *b, float *ms)
{
    if (!b || !ms) return CCH_E_INVALID_ARG;
    *ms = b->last_ms;
    return CCH_OK;
}

cch_status cch_batch_info(const cch_batch *b, int32_t *o)
{
    if (!b || !o) return CCH_E_INVALID_ARG;
    o[0] = b->bm;
    o[1] = b->g_gemm;
    o[2] = b->g_c4;
    o[3] = b->g_l2;
    o[4] = b->tuned;
    o[5] = b->cached;
    o[6] = (int32_t)b->nodes;
    o[7] = (int32_t)b->cs.size();
    return CCH_OK;
}

cch_status cch_batch_destroy(cch_batch *b)
{
    if (!b) return CCH_OK;
    (void)hipSetDevice(b->device);
    if (b->st) (void)hipStreamSynchronize(b->st);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void *p : b->allocs) (void)hipFree(p);
    if (b->e0) (void)hipEventDestroy(b->e0);
    if (b->e1) (void)hipEventDestroy(b->e1);
    if (b->st) (void)hipStreamDestroy(b->st);
    delete b;
    return CCH_OK;
}

const char *cch_batch_last_error(const cch_batch *b) { return b ? b->err.c_str() : g_create_err.c_str(); }

// ---------------------------------------------------------------------------
// block Davidson driver
//   basis V (m vectors) and W = H V are rotated to the Ritz basis after every
//   Rayleigh-Ritz step, so G = V^T H V is diag(theta) plus the rows of the
//   newest block; a thick restart keeps the lowest kr Ritz vectors.
//   New directions: diagonal (Jacobi) corrections, orthogonalised against V
//   by two classical Gram-Schmidt passes and inside the block by pivoted
//   Cholesky QR, twice.
// ---------------------------------------------------------------------------
namespace {
struct DavBufs {
    double *V = nullptr, *Wv = nullptr, *V2 = nullptr, *W2 = nullptr, *G = nullptr, *theta = nullptr,
           *Y = nullptr, *R = nullptr, *T = nullptr, *T2 = nullptr, *C = nullptr, *P0 = nullptr, *P1 = nullptr,
           *part = nullptr, *norms = nullptr, *Wp = nullptr, *rho = nullptr;
    int32_t *idx = nullptr, *nfb = nullptr, *rrfb = nullptr;
    float *mx = nullptr, *mg = nullptr;
};
}  // namespace

// Directions that carry the previous iteration's Ritz vectors over a restart.
// y holds kp rows of nt coefficients (row e: previous Ritz vector e along the
// nt discarded Ritz vectors, whose Ritz values are th). The rows are
// orthonormalised in order by modified Gram-Schmidt, twice; a row whose part
// left over is at most 1e-8 (the whole vector has norm 1) is dropped. q
// receives the kx orthonormal columns (q[j * ldq + e], j < nt), gx the
// projected block q^T diag(th) q (gx[e * ldg + f], symmetric). Returns kx.
static int restart_directions(const double *y, int nt, int kp, const double *th, double *q, int ldq, double *gx,
                              int ldg)
{
    std::vector<double> a(nt);
    int kx = 0;
    for (int e = 0; e < kp; ++e) {
        for (int j = 0; j < nt; ++j) a[j] = y[(int64_t)e * nt + j];
        for (int pass = 0; pass < 2; ++pass)
            for (int f = 0; f < kx; ++f) {
                double d = 0.0;
                for (int j = 0; j < nt; ++j) d += q[j * ldq + f] * a[j];
                for (int j = 0; j < nt; ++j) a[j] -= d * q[j * ldq + f];
            }
        double nrm = 0.0;
        for (int j = 0; j < nt; ++j) nrm += a[j] * a[j];
        nrm = std::sqrt(nrm);
        if (!(nrm > 1e-8)) continue;
        for (int j = 0; j < nt; ++j) q[j * ldq + kx] = a[j] / nrm;
        ++kx;
    }
    for (int e = 0; e < kx; ++e)
        for (int f = e; f < kx; ++f) {
            double s = 0.0;
            for (int j = 0; j < nt; ++j) s += q[j * ldq + e] * th[j] * q[j * ldq + f];
            gx[e * ldg + f] = s;
            gx[f * ldg + e] = s;
        }
    return kx;
}

// CSR of the L2 block of the current build (kept until the next build)
static cch_status ensure_l2csr(cch_ctx *c, hipStream_t st)
{
    if (c->csr.gen == c->build_gen) return CCH_OK;
    const int nl2 = c->n_l2r, Dc = (int)c->Dc;
    if (!c->csr.off && hipMalloc((void **)&c->csr.off, 8 * ((size_t)nl2 + 1)) != hipSuccess)
        return fail(c, CCH_E_OOM, "L2 row offsets");
    int64_t *cnt = nullptr;
    if (hipMalloc((void **)&cnt, 8 * (size_t)nl2) != hipSuccess) return fail(c, CCH_E_OOM, "L2 row counts");
    int64_t nnz = 0;
    hipError_t e = launch_l2_csr_count(c->d_H, c->ld, Dc, nl2, cnt, st);
    if (e == hipSuccess) e = launch_exclusive_scan(cnt, c->csr.off, nl2, c->csr.off + nl2, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&nnz, c->csr.off + nl2, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(cnt);
    if (e != hipSuccess) return fail(c, CCH_E_HIP, "L2 non-zero count: %s", hipGetErrorString(e));
    if (nnz > c->csr.cap) {
        (void)hipFree(c->csr.col);
        (void)hipFree(c->csr.val);
        c->csr.col = nullptr;
        c->csr.val = nullptr;
        c->csr.cap = 0;
        if (hipMalloc((void **)&c->csr.col, 4 * (size_t)std::max<int64_t>(nnz, 1)) != hipSuccess ||
            hipMalloc((void **)&c->csr.val, 8 * (size_t)std::max<int64_t>(nnz, 1)) != hipSuccess)
            return fail(c, CCH_E_OOM, "L2 CSR of %lld non-zeros", (long long)nnz);
        c->csr.cap = nnz;
    }
    HIPCK(c, launch_l2_csr_fill(c->d_H, c->ld, Dc, nl2, c->csr.off, c->csr.col, c->csr.val, st));
    c->csr.gen = c->build_gen;
    c->csr.nnz = nnz;
    return CCH_OK;
}

cch_status cch_davidson(cch_ctx *c, const cch_dav_opts *o, double *evals, double *evecs, cch_dav_info *info,
                        int32_t flags)
{
    if (!c || !o) return CCH_E_INVALID_ARG;
    if (!c->built) return fail(c, CCH_E_STATE, "build first");
    const int D = (int)c->D, k = o->k;
    if (k <= 0 || k > D) return fail(c, CCH_E_INVALID_ARG, "k out of range");
    if (k > 16) return fail(c, CCH_E_LIMIT, "k > 16 eigenpairs per solve");
    if (!(o->tol > 0.0)) return fail(c, CCH_E_INVALID_ARG, "tol must be positive");
    if (o->precond != CCH_PRECOND_JACOBI && o->precond != CCH_PRECOND_MLP)
        return fail(c, CCH_E_INVALID_ARG, "unknown preconditioner %d", o->precond);
    if (o->precond == CCH_PRECOND_MLP && !c->mlp) return fail(c, CCH_E_STATE, "no network attached (cch_davidson_set_mlp)");
    // default basis limit: max(8k, 64); from D = 20000 on the mat-vec outweighs
    // the Rayleigh-Ritz step, and the largest basis (fewer restarts) wins
    int mmax = o->max_subspace > 0 ? o->max_subspace : (D >= 20000 ? 96 : std::max(8 * k, 64));
    mmax = std::min(mmax, 96);
    mmax = std::min(mmax, D);
    const int k0 = std::min(2 * k, D);         // the first block
    if (k0 + k > mmax && mmax < D) return fail(c, CCH_E_INVALID_ARG, "k too large for the subspace limit");
    if (o->restart < CCH_RESTART_AUTO || o->restart > CCH_RESTART_PREV)
        return fail(c, CCH_E_INVALID_ARG, "unknown restart mode %d", o->restart);
    // a restart keeps the lowest kr Ritz vectors and, with the previous
    // iteration's Ritz vectors, up to kp more directions
    const bool prev = o->restart == CCH_RESTART_PREV || (o->restart == CCH_RESTART_AUTO && mmax >= 96);
    int kr = k0, kp = 0;
    if (prev && std::min(4 * k, mmax - 2 * k) >= 2 * k) {
        kr = std::min(4 * k, mmax - 2 * k);
        kp = k;
    }
    const int blk = o->block > 0 ? o->block : k;   // wanted + guard pairs corrected per iteration
    if (blk < k || blk > 16) return fail(c, CCH_E_INVALID_ARG, "block must lie in [k, 16]");
    const int max_iter = o->max_iter > 0 ? o->max_iter : 200;
    HIPCK(c, hipSetDevice(c->device));
    hipStream_t st = c->stream;
    auto t0 = std::chrono::steady_clock::now();
    // the L2 block as CSR in the mat-vec (formed here, inside the solve's time)
    const bool sparse = ((flags & CCH_DAV_SPARSE_L2) || c->sparse) && c->n_l2r > 0;
    if (sparse && !c->sparse) TRY(ensure_l2csr(c, st));

    const int64_t ldv = ((int64_t)D + 31) / 32 * 32;
    const int BMAX = 32;                       // block columns (<= 2k <= 32)
    std::vector<void *> tmp;
    void *tmp_host = nullptr;
    auto cleanup = [&]() {
        for (void *p : tmp) (void)hipFree(p);
        if (tmp_host) (void)hipHostFree(tmp_host);
        tmp_host = nullptr;
    };
    auto A = [&](void **p, size_t bytes) -> bool {
        if (hipMalloc(p, bytes ? bytes : 8) != hipSuccess) return false;
        tmp.push_back(*p);
        return true;
    };
    DavBufs b;
    const int nch = (D + 1023) / 1024;
    bool ok = A((void **)&b.V, 8 * ldv * mmax) && A((void **)&b.Wv, 8 * ldv * mmax) &&
              A((void **)&b.V2, 8 * ldv * mmax) && A((void **)&b.W2, 8 * ldv * mmax) &&
              A((void **)&b.G, 8 * (size_t)mmax * mmax) && A((void **)&b.theta, 8 * (size_t)mmax) &&
              A((void **)&b.Y, 8 * (size_t)mmax * mmax) && A((void **)&b.R, 8 * ldv * blk) &&
              A((void **)&b.T, 8 * ldv * BMAX) && A((void **)&b.T2, 8 * ldv * BMAX) &&
              A((void **)&b.C, 8 * (size_t)mmax * BMAX) && A((void **)&b.P0, 8 * (size_t)mmax * BMAX) &&
              A((void **)&b.P1, 8 * (size_t)mmax * BMAX) &&
              A((void **)&b.part, 8 * (size_t)std::max<int64_t>((int64_t)nch * mmax * 16, tn_part_doubles())) && A((void **)&b.norms, 8 * (size_t)blk) &&
              A((void **)&b.idx, 4 * (size_t)mmax) &&
              A((void **)&b.Wp, 8 * (size_t)std::max<int64_t>(matvec_scratch_doubles(D),
                                                                sparse ? l2csr_scratch(D, (int)c->Dc) : 0)) &&
              A((void **)&b.nfb, 4) &&
              A((void **)&b.rrfb, 4);
    const bool want_mlp = o->precond == CCH_PRECOND_MLP;
    if (ok && want_mlp)
        ok = A((void **)&b.rho, 8 * (size_t)D) && A((void **)&b.mx, 16 * (size_t)D * blk) &&
             A((void **)&b.mg, 4 * (size_t)D * blk);
    if (!ok) {
        cleanup();
        return fail(c, CCH_E_OOM, "Davidson buffers");
    }
#define DCK(x)                                                                                  \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) {                                                                 \
            cleanup();                                                                          \
            return fail(c, CCH_E_HIP, "%s: %s", #x, hipGetErrorString(e_));                    \
        }                                                                                       \
    } while (0)

    // initial block: the lowest 2k Ritz vectors of the principal submatrix on the
    // mmax smallest diagonal entries (ties: lower index)
    std::vector<double> hdiag(D);
    DCK(hipMemcpyAsync(hdiag.data(), c->d_diag, 8 * (size_t)D, hipMemcpyDeviceToHost, st));
    DCK(hipStreamSynchronize(st));
    int nb = k0;
    const int ns = std::min(mmax, D);
    // only the first ns of the order (by value, then index) are needed
    std::vector<int32_t> order(D);
    for (int i = 0; i < D; ++i) order[i] = i;
    std::partial_sort(order.begin(), order.begin() + ns, order.end(), [&](int a, int bb) {
        return hdiag[a] < hdiag[bb] || (!(hdiag[bb] < hdiag[a]) && a < bb);
    });
    DCK(hipMemcpy(b.idx, order.data(), 4 * (size_t)ns, hipMemcpyHostToDevice));
    if (c->sparse) DCK(launch_sparse_principal(sparse_mat(c), b.idx, ns, b.G, mmax, st));
    else DCK(launch_gather_principal(c->d_H, c->ld, b.idx, ns, b.G, mmax, st));
    DCK(launch_rr_eig(b.G, mmax, ns, b.theta, b.Y, mmax, b.rrfb, st));
    DCK(launch_fill_f64(b.T, 0.0, (int64_t)nb * ldv, st));
    DCK(launch_seed_scatter(b.T, ldv, b.idx, b.Y, mmax, ns, nb, st));

    int m = 0, iters = 0, matvecs = 0, nconv = 0, mv_launches = 0, fallbacks = 0;
    double mv_ms = 0.0, maxres = 0.0, best_res = 1e300, rr_ms = 0.0, rr_flops = 0.0;
    int rr_calls = 0, dropped = 0, restarts = 0, prev_kept = 0;
    bool use_mlp = want_mlp;
    if (want_mlp) {
        if (c->sparse) DCK(launch_sparse_row_norms(sparse_mat(c), D, b.rho, st));
        else DCK(launch_row_norms(c->d_H, c->ld, D, b.rho, st));
        DCK(hipMemsetAsync(b.nfb, 0, 4, st));
    }
    DCK(hipMemsetAsync(b.rrfb, 0, 4, st));
    // pinned, host-coherent block that the kernels write directly (the rank of
    // the new block, the residual norms): one synchronisation per iteration
    struct HostIO {
        int32_t rank;
        int32_t seq;   // written by the stream after each iteration's last kernel
        double res[16];
        // a restart with the previous Ritz vectors: rows of Y past the kept
        // columns, the discarded Ritz values, the orthonormal combination and
        // the projected block it gives
        double y[16 * 96], th[96], q[96 * 32], gx[16 * 16];
    };
    HostIO *hio = nullptr;
    int32_t seqno = 0;
    if (hipHostMalloc((void **)&hio, sizeof(HostIO), hipHostMallocCoherent) != hipSuccess) {
        cleanup();
        return fail(c, CCH_E_OOM, "pinned host buffer");
    }
    tmp_host = hio;
    __atomic_store_n(&hio->seq, 0, __ATOMIC_RELEASE);   // before any posted number
    double *hres = hio->res;
    DavSel sel{};
    cch_status rc = CCH_E_NOT_CONVERGED;
    // Rayleigh-Ritz on the leading m x m block of G, rotation of V and W to the
    // Ritz basis, residuals of the first kg pairs (norms to the host block)
    auto rayleigh_ritz = [&](int mm) -> hipError_t {
        hipError_t e;
        if ((e = hipEventRecord(c->rr0, st)) != hipSuccess) return e;
        if ((e = launch_rr_eig(b.G, mmax, mm, b.theta, b.Y, mmax, b.rrfb, st)) != hipSuccess) return e;
        if ((e = hipEventRecord(c->rr1, st)) != hipSuccess) return e;
        ++rr_calls;
        rr_flops += (10.0 / 3.0) * (double)mm * mm * mm;   // tridiagonalisation + back-transformation
        // V2 = V Y and W2 = W Y in one launch
        if ((e = launch_nn(b.V, ldv, mm, nullptr, 0, mm, D, b.Y, mmax, mm, nullptr, 0, 0.0, 1.0, b.V2, ldv, st, b.Wv,
                           b.W2)) != hipSuccess)
            return e;
        std::swap(b.V, b.V2);
        std::swap(b.Wv, b.W2);
        return launch_residual(b.Wv, b.V, ldv, D, b.theta, std::min(blk, mm), b.R, b.part, hres, st);
    };
    for (iters = 1; iters <= max_iter; ++iters) {
        // Orthogonalisation of the new block T against V and within itself:
        // [V | T]^T T in one product gives both the projection S = V^T T and the
        // Gram matrix T^T T; the pivoted Cholesky step then takes the Gram matrix
        // of T - V S as T^T T - S^T S and returns [-S B; B], so projection and
        // normalisation are one product [V | T] [-S B; B] = (T - V S) B.
        // First pass: project once explicitly, then once more folded into the
        // normalisation, with the drop test against the raw norms; the second
        // pass repeats project + normalise once (CholQR2 with re-projection).
        const double *ref = b.P0 + (int64_t)m * BMAX;   // diag of the raw T^T T, stride BMAX + 1
        DCK(launch_tn(b.V, ldv, m, b.T, ldv, m + nb, b.T, ldv, nb, D, b.part, b.P0, BMAX, 0, st));
        const double *P = b.P0;
        if (m > 0) {
            DCK(launch_nn(b.V, ldv, m, nullptr, 0, m, D, b.P0, BMAX, nb, b.T, ldv, 1.0, -1.0, b.T, ldv, st));
            DCK(launch_tn(b.V, ldv, m, b.T, ldv, m + nb, b.T, ldv, nb, D, b.part, b.P1, BMAX, 0, st));
            P = b.P1;
        }
        DCK(launch_pchol(P + (int64_t)m * BMAX, BMAX, nb, P, BMAX, m, ref, BMAX + 1, 1e-7, b.C, BMAX, &hio->rank,
                         st));
        DCK(launch_nn(b.V, ldv, m, b.T, ldv, m + nb, D, b.C, BMAX, nb, nullptr, 0, 0.0, 1.0, b.T2, ldv, st));
        DCK(launch_tn(b.V, ldv, m, b.T2, ldv, m + nb, b.T2, ldv, nb, D, b.part, b.P1, BMAX, 0, st));
        DCK(launch_pchol(b.P1 + (int64_t)m * BMAX, BMAX, nb, b.P1, BMAX, m, nullptr, 0, 1e-12, b.C, BMAX,
                         &hio->rank, st));
        // the orthonormal block goes straight into V; columns past the rank are zero
        DCK(launch_nn(b.V, ldv, m, b.T2, ldv, m + nb, D, b.C, BMAX, nb, nullptr, 0, 0.0, 1.0, b.V + (int64_t)m * ldv,
                      ldv, st));
        // W for the new vectors and the new rows of G, taking all nb directions as
        // kept; the rank is read with the residual norms below
        const int m0 = m;
        DCK(hipEventRecord(c->mv0, st));
        if (sparse)
            DCK(launch_matvec_l2csr(c->d_H, c->ld, c->sparse ? c->d_R : c->d_H, c->sparse ? c->ldr : c->ld,
                                    c->sparse ? (int)c->Dc : 0, D, (int)c->Dc, c->csr.off, c->csr.col, c->csr.val,
                                    b.V + (int64_t)m * ldv, ldv, nb, b.Wv + (int64_t)m * ldv, ldv, b.Wp, st));
        else
            DCK(launch_matvec(c->d_H, c->ld, D, b.V + (int64_t)m * ldv, ldv, nb, b.Wv + (int64_t)m * ldv, ldv, b.Wp,
                              st));
        DCK(hipEventRecord(c->mv1, st));
        matvecs += nb;
        mv_launches += (nb + 15) / 16;
        // rows m.. of G and their mirror in the columns m.. of the rows before m
        DCK(launch_tn(b.Wv + (int64_t)m * ldv, ldv, nb, nullptr, 0, nb, b.V, ldv, m + nb, D, b.part,
                      b.G + (int64_t)m * mmax, mmax, 0, st, b.G + m, m));
        m = m0 + nb;
        DCK(rayleigh_ritz(m));
        // the stream posts the iteration's number into the pinned block after its
        // last kernel; the host spins on it (bounded), then falls back to a
        // stream synchronisation, which also covers a missed post
        ++seqno;
        DCK(hipStreamWriteValue32(st, &hio->seq, (uint32_t)seqno, 0));
        {
            bool seen = false;
            const auto ts = std::chrono::steady_clock::now();
            for (int spin = 0; !seen; ++spin) {
                seen = __atomic_load_n(&hio->seq, __ATOMIC_ACQUIRE) == seqno;
                if (!seen && (spin & 1023) == 1023 &&
                    std::chrono::steady_clock::now() - ts > std::chrono::milliseconds(20))
                    break;
            }
            if (!seen) DCK(hipStreamSynchronize(st));
        }
        {
            float ms = 0.0f;
            DCK(hipEventSynchronize(c->rr1));
            DCK(hipEventElapsedTime(&ms, c->mv0, c->mv1));
            mv_ms += ms;
            DCK(hipEventElapsedTime(&ms, c->rr0, c->rr1));
            rr_ms += ms;
        }
        const int added = hio->rank;
        if (added < nb) {
            dropped += nb - std::max(added, 0);
            // dropped directions: V holds zero columns past the rank. Back to the
            // basis before the rotation; the leading m0 + added block of G is
            // exact (G was diag(theta) on the first m0), so Rayleigh-Ritz is redone
            // on it. No new direction at all: stagnation, stop there.
            std::swap(b.V, b.V2);
            std::swap(b.Wv, b.W2);
            m = m0 + std::max(added, 0);
            if (m > 0) {
                DCK(rayleigh_ritz(m));
                DCK(hipStreamSynchronize(st));
                float ms = 0.0f;
                DCK(hipEventElapsedTime(&ms, c->rr0, c->rr1));
                rr_ms += ms;
            }
            if (added <= 0) break;
        }
        const int kk = std::min(k, m), kg = std::min(blk, m);
        std::vector<int32_t> un;
        maxres = 0.0;
        for (int e = 0; e < kk; ++e) {
            maxres = std::max(maxres, hres[e]);
            if (!(hres[e] <= o->tol)) un.push_back(e);
        }
        nconv = kk - (int)un.size();
        if (!un.empty())   // guard pairs ride along in the same mat-vec pass
            for (int e = kk; e < kg; ++e)
                if (!(hres[e] <= o->tol)) un.push_back(e);
        // judge of the learned step: a residual that grows tenfold over the best so far
        // switches the rest of the solve to the diagonal step
        if (use_mlp && iters > 3 && maxres > 10.0 * best_res) {
            use_mlp = false;
            ++fallbacks;
        }
        best_res = std::min(best_res, maxres);
        if (kk == k && un.empty()) {
            rc = CCH_OK;
            break;
        }
        if (m >= D) {   // the whole space is spanned: the Ritz pairs are exact
            rc = CCH_OK;
            nconv = kk;
            break;
        }
        // G in the rotated basis
        if (m + (int)un.size() > mmax) {
            const int mold = m;
            m = std::min(kr, m);
            ++restarts;
            // the previous iteration's lowest kp Ritz vectors are the first kp
            // vectors of the basis this iteration started from, rows of Y; their
            // parts outside the kept Ritz vectors lie in the span of the
            // discarded ones, columns m..mold-1 of Y
            int kx = 0;
            const int nt = mold - m;
            if (kp > 0 && m0 >= kp && nt > 0) {
                DCK(hipMemcpy2DAsync(hio->y, 8 * (size_t)nt, b.Y + m, 8 * (size_t)mmax, 8 * (size_t)nt, kp,
                                     hipMemcpyDeviceToHost, st));
                DCK(hipMemcpyAsync(hio->th, b.theta + m, 8 * (size_t)nt, hipMemcpyDeviceToHost, st));
                DCK(hipStreamSynchronize(st));
                kx = restart_directions(hio->y, nt, kp, hio->th, hio->q, BMAX, hio->gx, 16);
            }
            DCK(launch_g_ritz(b.G, mmax, m + kx, b.theta, st));
            if (kx > 0) {
                // V, W rows m..m+kx-1 = the discarded Ritz vectors times Q (formed
                // beside, then copied in); G's block there = Q^T diag(theta) Q
                DCK(hipMemcpyAsync(b.C, hio->q, 8 * (size_t)nt * BMAX, hipMemcpyHostToDevice, st));
                DCK(launch_nn(b.V + (int64_t)m * ldv, ldv, nt, nullptr, 0, nt, D, b.C, BMAX, kx, nullptr, 0, 0.0, 1.0,
                              b.V2 + (int64_t)m * ldv, ldv, st, b.Wv + (int64_t)m * ldv, b.W2 + (int64_t)m * ldv));
                DCK(hipMemcpy2DAsync(b.V + (int64_t)m * ldv, 8 * ldv, b.V2 + (int64_t)m * ldv, 8 * ldv, 8 * (size_t)D,
                                     kx, hipMemcpyDeviceToDevice, st));
                DCK(hipMemcpy2DAsync(b.Wv + (int64_t)m * ldv, 8 * ldv, b.W2 + (int64_t)m * ldv, 8 * ldv,
                                     8 * (size_t)D, kx, hipMemcpyDeviceToDevice, st));
                DCK(hipMemcpy2DAsync(b.G + (int64_t)m * mmax + m, 8 * (size_t)mmax, hio->gx, 8 * 16, 8 * (size_t)kx,
                                     kx, hipMemcpyHostToDevice, st));
                m += kx;
                prev_kept += kx;
            }
        } else {
            DCK(launch_g_ritz(b.G, mmax, m, b.theta, st));
        }
        // corrections for the unconverged pairs (never more than the basis has room for)
        nb = std::min((int)un.size(), mmax - m);
        if (nb <= 0) break;
        for (int e = 0; e < nb; ++e) sel.e[e] = un[e];
        if (use_mlp) {
            const cch_mlp *net = c->mlp;
            DCK(launch_mlp_dav(net->w, net->w2, net->w2t, b.R, ldv, D, (int)c->Dc, c->d_diag, b.rho, b.theta, sel, nb,
                               b.mx, b.mg, b.T, ldv, b.nfb, st));
        } else {
            DCK(launch_jacobi_correct(b.R, ldv, D, c->d_diag, b.theta, sel, nb, b.T, ldv, st));
        }
    }
    if (iters > max_iter) iters = max_iter;
    const int kk = std::min(k, m);
    if (evals) {
        std::vector<double> th(kk);
        DCK(hipMemcpyAsync(th.data(), b.theta, 8 * (size_t)kk, hipMemcpyDeviceToHost, st));
        DCK(hipStreamSynchronize(st));
        if (flags & CCH_MEM_DEVICE) DCK(hipMemcpy(evals, th.data(), 8 * (size_t)kk, hipMemcpyHostToDevice));
        else memcpy(evals, th.data(), 8 * (size_t)kk);
    }
    int32_t elem_fb = 0, rr_fb = 0;
    if (want_mlp) DCK(hipMemcpyAsync(&elem_fb, b.nfb, 4, hipMemcpyDeviceToHost, st));
    DCK(hipMemcpyAsync(&rr_fb, b.rrfb, 4, hipMemcpyDeviceToHost, st));
    DCK(hipStreamSynchronize(st));
    if (evecs) {
        const hipMemcpyKind kind = (flags & CCH_MEM_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        DCK(hipMemcpy2DAsync(evecs, 8 * (size_t)D, b.V, ldv * 8, 8 * (size_t)D, kk, kind, st));
        if (flags & CCH_DAV_RESIDUALS) {
            // residuals of the returned Ritz pairs (b.R holds those of the last Rayleigh-Ritz step)
            DCK(launch_residual(b.Wv, b.V, ldv, D, b.theta, kk, b.R, b.part, b.norms, st));
            DCK(hipMemcpy2DAsync(evecs + (size_t)k * D, 8 * (size_t)D, b.R, ldv * 8, 8 * (size_t)D, kk, kind, st));
        }
    }
    DCK(hipStreamSynchronize(st));
    cleanup();
    if (info) {
        info->iterations = iters;
        info->matvecs = matvecs;
        info->converged = nconv;
        info->fallbacks = fallbacks + (elem_fb > 0 ? 1 : 0);
        info->max_residual = maxres;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->matvec_ms = mv_ms;
        info->matvec_launches = mv_launches;
        info->rr_fallbacks = rr_fb;
        info->rr_ms = rr_ms;
        info->rr_flops = rr_flops;
        info->rr_calls = rr_calls;
        info->dropped = dropped;
        info->restarts = restarts;
        info->prev_kept = prev_kept;
    }
    if (rc != CCH_OK) fail(c, rc, "Davidson did not converge in %d iterations (max residual %.3e)", max_iter, maxres);
    return rc;
}
