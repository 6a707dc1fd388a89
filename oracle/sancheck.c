/* Sanitizer driver for the CPU oracle: TEST INFRASTRUCTURE ONLY.
 *
 * The CPU tests compile this file together with ccoracle.c under
 * AddressSanitizer and UndefinedBehaviorSanitizer (gcc) and run it on small
 * instances: every input array sits in a heap block of exactly its own size,
 * so a read past the end of an integral, determinant or CI array, an
 * unaligned or overflowing index, or a use of freed memory stops the run.
 * The outputs are written back so the test can check that the sanitized
 * build gives the same matrix as the ordinary one.
 *
 * Input file: a sequence of records, each an int64 byte count followed by
 * that many bytes, in this order:
 *   int32 header[10]: n_o, n_cont, n_elec, n_words, n_sym, n_l2,
 *                     total_irrep, n_irrep, packed, n_sample
 *   double e_core
 *   double h, tttt, tttc, ttcc, tctc
 *   (packed only) int64 pk_rec, pk_blk; int32 t_irrep, c_irrep, c_local, c_count
 *   int32 cont_start, sym_irrep, sym_ndet, sym_nstate
 *   per symmetry: uint64 dets, double ci
 *   uint64 l2_dets
 *   int64 sample rows, sample cols
 * Output file: the full D x D matrix (row-major doubles), then the n_sample
 * sampled elements, then the excitation pairs of the first symmetry with
 * itself (lower triangle) and of the L2 determinants with the first
 * symmetry's determinants (each: count, then x, y, degree, sign per pair).
 */
#include <stdio.h>

#include "ccoracle.c"

static void *read_record(FILE *f, int64_t *nbytes)
{
    int64_t n = 0;
    if (fread(&n, sizeof n, 1, f) != 1 || n < 0) {
        fprintf(stderr, "sancheck: truncated input\n");
        exit(2);
    }
    /* malloc(0) may return NULL; keep a distinct block so NULL means absent */
    void *p = malloc(n > 0 ? (size_t)n : 1);
    if (!p || (n > 0 && fread(p, 1, (size_t)n, f) != (size_t)n)) {
        fprintf(stderr, "sancheck: truncated input\n");
        exit(2);
    }
    if (nbytes) *nbytes = n;
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: sancheck <instance file> <output file>\n");
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t nb = 0;
    int32_t *hd = read_record(f, &nb);
    if (nb != 10 * (int64_t)sizeof(int32_t)) return 2;
    double *ecore = read_record(f, NULL);

    orc_inst I;
    memset(&I, 0, sizeof I);
    I.ints.n_o = hd[0];
    I.ints.n_cont = hd[1];
    I.n_elec = hd[2];
    I.n_words = hd[3];
    I.n_sym = hd[4];
    I.n_l2 = hd[5];
    I.total_irrep = hd[6];
    I.ints.n_irrep = hd[7];
    const int packed = hd[8], n_sample = hd[9];
    I.ints.e_core = *ecore;
    I.ints.h = read_record(f, NULL);
    I.ints.tttt = read_record(f, NULL);
    I.ints.tttc = read_record(f, NULL);
    I.ints.ttcc = read_record(f, NULL);
    I.ints.tctc = read_record(f, NULL);
    if (packed) {
        I.ints.pk_rec = read_record(f, NULL);
        I.ints.pk_blk = read_record(f, NULL);
        I.ints.t_irrep = read_record(f, NULL);
        I.ints.c_irrep = read_record(f, NULL);
        I.ints.c_local = read_record(f, NULL);
        I.ints.c_count = read_record(f, NULL);
    }
    I.cont_start = read_record(f, NULL);
    I.sym_irrep = read_record(f, NULL);
    I.sym_ndet = read_record(f, NULL);
    I.sym_nstate = read_record(f, NULL);
    const uint64_t **dets = malloc(sizeof(void *) * (I.n_sym > 0 ? I.n_sym : 1));
    const double **ci = malloc(sizeof(void *) * (I.n_sym > 0 ? I.n_sym : 1));
    for (int s = 0; s < I.n_sym; ++s) {
        dets[s] = read_record(f, NULL);
        ci[s] = read_record(f, NULL);
    }
    I.sym_dets = dets;
    I.sym_ci = ci;
    I.l2_dets = read_record(f, NULL);
    const int64_t *rows = read_record(f, NULL);
    const int64_t *cols = read_record(f, NULL);
    fclose(f);

    const int64_t D = orc_dim(&I);
    double *H = malloc(sizeof(double) * (size_t)(D * D > 0 ? D * D : 1));
    double *Ha = malloc(sizeof(double) * (size_t)(D * D > 0 ? D * D : 1));
    int32_t *Hc = malloc(sizeof(int32_t) * (size_t)(D * D > 0 ? D * D : 1));
    orc_build(&I, 0, D, H, Ha, Hc);
    double *v = malloc(sizeof(double) * (n_sample > 0 ? n_sample : 1));
    double *va = malloc(sizeof(double) * (n_sample > 0 ? n_sample : 1));
    int32_t *vc = malloc(sizeof(int32_t) * (n_sample > 0 ? n_sample : 1));
    orc_elements(&I, n_sample, rows, cols, v, va, vc);

    /* excitation pairs: the first symmetry with itself, the L2 determinants
     * with the first symmetry */
    int64_t np[2] = {0, 0};
    int32_t *px[2] = {NULL, NULL}, *py[2] = {NULL, NULL};
    int8_t *pdeg[2] = {NULL, NULL}, *ph[2] = {NULL, NULL};
    if (I.n_sym > 0) {
        const int nd = I.sym_ndet[0];
        const int64_t cap[2] = {(int64_t)nd * nd, (int64_t)nd * I.n_l2};
        for (int w = 0; w < 2; ++w) {
            const size_t c = (size_t)(cap[w] > 0 ? cap[w] : 1);
            px[w] = malloc(sizeof(int32_t) * c);
            py[w] = malloc(sizeof(int32_t) * c);
            pdeg[w] = malloc(c);
            ph[w] = malloc(c);
            uint64_t *lab = malloc(sizeof(uint64_t) * c);
            if (w == 0)
                np[0] = orc_pairs(I.sym_dets[0], nd, I.sym_dets[0], nd, I.n_words, 1, cap[0], px[0], py[0],
                                  pdeg[0], lab, ph[0]);
            else
                np[1] = orc_pairs_l2tgt(I.l2_dets, I.n_l2, I.sym_dets[0], nd, I.n_words, 2 * I.ints.n_o, cap[1],
                                        px[1], py[1], pdeg[1], lab, ph[1]);
            free(lab);
        }
    }

    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(H, sizeof(double), (size_t)(D * D), o);
    fwrite(v, sizeof(double), (size_t)n_sample, o);
    for (int w = 0; w < 2; ++w) {
        fwrite(&np[w], sizeof(int64_t), 1, o);
        if (np[w] > 0) {
            fwrite(px[w], sizeof(int32_t), (size_t)np[w], o);
            fwrite(py[w], sizeof(int32_t), (size_t)np[w], o);
            fwrite(pdeg[w], 1, (size_t)np[w], o);
            fwrite(ph[w], 1, (size_t)np[w], o);
        }
    }
    fclose(o);

    for (int w = 0; w < 2; ++w) { free(px[w]); free(py[w]); free(pdeg[w]); free(ph[w]); }
    free(H); free(Ha); free(Hc); free(v); free(va); free(vc);
    free((void *)rows); free((void *)cols);
    for (int s = 0; s < I.n_sym; ++s) { free((void *)dets[s]); free((void *)ci[s]); }
    free(dets); free(ci);
    free((void *)I.l2_dets);
    free((void *)I.cont_start); free((void *)I.sym_irrep); free((void *)I.sym_ndet); free((void *)I.sym_nstate);
    if (packed) {
        free((void *)I.ints.pk_rec); free((void *)I.ints.pk_blk); free((void *)I.ints.t_irrep);
        free((void *)I.ints.c_irrep); free((void *)I.ints.c_local); free((void *)I.ints.c_count);
    }
    free((void *)I.ints.h); free((void *)I.ints.tttt); free((void *)I.ints.tttc);
    free((void *)I.ints.ttcc); free((void *)I.ints.tctc);
    free(ecore); free(hd);
    return 0;
}
