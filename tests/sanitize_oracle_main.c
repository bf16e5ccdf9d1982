/* Driver of the CPU oracle for the AddressSanitizer / UndefinedBehavior-
 * Sanitizer build of tests/test_sanitize.py.
 * usage: sanitize_oracle_main <graph.bin> <out.bin>
 * graph.bin: uint32 n, uint32 row_ptr[n+1], uint32 col_idx[row_ptr[n]].
 * out.bin: induced counts (n x 73), non-induced counts (n x 73), edge counts
 * (2m x 12), rooted counts of every vertex with a budget of 50 subsets
 * (n x 73) and their completion flags (n bytes). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_induced_counts(const uint32_t *rp, const uint32_t *ci, uint32_t n, int kmax,
                          uint64_t *counts, int nthreads);
int oracle_noninduced_counts(const uint32_t *rp, const uint32_t *ci, uint32_t n, int kmax,
                             uint64_t *counts, int nthreads);
int oracle_edge_counts(const uint32_t *rp, const uint32_t *ci, uint32_t n, uint64_t *ecounts,
                       int nthreads);
int oracle_rooted_counts(const uint32_t *rp, const uint32_t *ci, uint32_t n, int kmax,
                         const uint32_t *roots, uint32_t nroots, uint64_t budget,
                         uint64_t *counts, uint8_t *complete, int nthreads);

static void *read_exact(FILE *f, size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    uint32_t n = 0;
    if (fread(&n, 4, 1, f) != 1) return 2;
    uint32_t *rp = read_exact(f, 4ull * (n + 1));
    uint32_t *ci = read_exact(f, 4ull * rp[n]);
    fclose(f);
    const size_t rows = (size_t)n * 73, erows = (size_t)rp[n] * 12;
    uint64_t *ind = calloc(rows + 1, 8), *non = calloc(rows + 1, 8), *edg = calloc(erows + 1, 8),
             *root = calloc(rows + 1, 8);
    uint8_t *done = calloc(n + 1, 1);
    uint32_t *roots = malloc(4ull * (n + 1));
    for (uint32_t i = 0; i < n; i++) roots[i] = i;
    int rc = oracle_induced_counts(rp, ci, n, 5, ind, 4);
    if (!rc) rc = oracle_noninduced_counts(rp, ci, n, 5, non, 2);
    if (!rc) rc = oracle_edge_counts(rp, ci, n, edg, 3);
    if (!rc) rc = oracle_rooted_counts(rp, ci, n, 5, roots, n, 50, root, done, 4);
    if (rc) {
        fprintf(stderr, "oracle status %d\n", rc);
        return 3;
    }
    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(ind, 8, rows, o);
    fwrite(non, 8, rows, o);
    fwrite(edg, 8, erows, o);
    fwrite(root, 8, rows, o);
    fwrite(done, 1, n, o);
    fclose(o);
    free(rp); free(ci); free(ind); free(non); free(edg); free(root); free(done); free(roots);
    return 0;
}
