/* Host driver for the sanitizer build of the oracle's combinatorics
 * (oracle/comb.c): tree, lists, every constraint graph and its DSatur
 * coloring for several point sets.  Run under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitize.py.
 *
 *   comb_main <points.f64> <n> <dim> <leaf> <index_binary> <weak>   (repeatable) */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void *orc_build(const double *pts, int64_t n, int dim, int leaf, int index_binary, int weak);
int orc_nlev(void *t);
void orc_graph_sizes(void *t, int g, int *nv, int64_t *nadj, int *nset, int *npairs);
void orc_graph(void *t, int g, int *vbox, int *vset_ptr, int *vset, int64_t *xadj, int *adj,
               int *pa, int *pb, int *pv);
int orc_dsatur(int nv, const int64_t *xadj, const int *adj, int *color);
void orc_free(void *t);

int main(int argc, char **argv) {
  if ((argc - 1) % 6 != 0 || argc < 7) {
    fprintf(stderr, "usage: comb_main (points n dim leaf index_binary weak)...\n");
    return 2;
  }
  for (int a = 1; a < argc; a += 6) {
    const int64_t n = atol(argv[a + 1]);
    const int dim = atoi(argv[a + 2]), leaf = atoi(argv[a + 3]);
    const int ib = atoi(argv[a + 4]), weak = atoi(argv[a + 5]);
    double *pts = malloc(sizeof(double) * (size_t)(n * dim));
    FILE *f = fopen(argv[a], "rb");
    if (!pts || !f || fread(pts, sizeof(double), (size_t)(n * dim), f) != (size_t)(n * dim)) {
      fprintf(stderr, "cannot read %s\n", argv[a]);
      return 2;
    }
    fclose(f);
    void *T = orc_build(pts, n, dim, leaf, ib, weak);
    const int nlev = orc_nlev(T);
    int total = 0;
    for (int g = 0; g <= nlev; ++g) {  /* level graphs, then the leaf graph */
      int nv, nset, np;
      int64_t nadj;
      orc_graph_sizes(T, g, &nv, &nadj, &nset, &np);
      int *vbox = malloc(sizeof(int) * (size_t)(nv + 1));
      int *vptr = malloc(sizeof(int) * (size_t)(nv + 1));
      int *vset = malloc(sizeof(int) * (size_t)(nset + 1));
      int64_t *xadj = malloc(sizeof(int64_t) * (size_t)(nv + 1));
      int *adj = malloc(sizeof(int) * (size_t)(nadj + 1));
      int *pa = malloc(sizeof(int) * (size_t)(np + 1));
      int *pb = malloc(sizeof(int) * (size_t)(np + 1));
      int *pv = malloc(sizeof(int) * (size_t)(np + 1));
      int *col = malloc(sizeof(int) * (size_t)(nv + 1));
      orc_graph(T, g, vbox, vptr, vset, xadj, adj, pa, pb, pv);
      total += nv > 0 ? orc_dsatur(nv, xadj, adj, col) : 0;
      free(vbox); free(vptr); free(vset); free(xadj); free(adj);
      free(pa); free(pb); free(pv); free(col);
    }
    orc_free(T);
    free(pts);
    printf("%s: n=%ld levels=%d colors=%d\n", argv[a], (long)n, nlev, total);
  }
  return 0;
}
