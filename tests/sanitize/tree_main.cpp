// Host driver for the sanitizer build of the library's tree code
// (csrc/tree.cpp): trees, lists and constraint graphs of several point sets,
// every graph DSatur-colored, the uniform graphs, and a forest.  Run under
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitize.py;
// any report ends the run with a nonzero status.
//
//   tree_main <points.f64> <n> <dim> <leaf> <kind> <adm>   (repeatable groups)
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hm_internal.h"

static int color_all(hm::Tree &T) {
  int ncol = 0;
  for (hm::Graph &G : T.graphs) {
    G.color.assign(G.nv(), -1);
    G.ncolors = hm::dsatur(G.nv(), G.xadj.data(), G.adj.data(), G.color.data());
    G.colored = true;
    ncol += G.ncolors;
  }
  return ncol;
}

int main(int argc, char **argv) {
  if ((argc - 1) % 6 != 0 || argc < 7) {
    std::fprintf(stderr, "usage: tree_main (points n dim leaf kind adm)...\n");
    return 2;
  }
  for (int a = 1; a < argc; a += 6) {
    const long n = std::atol(argv[a + 1]);
    const int dim = std::atoi(argv[a + 2]), leaf = std::atoi(argv[a + 3]);
    const int kind = std::atoi(argv[a + 4]), adm = std::atoi(argv[a + 5]);
    std::vector<double> pts((size_t)n * dim);
    FILE *f = std::fopen(argv[a], "rb");
    if (!f || std::fread(pts.data(), sizeof(double), pts.size(), f) != pts.size()) {
      std::fprintf(stderr, "cannot read %s\n", argv[a]);
      return 2;
    }
    std::fclose(f);
    hm::Tree T;
    if (hm::build_tree(pts.data(), n, dim, leaf, kind, adm, T) != HM_OK) {
      std::fprintf(stderr, "build_tree failed on %s\n", argv[a]);
      return 3;
    }
    const int ncol = color_all(T);
    int nucol = 0;
    if (adm == HM_ADM_STRONG && kind == HM_TREE_GEOMETRIC) {
      hm::build_uniform_graphs(T);
      for (const hm::Graph &G : T.ugraphs) nucol += G.ncolors;
    }
    // the same points as a forest of three instances
    const int64_t counts[3] = {n / 3, n / 3, n - 2 * (n / 3)};
    hm::Tree F;
    if (hm::build_forest(pts.data(), counts, 3, dim, leaf, kind, adm, F) != HM_OK) {
      std::fprintf(stderr, "build_forest failed on %s\n", argv[a]);
      return 3;
    }
    const int fcol = color_all(F);
    std::printf("%s: n=%ld dim=%d levels=%d colors=%d uniform_colors=%d forest_levels=%d "
                "forest_colors=%d\n",
                argv[a], n, dim, T.nlev(), ncol, nucol, F.nlev(), fcol);
  }
  return 0;
}
