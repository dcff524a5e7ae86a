// Host combinatorics of colored peeling: box tree, neighbor / interaction
// lists, constraint incompatibility graphs and DSatur coloring.
//
// Paper: Levitt & Martinsson, arXiv 2205.03406 -- section "Rank-structured
// matrices" (tree and lists), eq:h1constraints and def:incompatibility_graph
// (level graphs), the leaf-extraction section (leaf graph), alg:dsatur.
//
// Design notes: this runs on the host once per geometry.  It
// works level by level with candidate sets drawn from the parent level
// (a box's neighbors are among the children of its parent's neighbors), so
// the cost is O(N log N + boxes * 6^d + edges) rather than quadratic.
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <tuple>
#include <unordered_map>

#include "hm_internal.h"

namespace hm {

// Set on the threads of a forest build's pool: the trees they build use no
// worker threads of their own (the pool already holds the CPUs).
static thread_local bool t_in_pool = false;

int host_threads() {
  cpu_set_t set;
  int n = 0;
  if (sched_getaffinity(0, sizeof(set), &set) == 0) n = CPU_COUNT(&set);
  if (n <= 0) n = (int)std::thread::hardware_concurrency();
  return std::max(1, std::min(n, 16));
}

namespace {

// Key bits per coordinate: 21 for d <= 3, floor(63 / d) for 4 <= d <= 8, so
// that the interleaved key of all coordinates fits 64 bits.
int key_bits(int dim) { return dim <= 3 ? 21 : 63 / dim; }

// Spread the low kb bits of v so that bit i lands at bit i*stride
// (shift-and-mask interleave for strides 1, 2 and 3 with 21 bits, a bit
// loop for wider strides).
uint64_t spread(uint32_t v, int stride, int kb) {
  uint64_t x = v & ((1u << kb) - 1);
  if (stride > 3) {
    uint64_t y = 0;
    for (int b = 0; b < kb; ++b) y |= ((x >> b) & 1u) << (b * stride);
    return y;
  }
  if (stride == 2) {
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
  } else if (stride == 3) {
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
  }
  return x;
}

// Integer cell of one coordinate: floor(((x - lo) / s) * 2^kb), clamped.
// x >= lo, so the quotient is non-negative and truncation is the floor; the
// division and the (exact) power-of-two product are separate roundings.
uint32_t cell(double x, double lo, double s, int kb) {
  const uint32_t top = (1u << kb) - 1;
  const double t = ((x - lo) / s) * std::ldexp(1.0, kb);
  if (t >= double(top)) return top;
  return uint32_t(t);
}

struct Builder {
  Tree &T;
  int workers = 1;  // threads per graph's edge passes
  explicit Builder(Tree &t) : T(t) {}

  // children[l][P] = boxes of level l+1 whose parent is P
  std::vector<std::vector<int32_t>> kids_ptr, kids;

  void child_index(int l) {  // children of level-l boxes (needs level l+1)
    const Level &C = T.lev[l + 1];
    int nbp = T.lev[l].nbox();
    std::vector<int32_t> ptr(nbp + 1, 0), idx(C.nbox());
    for (int b = 0; b < C.nbox(); ++b) ptr[C.parent[b] + 1]++;
    for (int P = 0; P < nbp; ++P) ptr[P + 1] += ptr[P];
    std::vector<int32_t> pos(ptr.begin(), ptr.end() - 1);
    for (int b = 0; b < C.nbox(); ++b) idx[pos[C.parent[b]]++] = b;
    kids_ptr[l] = std::move(ptr);
    kids[l] = std::move(idx);
  }

  void geometric(const double *pts) {
    const int64_t n = T.n;
    const int dim = T.dim;
    const int kb = T.kbits, os = T.ostride;
    double lo[8] = {0}, hi[8] = {0};
    for (int d = 0; d < dim; ++d) lo[d] = hi[d] = pts[d];
    for (int64_t i = 1; i < n; ++i)
      for (int d = 0; d < dim; ++d) {
        lo[d] = std::min(lo[d], pts[i * dim + d]);
        hi[d] = std::max(hi[d], pts[i * dim + d]);
      }
    double s = 0;
    for (int d = 0; d < dim; ++d) s = std::max(s, hi[d] - lo[d]);
    if (!(s > 0)) s = 1.0;
    std::vector<std::pair<uint64_t, int64_t>> key(n);
    std::vector<uint32_t> cells(n * dim);
    for (int64_t i = 0; i < n; ++i) {
      uint64_t k = 0;
      for (int d = 0; d < dim; ++d) {
        uint32_t c = cell(pts[i * dim + d], lo[d], s, kb);
        cells[i * dim + d] = c;
        k |= spread(c, dim, kb) << d;
      }
      key[i] = {k, i};
    }
    std::sort(key.begin(), key.end());
    T.perm.resize(n);
    std::vector<uint64_t> skey(n);
    for (int64_t i = 0; i < n; ++i) {
      T.perm[i] = key[i].second;
      skey[i] = key[i].first;
    }
    // level 0: the root cube
    Level root;
    root.start = {0, n};
    root.parent = {-1};
    root.org.assign(T.ostride, 0);
    root.blev = {0};
    T.lev.push_back(std::move(root));
    const int m = T.leaf;
    for (int l = 0; l < kb; ++l) {
      const Level &P = T.lev[l];
      bool split_any = false;
      for (int b = 0; b < P.nbox(); ++b)
        if (P.start[b + 1] - P.start[b] > m) split_any = true;
      if (!split_any) break;
      Level C;
      const int shift = (kb - 1 - l) * dim;  // key bits below the child digit
      for (int b = 0; b < P.nbox(); ++b) {
        int64_t s0 = P.start[b], s1 = P.start[b + 1];
        if (s1 - s0 <= m) {  // leaf: carried to the next level unchanged
          C.start.push_back(s0);
          C.parent.push_back(b);
          for (int d = 0; d < os; ++d) C.org.push_back(P.org[os * b + d]);
          C.blev.push_back(P.blev[b]);
          continue;
        }
        // runs of equal key prefix are the non-empty children, in order
        int64_t i = s0;
        while (i < s1) {
          uint64_t pre = skey[i] >> shift;
          int64_t j = i + 1;
          while (j < s1 && (skey[j] >> shift) == pre) ++j;
          int digit = int(pre & ((uint64_t(1) << dim) - 1));
          C.start.push_back(i);
          C.parent.push_back(b);
          for (int d = 0; d < os; ++d) {
            int64_t o = P.org[os * b + d];
            if (d < dim && ((digit >> d) & 1)) o += int64_t(1) << (kb - 1 - l);
            C.org.push_back(o);
          }
          C.blev.push_back(l + 1);
          i = j;
        }
      }
      C.start.push_back(n);
      T.lev.push_back(std::move(C));
    }
  }

  void index_binary(const double *pts) {
    const int64_t n = T.n;
    std::vector<int64_t> order(n);
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return pts[a * T.dim] < pts[b * T.dim]; });
    T.perm = order;
    Level root;
    root.start = {0, n};
    root.parent = {-1};
    root.org.assign(T.ostride, 0);
    root.blev = {0};
    T.lev.push_back(std::move(root));
    const int m = T.leaf;
    for (int l = 0;; ++l) {
      const Level &P = T.lev[l];
      bool split_any = false;
      for (int b = 0; b < P.nbox(); ++b)
        if (P.start[b + 1] - P.start[b] > m) split_any = true;
      if (!split_any) break;
      Level C;
      for (int b = 0; b < P.nbox(); ++b) {
        int64_t s0 = P.start[b], s1 = P.start[b + 1];
        bool split = s1 - s0 > m;
        C.start.push_back(s0);
        C.parent.push_back(b);
        C.blev.push_back(split ? l + 1 : P.blev[b]);
        if (split) {
          C.start.push_back(s0 + (s1 - s0) / 2);
          C.parent.push_back(b);
          C.blev.push_back(l + 1);
        }
      }
      C.org.assign((size_t)T.ostride * C.parent.size(), 0);
      C.start.push_back(n);
      T.lev.push_back(std::move(C));
    }
  }

  bool touching(const Level &Lv, int a, int b) const {
    for (int d = 0; d < T.dim; ++d) {
      const int os = T.ostride;
      int64_t oa = Lv.org[os * a + d], ob = Lv.org[os * b + d];
      int64_t ea = oa + (int64_t(1) << (T.kbits - Lv.blev[a]));
      int64_t eb = ob + (int64_t(1) << (T.kbits - Lv.blev[b]));
      if (ob > ea || oa > eb) return false;
    }
    return true;
  }

  // S(P) for a box P of level l-1: children of its neighbors, ascending
  void kids_of_neighbors(int l, int P, std::vector<int32_t> &out) const {
    out.clear();
    const Level &Q = T.lev[l - 1];
    for (int t = Q.nei_ptr[P]; t < Q.nei_ptr[P + 1]; ++t) {
      int nb = Q.nei[t];
      for (int q = kids_ptr[l - 1][nb]; q < kids_ptr[l - 1][nb + 1]; ++q)
        out.push_back(kids[l - 1][q]);
    }
    std::sort(out.begin(), out.end());
  }

  void lists() {
    const int nl = T.nlev();
    kids_ptr.assign(nl, {});
    kids.assign(nl, {});
    for (int l = 0; l + 1 < nl; ++l) child_index(l);
    // level 0
    T.lev[0].nei_ptr = {0, 1};
    T.lev[0].nei = {0};
    T.lev[0].int_ptr = {0, 0};
    T.lev[0].intl.clear();
    std::vector<int32_t> cand;
    for (int l = 1; l < nl; ++l) {
      Level &Lv = T.lev[l];
      const int nb = Lv.nbox();
      Lv.nei_ptr.assign(1, 0);
      Lv.int_ptr.assign(1, 0);
      Lv.nei.clear();
      Lv.intl.clear();
      for (int a = 0; a < nb; ++a) {
        const int P = Lv.parent[a];
        if (T.adm == HM_ADM_WEAK) {
          Lv.nei.push_back(a);
          for (int q = kids_ptr[l - 1][P]; q < kids_ptr[l - 1][P + 1]; ++q)
            if (kids[l - 1][q] != a) Lv.intl.push_back(kids[l - 1][q]);
        } else {
          kids_of_neighbors(l, P, cand);
          for (int32_t b : cand) {
            if (touching(Lv, a, b))
              Lv.nei.push_back(b);
            else
              Lv.intl.push_back(b);
          }
        }
        Lv.nei_ptr.push_back((int32_t)Lv.nei.size());
        Lv.int_ptr.push_back((int32_t)Lv.intl.size());
      }
    }
  }

  // Finish a graph from its vertex table: u ~ v iff the active box of v lies
  // in the box set of u or the active box of u lies in the box set of v, and
  // the two active boxes differ.
  void edges(Graph &G, const std::vector<std::vector<int32_t>> &sets, int nboxes) {
    const int64_t nv = G.nv();
    // CSR: vertices by active box, and vertices whose box set holds a box
    std::vector<int64_t> pa(nboxes + 1, 0), pc(nboxes + 1, 0);
    for (int64_t v = 0; v < nv; ++v) {
      pa[G.vbox[v] + 1]++;
      for (int32_t g : sets[G.vclass[v]]) pc[g + 1]++;
    }
    for (int b = 0; b < nboxes; ++b) {
      pa[b + 1] += pa[b];
      pc[b + 1] += pc[b];
    }
    std::vector<int32_t> by_active(pa[nboxes]), containing(pc[nboxes]);
    {
      std::vector<int64_t> fa(pa.begin(), pa.end() - 1), fc(pc.begin(), pc.end() - 1);
      for (int64_t v = 0; v < nv; ++v) {
        by_active[fa[G.vbox[v]]++] = (int32_t)v;
        for (int32_t g : sets[G.vclass[v]]) containing[fc[g]++] = (int32_t)v;
      }
    }
    // each row is marked in a vertex bitmap and read back in ascending order.
    // Rows are independent: chunks of kRows rows go to worker threads, each
    // with its own bitmap.  A first pass counts every row, a second writes
    // it at its offset, so the result does not depend on the number of
    // threads and the adjacency is written once, in place.
    const int64_t words = (nv + 63) / 64;
    constexpr int64_t kRows = 64;
    const int64_t nchunk = (nv + kRows - 1) / kRows;
    const int nth = (int)std::min<int64_t>(workers, nchunk);
    G.xadj.assign(nv + 1, 0);
    std::atomic<int64_t> next{0};
    auto pass = [&](bool write) {
      std::vector<uint64_t> mark(words, 0);
      std::vector<int64_t> touched;
      int64_t wlo = 0, whi = -1;  // range of the touched words
      auto put = [&](int32_t v) {
        uint64_t &w = mark[v >> 6];
        if (!w) {
          touched.push_back(v >> 6);
          wlo = std::min<int64_t>(wlo, v >> 6);
          whi = std::max<int64_t>(whi, v >> 6);
        }
        w |= uint64_t(1) << (v & 63);
      };
      for (int64_t c = next++; c < nchunk; c = next++) {
        for (int64_t u = c * kRows; u < std::min(nv, (c + 1) * kRows); ++u) {
          touched.clear();
          wlo = words;
          whi = -1;
          const int bu = G.vbox[u];
          for (int32_t g : sets[G.vclass[u]])
            if (g != bu)
              for (int64_t q = pa[g]; q < pa[g + 1]; ++q) put(by_active[q]);
          for (int64_t q = pc[bu]; q < pc[bu + 1]; ++q)
            if (G.vbox[containing[q]] != bu) put(containing[q]);
          if (!write) {
            int64_t cnt = 0;
            for (int64_t w : touched) {
              cnt += __builtin_popcountll(mark[w]);
              mark[w] = 0;
            }
            G.xadj[u + 1] = cnt;  // row length, summed below
            continue;
          }
          int32_t *o = G.adj.data() + G.xadj[u];
          auto emit = [&](int64_t w) {
            uint64_t bits = mark[w];
            mark[w] = 0;
            while (bits) {
              *o++ = (int32_t)(w * 64 + __builtin_ctzll(bits));
              bits &= bits - 1;
            }
          };
          if (whi - wlo + 1 <= 8 * (int64_t)touched.size()) {
            // dense row: walk the touched range in order (no sort)
            for (int64_t w = wlo; w <= whi; ++w)
              if (mark[w]) emit(w);
          } else {
            std::sort(touched.begin(), touched.end());
            for (int64_t w : touched) emit(w);
          }
        }
      }
    };
    auto run = [&](bool write) {
      next = 0;
      std::vector<std::thread> th;
      for (int t = 1; t < nth; ++t) th.emplace_back(pass, write);
      pass(write);
      for (auto &t : th) t.join();
    };
    run(false);
    for (int64_t u = 0; u < nv; ++u) G.xadj[u + 1] += G.xadj[u];
    G.adj.clear();
    G.adj.resize((size_t)G.xadj[nv]);  // uninitialized: the second pass writes every entry
    run(true);
  }

  void level_graph(int l, Graph &G) {
    G = Graph();
    if (l == 0) {
      G.xadj = {0};
      return;
    }
    const Level &Lv = T.lev[l];
    const Level &Q = T.lev[l - 1];
    const int nbp = Q.nbox();
    // parents with identical neighbor lists have identical box sets S(P)
    std::map<std::vector<int32_t>, int32_t> cls_of;
    std::vector<int32_t> pcls(nbp);
    std::vector<std::vector<int32_t>> sets;
    std::vector<int32_t> tmp;
    for (int P = 0; P < nbp; ++P) {
      std::vector<int32_t> key(Q.nei.begin() + Q.nei_ptr[P], Q.nei.begin() + Q.nei_ptr[P + 1]);
      auto it = cls_of.find(key);
      if (it == cls_of.end()) {
        int32_t c = (int32_t)sets.size();
        cls_of.emplace(std::move(key), c);
        kids_of_neighbors(l, P, tmp);
        sets.push_back(tmp);
        pcls[P] = c;
      } else {
        pcls[P] = it->second;
      }
    }
    std::unordered_map<int64_t, int32_t> vid;  // (active, class) -> vertex
    vid.reserve((size_t)Lv.nbox() * 8);
    auto vkey = [](int32_t b, int32_t c) { return ((int64_t)b << 32) | (uint32_t)c; };
    std::vector<int32_t> act;
    for (int P = 0; P < nbp; ++P) {
      act.clear();
      for (int q = kids_ptr[l - 1][P]; q < kids_ptr[l - 1][P + 1]; ++q) {
        int a = kids[l - 1][q];
        act.insert(act.end(), Lv.intl.begin() + Lv.int_ptr[a], Lv.intl.begin() + Lv.int_ptr[a + 1]);
      }
      std::sort(act.begin(), act.end());
      act.erase(std::unique(act.begin(), act.end()), act.end());
      for (int32_t b : act) {
        if (vid.emplace(vkey(b, pcls[P]), (int32_t)G.vbox.size()).second) {
          G.vbox.push_back(b);
          G.vclass.push_back(pcls[P]);
        }
      }
    }
    for (int a = 0; a < Lv.nbox(); ++a)
      for (int t = Lv.int_ptr[a]; t < Lv.int_ptr[a + 1]; ++t) {
        G.pa.push_back(a);
        G.pb.push_back(Lv.intl[t]);
        G.pv.push_back(vid.at(vkey(Lv.intl[t], pcls[Lv.parent[a]])));
      }
    edges(G, sets, Lv.nbox());
  }

  void leaf_graph(Graph &G) {
    G = Graph();
    const Level &Lv = T.lev[T.L()];
    std::map<std::vector<int32_t>, int32_t> cls_of;
    std::vector<std::vector<int32_t>> sets;
    std::map<std::pair<int32_t, int32_t>, int32_t> vid;
    for (int a = 0; a < Lv.nbox(); ++a) {
      std::vector<int32_t> key(Lv.nei.begin() + Lv.nei_ptr[a], Lv.nei.begin() + Lv.nei_ptr[a + 1]);
      int32_t c;
      auto it = cls_of.find(key);
      if (it == cls_of.end()) {
        c = (int32_t)sets.size();
        sets.push_back(key);
        cls_of.emplace(std::move(key), c);
      } else {
        c = it->second;
      }
      for (int t = Lv.nei_ptr[a]; t < Lv.nei_ptr[a + 1]; ++t) {
        int32_t b = Lv.nei[t];
        auto k = std::make_pair(b, c);
        auto jt = vid.find(k);
        int32_t v;
        if (jt == vid.end()) {
          v = (int32_t)G.vbox.size();
          vid.emplace(k, v);
          G.vbox.push_back(b);
          G.vclass.push_back(c);
        } else {
          v = jt->second;
        }
        G.pa.push_back(a);
        G.pb.push_back(b);
        G.pv.push_back(v);
      }
    }
    edges(G, sets, Lv.nbox());
  }
};

}  // namespace

int32_t Tree::leaf_width() const {
  int64_t w = 0;
  const Level &Lv = lev[L()];
  for (int b = 0; b < Lv.nbox(); ++b) w = std::max(w, Lv.start[b + 1] - Lv.start[b]);
  return (int32_t)w;
}

hm_status build_tree(const double *pts, int64_t n, int dim, int leaf, int kind, int adm,
                     Tree &T) {
  T = Tree();
  T.n = n;
  T.dim = dim;
  T.kbits = key_bits(dim);
  T.ostride = std::max(3, dim);
  T.kind = kind;
  T.adm = adm;
  T.leaf = leaf;
  T.pts.assign(pts, pts + n * dim);
  Builder B(T);
  B.workers = t_in_pool ? 1 : host_threads();
  const bool timing = std::getenv("HM_TIMING") != nullptr;
  auto t0 = std::chrono::steady_clock::now();
  auto lap = [&](const char *what) {
    if (!timing) return;
    auto t1 = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[hm] %s %.2f ms\n", what,
                 std::chrono::duration<double, std::milli>(t1 - t0).count());
    t0 = t1;
  };
  if (kind == HM_TREE_GEOMETRIC)
    B.geometric(pts);
  else
    B.index_binary(pts);
  lap("tree");
  B.lists();
  lap("lists");
  T.graphs.resize(T.nlev() + 1);
  // the graphs of different levels are independent: large levels get a
  // thread each, small ones are built on this thread
  {
    std::vector<std::thread> th;
    for (int l = 0; l < T.nlev(); ++l) {
      if (T.lev[l].nbox() > 128)
        th.emplace_back([&B, &T, l] { B.level_graph(l, T.graphs[l]); });
      else
        B.level_graph(l, T.graphs[l]);
    }
    if (T.lev[T.L()].nbox() > 128)
      th.emplace_back([&B, &T] { B.leaf_graph(T.graphs.back()); });
    else
      B.leaf_graph(T.graphs.back());
    for (auto &t : th) t.join();
  }
  lap("graphs");
  T.inst_off = {0, n};
  T.gvoff.clear();
  for (const Graph &G : T.graphs) T.gvoff.push_back({0, G.nv()});
  return HM_OK;
}

hm_status build_forest(const double *pts, const int64_t *counts, int ninst, int dim, int leaf,
                       int kind, int adm, Tree &F) {
  std::vector<Tree> parts(ninst);
  std::vector<int64_t> off(ninst + 1, 0);
  for (int i = 0; i < ninst; ++i) off[i + 1] = off[i] + counts[i];
  std::vector<hm_status> rc(ninst, HM_OK);
  {
    // instances are independent: a pool of host threads takes them in turn
    const int nth = std::max(1, std::min<int>(ninst, host_threads()));
    std::vector<std::thread> th;
    std::atomic<int> next{0};
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&] {
        t_in_pool = true;
        for (int i = next++; i < ninst; i = next++)
          rc[i] = build_tree(pts + off[i] * dim, counts[i], dim, leaf, kind, adm, parts[i]);
      });
    for (auto &t : th) t.join();
  }
  for (int i = 0; i < ninst; ++i)
    if (rc[i] != HM_OK) return rc[i];
  int nlev = 0;
  for (const Tree &P : parts) nlev = std::max(nlev, P.nlev());
  F = Tree();
  F.n = off[ninst];
  F.dim = dim;
  F.kbits = key_bits(dim);
  F.ostride = std::max(3, dim);
  F.kind = kind;
  F.adm = adm;
  F.leaf = leaf;
  F.pts.assign(pts, pts + F.n * dim);
  F.inst_off = off;
  F.perm.resize(F.n);
  for (int i = 0; i < ninst; ++i)
    for (int64_t t = 0; t < counts[i]; ++t) F.perm[off[i] + t] = parts[i].perm[t] + off[i];
  // boxes of instance i at forest level l: its own level min(l, L_i)
  std::vector<std::vector<int32_t>> boff(nlev, std::vector<int32_t>(ninst + 1, 0));
  for (int l = 0; l < nlev; ++l)
    for (int i = 0; i < ninst; ++i)
      boff[l][i + 1] = boff[l][i] + parts[i].lev[std::min(l, parts[i].L())].nbox();
  // the levels, and below the graphs, are independent of each other: each
  // is filled by one thread of a pool, into vectors sized up front
  auto pool = [](int count, const std::function<void(int)> &f) {
    std::atomic<int> next{0};
    auto run = [&] {
      for (int k = next++; k < count; k = next++) f(k);
    };
    const int nth = std::max(1, std::min(count, host_threads()));
    std::vector<std::thread> th;
    for (int t = 1; t < nth; ++t) th.emplace_back(run);
    run();
    for (auto &t : th) t.join();
  };
  F.lev.resize(nlev);
  pool(nlev, [&](int l) {
    Level &Lv = F.lev[l];
    const int64_t nb = boff[l][ninst];
    int64_t nn = 0, ni = 0;
    for (int i = 0; i < ninst; ++i) {
      const Tree &P = parts[i];
      const Level &S = P.lev[std::min(l, P.L())];
      nn += S.nei_ptr[S.nbox()];
      if (l <= P.L()) ni += S.int_ptr[S.nbox()];
    }
    Lv.start.reserve(nb + 1);
    Lv.parent.reserve(nb);
    Lv.org.reserve(nb * F.ostride);
    Lv.blev.reserve(nb);
    Lv.nei.reserve(nn);
    Lv.nei_ptr.reserve(nb + 1);
    Lv.intl.reserve(ni);
    Lv.int_ptr.reserve(nb + 1);
    Lv.nei_ptr.push_back(0);
    Lv.int_ptr.push_back(0);
    for (int i = 0; i < ninst; ++i) {
      const Tree &P = parts[i];
      const int sl = std::min(l, P.L());
      const bool carried = l > P.L();
      const Level &S = P.lev[sl];
      const int32_t b0 = boff[l][i];
      for (int b = 0; b < S.nbox(); ++b) {
        Lv.start.push_back(S.start[b] + off[i]);
        Lv.parent.push_back(l == 0 ? -1 : (carried ? b : S.parent[b]) + boff[l - 1][i]);
        for (int d = 0; d < F.ostride; ++d) Lv.org.push_back(S.org[F.ostride * b + d]);
        Lv.blev.push_back(S.blev[b]);
        for (int t = S.nei_ptr[b]; t < S.nei_ptr[b + 1]; ++t) Lv.nei.push_back(S.nei[t] + b0);
        Lv.nei_ptr.push_back((int32_t)Lv.nei.size());
        if (!carried)
          for (int t = S.int_ptr[b]; t < S.int_ptr[b + 1]; ++t) Lv.intl.push_back(S.intl[t] + b0);
        Lv.int_ptr.push_back((int32_t)Lv.intl.size());
      }
    }
    Lv.start.push_back(F.n);
  });
  // graphs: disjoint unions, instance-major vertex numbering
  F.graphs.resize(nlev + 1);
  F.gvoff.assign(nlev + 1, std::vector<int64_t>(ninst + 1, 0));
  static const Graph empty;
  pool(nlev + 1, [&](int g) {
    Graph &G = F.graphs[g];
    const int bl = g < nlev ? g : nlev - 1;  // box level of the graph's ids
    auto part = [&](int i) -> const Graph & {
      const Tree &P = parts[i];
      return g == nlev ? P.leaf_graph() : (g <= P.L() ? P.graphs[g] : empty);
    };
    int64_t tv = 0, ta = 0, tp = 0;
    for (int i = 0; i < ninst; ++i) {
      const Graph &S = part(i);
      tv += S.nv();
      ta += (int64_t)S.adj.size();
      tp += (int64_t)S.pa.size();
    }
    G.vbox.reserve(tv);
    G.vclass.reserve(tv);
    G.xadj.reserve(tv + 1);
    G.adj.reserve(ta);
    G.pa.reserve(tp);
    G.pb.reserve(tp);
    G.pv.reserve(tp);
    G.xadj.push_back(0);
    int32_t cls0 = 0;
    for (int i = 0; i < ninst; ++i) {
      const Graph &S = part(i);
      const int64_t v0 = G.nv();
      F.gvoff[g][i] = v0;
      const int32_t b0 = boff[bl][i];
      int32_t cmax = -1;
      for (int64_t v = 0; v < S.nv(); ++v) {
        G.vbox.push_back(S.vbox[v] + b0);
        G.vclass.push_back(S.vclass[v] + cls0);
        cmax = std::max(cmax, S.vclass[v]);
        for (int64_t t = S.xadj[v]; t < S.xadj[v + 1]; ++t)
          G.adj.push_back((int32_t)(S.adj[t] + v0));
        G.xadj.push_back((int64_t)G.adj.size());
      }
      cls0 += cmax + 1;
      for (size_t q = 0; q < S.pa.size(); ++q) {
        G.pa.push_back(S.pa[q] + b0);
        G.pb.push_back(S.pb[q] + b0);
        G.pv.push_back((int32_t)(S.pv[q] + v0));
      }
    }
    F.gvoff[g][ninst] = G.nv();
  });
  return HM_OK;
}

void build_uniform_graphs(Tree &T) {
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  if (T.uniform_built) return;
  T.ugraphs.assign(T.nlev(), Graph());
  for (int l = 0; l < T.nlev(); ++l) {
    const Level &Lv = T.lev[l];
    Graph &G = T.ugraphs[l];
    const int nb = Lv.nbox();
    std::vector<int32_t> vid(nb, -1);
    for (int a = 0; a < nb; ++a)
      if (Lv.int_ptr[a + 1] > Lv.int_ptr[a]) {
        vid[a] = (int32_t)G.vbox.size();
        G.vbox.push_back(a);
        G.vclass.push_back(0);
      }
    // conflicts of a: a neighbor of a box in a's interaction list, or a box
    // in the interaction list of one of a's neighbors (neighbor and
    // interaction relations are symmetric)
    std::vector<uint8_t> mark(nb, 0);
    std::vector<int32_t> cand;
    G.xadj.assign(1, 0);
    for (int32_t a : G.vbox) {
      cand.clear();
      for (int t = Lv.int_ptr[a]; t < Lv.int_ptr[a + 1]; ++t) {
        const int b = Lv.intl[t];
        for (int u = Lv.nei_ptr[b]; u < Lv.nei_ptr[b + 1]; ++u) {
          const int c = Lv.nei[u];
          if (c != a && vid[c] >= 0 && !mark[c]) {
            mark[c] = 1;
            cand.push_back(c);
          }
        }
      }
      for (int t = Lv.nei_ptr[a]; t < Lv.nei_ptr[a + 1]; ++t) {
        const int b = Lv.nei[t];
        for (int u = Lv.int_ptr[b]; u < Lv.int_ptr[b + 1]; ++u) {
          const int c = Lv.intl[u];
          if (c != a && vid[c] >= 0 && !mark[c]) {
            mark[c] = 1;
            cand.push_back(c);
          }
        }
      }
      std::sort(cand.begin(), cand.end());
      for (int32_t c : cand) {
        mark[c] = 0;
        G.adj.push_back(vid[c]);
      }
      G.xadj.push_back((int64_t)G.adj.size());
    }
    G.color.assign(G.nv(), 0);
    G.ncolors = dsatur(G.nv(), G.xadj.data(), G.adj.data(), G.color.data());
    G.colored = true;
  }
  T.uniform_built = true;
}

// DSatur.  Vertices are ranked once by (degree descending, id ascending); the
// uncolored vertices of each saturation value sit in a bitset over ranks, so
// the next vertex is the lowest set rank of the highest non-empty saturation.
// Bitsets record the colors already on a neighbor of each vertex, stored
// color word major (word q of all vertices together), so that coloring a
// vertex with c touches one array of nv words while it updates its
// neighbors.
int32_t dsatur(int64_t nv, const int64_t *xadj, const int32_t *adj, int32_t *color) {
  if (nv <= 0) return 0;
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < nv; ++v) maxdeg = std::max(maxdeg, xadj[v + 1] - xadj[v]);
  const int64_t cwords = (maxdeg + 2 + 63) / 64;
  std::vector<uint64_t> seen((size_t)(nv * cwords), 0);
  std::vector<int64_t> byrank(nv), rank(nv);
  for (int64_t v = 0; v < nv; ++v) byrank[v] = v;
  std::stable_sort(byrank.begin(), byrank.end(), [&](int64_t a, int64_t b) {
    return xadj[a + 1] - xadj[a] > xadj[b + 1] - xadj[b];
  });
  for (int64_t i = 0; i < nv; ++i) rank[byrank[i]] = i;
  const int64_t words = (nv + 63) / 64;
  std::vector<std::vector<uint64_t>> level(1, std::vector<uint64_t>(words, 0));
  std::vector<int64_t> count(1, nv), hint(1, 0);
  for (int64_t i = 0; i < nv; ++i) level[0][i >> 6] |= uint64_t(1) << (i & 63);
  std::vector<int32_t> sat(nv, 0);
  for (int64_t v = 0; v < nv; ++v) color[v] = -1;
  int64_t top = 0;
  int32_t ncol = 0;
  for (int64_t step = 0; step < nv; ++step) {
    while (count[top] == 0) --top;
    std::vector<uint64_t> &L = level[top];
    int64_t w = hint[top];
    while (!L[w]) ++w;
    hint[top] = w;
    const int64_t rk = w * 64 + __builtin_ctzll(L[w]);
    L[w] &= L[w] - 1;
    count[top]--;
    const int64_t v = byrank[rk];
    int32_t c = 0;
    for (int64_t q = 0; q < cwords; ++q) {
      const uint64_t sq = seen[(size_t)(q * nv + v)];
      if (~sq) {
        c = int32_t(q * 64 + __builtin_ctzll(~sq));
        break;
      }
    }
    color[v] = c;
    ncol = std::max(ncol, c + 1);
    const uint64_t mask = uint64_t(1) << (c % 64);
    for (int64_t t = xadj[v]; t < xadj[v + 1]; ++t) {
      const int64_t u = adj[t];
      uint64_t &bit = seen[(size_t)((c / 64) * nv + u)];
      if (bit & mask) continue;
      bit |= mask;
      if (color[u] >= 0) continue;
      const int64_t ru = rank[u];
      const int32_t s = sat[u];
      level[s][ru >> 6] &= ~(uint64_t(1) << (ru & 63));
      count[s]--;
      sat[u] = s + 1;
      if ((int64_t)level.size() <= s + 1) {
        level.emplace_back(words, 0);
        count.push_back(0);
        hint.push_back(words);
      }
      level[s + 1][ru >> 6] |= uint64_t(1) << (ru & 63);
      count[s + 1]++;
      hint[s + 1] = std::min(hint[s + 1], ru >> 6);
      top = std::max<int64_t>(top, s + 1);
    }
  }
  return ncol;
}

}  // namespace hm
