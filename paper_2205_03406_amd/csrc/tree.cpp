// Host combinatorics of colored peeling: box tree, neighbor / interaction
// lists, constraint incompatibility graphs and DSatur coloring.
//
// Paper: Levitt & Martinsson, arXiv 2205.03406 -- section "Rank-structured
// matrices" (tree and lists), eq:h1constraints and def:incompatibility_graph
// (level graphs), the leaf-extraction section (leaf graph), alg:dsatur.
//
// Design notes (MI355X build): this runs on the host once per geometry.  It
// works level by level with candidate sets drawn from the parent level
// (a box's neighbors are among the children of its parent's neighbors), so
// the cost is O(N log N + boxes * 6^d + edges) rather than quadratic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <tuple>
#include <unordered_map>

#include "hm_internal.h"

namespace hm {

namespace {

constexpr int kBits = 21;
constexpr uint32_t kMaxCell = (1u << kBits) - 1;

// Spread the low 21 bits of v so that bit i lands at bit i*stride.
uint64_t spread(uint32_t v, int stride) {
  uint64_t out = 0;
  uint64_t x = v;
  int pos = 0;
  while (x) {
    if (x & 1) out |= uint64_t(1) << (pos * stride);
    x >>= 1;
    ++pos;
  }
  return out;
}

uint32_t cell(double x, double lo, double s) {
  // Evaluated as written, one rounding per operation (no contraction).
  volatile double q = (x - lo) / s;
  double t = q * 2097152.0;
  double f = std::floor(t);
  if (f >= double(kMaxCell)) return kMaxCell;
  return uint32_t(f);
}

struct Builder {
  Tree &T;
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
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
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
        uint32_t c = cell(pts[i * dim + d], lo[d], s);
        cells[i * dim + d] = c;
        k |= spread(c, dim) << d;
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
    root.org = {0, 0, 0};
    root.blev = {0};
    T.lev.push_back(std::move(root));
    const int m = T.leaf;
    for (int l = 0; l < kBits; ++l) {
      const Level &P = T.lev[l];
      bool split_any = false;
      for (int b = 0; b < P.nbox(); ++b)
        if (P.start[b + 1] - P.start[b] > m) split_any = true;
      if (!split_any) break;
      Level C;
      const int shift = (kBits - 1 - l) * dim;  // key bits below the child digit
      for (int b = 0; b < P.nbox(); ++b) {
        int64_t s0 = P.start[b], s1 = P.start[b + 1];
        if (s1 - s0 <= m) {  // leaf: carried to the next level unchanged
          C.start.push_back(s0);
          C.parent.push_back(b);
          for (int d = 0; d < 3; ++d) C.org.push_back(P.org[3 * b + d]);
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
          for (int d = 0; d < 3; ++d) {
            int64_t o = P.org[3 * b + d];
            if (d < dim && ((digit >> d) & 1)) o += int64_t(1) << (kBits - 1 - l);
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
    root.org = {0, 0, 0};
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
      C.org.assign(3 * C.parent.size(), 0);
      C.start.push_back(n);
      T.lev.push_back(std::move(C));
    }
  }

  bool touching(const Level &Lv, int a, int b) const {
    for (int d = 0; d < T.dim; ++d) {
      int64_t oa = Lv.org[3 * a + d], ob = Lv.org[3 * b + d];
      int64_t ea = oa + (int64_t(1) << (kBits - Lv.blev[a]));
      int64_t eb = ob + (int64_t(1) << (kBits - Lv.blev[b]));
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
    std::vector<std::vector<int32_t>> by_active(nboxes), containing(nboxes);
    for (int64_t v = 0; v < nv; ++v) {
      by_active[G.vbox[v]].push_back((int32_t)v);
      for (int32_t g : sets[G.vclass[v]]) containing[g].push_back((int32_t)v);
    }
    G.xadj.assign(nv + 1, 0);
    G.adj.clear();
    std::vector<int32_t> row;
    for (int64_t u = 0; u < nv; ++u) {
      row.clear();
      const int bu = G.vbox[u];
      for (int32_t g : sets[G.vclass[u]])
        if (g != bu)
          for (int32_t v : by_active[g]) row.push_back(v);
      for (int32_t v : containing[bu])
        if (G.vbox[v] != bu) row.push_back(v);
      std::sort(row.begin(), row.end());
      row.erase(std::unique(row.begin(), row.end()), row.end());
      G.adj.insert(G.adj.end(), row.begin(), row.end());
      G.xadj[u + 1] = (int64_t)G.adj.size();
    }
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
    std::map<std::pair<int32_t, int32_t>, int32_t> vid;  // (active, class) -> vertex
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
        auto key = std::make_pair(b, pcls[P]);
        if (vid.find(key) == vid.end()) {
          vid.emplace(key, (int32_t)G.vbox.size());
          G.vbox.push_back(b);
          G.vclass.push_back(pcls[P]);
        }
      }
    }
    for (int a = 0; a < Lv.nbox(); ++a)
      for (int t = Lv.int_ptr[a]; t < Lv.int_ptr[a + 1]; ++t) {
        G.pa.push_back(a);
        G.pb.push_back(Lv.intl[t]);
        G.pv.push_back(vid.at({Lv.intl[t], pcls[Lv.parent[a]]}));
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
  T.kind = kind;
  T.adm = adm;
  T.leaf = leaf;
  T.pts.assign(pts, pts + n * dim);
  Builder B(T);
  if (kind == HM_TREE_GEOMETRIC)
    B.geometric(pts);
  else
    B.index_binary(pts);
  B.lists();
  T.graphs.resize(T.nlev() + 1);
  for (int l = 0; l < T.nlev(); ++l) B.level_graph(l, T.graphs[l]);
  B.leaf_graph(T.graphs.back());
  return HM_OK;
}

// DSatur with an ordered set keyed by (-saturation, -degree, id); per-vertex
// bitsets record which colors already sit on a neighbor.
int32_t dsatur(int64_t nv, const int64_t *xadj, const int32_t *adj, int32_t *color) {
  if (nv <= 0) return 0;
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < nv; ++v) maxdeg = std::max(maxdeg, xadj[v + 1] - xadj[v]);
  const int64_t words = (maxdeg + 2 + 63) / 64;
  std::vector<uint64_t> seen((size_t)(nv * words), 0);
  std::vector<int32_t> sat(nv, 0);
  using Key = std::tuple<int32_t, int64_t, int64_t>;  // (-sat, -deg, id)
  std::set<Key> q;
  for (int64_t v = 0; v < nv; ++v) {
    color[v] = -1;
    q.insert(Key(0, -(xadj[v + 1] - xadj[v]), v));
  }
  int32_t ncol = 0;
  while (!q.empty()) {
    const int64_t v = std::get<2>(*q.begin());
    q.erase(q.begin());
    const uint64_t *sv = &seen[(size_t)(v * words)];
    int32_t c = 0;
    for (int64_t w = 0; w < words; ++w) {
      if (~sv[w]) {
        c = int32_t(w * 64 + __builtin_ctzll(~sv[w]));
        break;
      }
    }
    color[v] = c;
    ncol = std::max(ncol, c + 1);
    for (int64_t t = xadj[v]; t < xadj[v + 1]; ++t) {
      const int64_t w = adj[t];
      uint64_t &bit = seen[(size_t)(w * words + c / 64)];
      const uint64_t mask = uint64_t(1) << (c % 64);
      if (bit & mask) continue;
      bit |= mask;
      if (color[w] >= 0) continue;
      const int64_t deg = xadj[w + 1] - xadj[w];
      q.erase(Key(-sat[w], -deg, w));
      sat[w]++;
      q.insert(Key(-sat[w], -deg, w));
    }
  }
  return ncol;
}

}  // namespace hm
