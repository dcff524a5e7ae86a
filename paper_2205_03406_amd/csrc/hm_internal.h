// Internal declarations shared by the host and device sources of libhm.
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hm.h"

namespace hm {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
hm_status fail(hm_status code, const std::string &msg);

struct Error {
  hm_status code;
  std::string msg;
};

// ------------------------------------------------------------------ device memory
// The caller's allocator (hm_allocator) in force on this thread: an entry
// point that was given one installs it for its duration, and every device
// allocation made meanwhile (its blocks and scratch) goes through it.
const hm_allocator *&alloc_scope();
struct AllocScope {
  const hm_allocator *prev;
  // a null or incomplete allocator leaves the one in force
  explicit AllocScope(const hm_allocator *a) : prev(alloc_scope()) {
    if (a && a->alloc && a->free) alloc_scope() = a;
  }
  ~AllocScope() { alloc_scope() = prev; }
  AllocScope(const AllocScope &) = delete;
  AllocScope &operator=(const AllocScope &) = delete;
};
// Flops per launch of the built-in kernel apply on this thread (0: whole
// launches).  The server sets it for its compressions, whose kernel applies
// then run as row slices of about that much work each, so that work on the
// other workers' streams (applies) gets the device between slices instead
// of waiting for a launch of seconds.
double &kapply_slice_flops();
struct SliceScope {
  double prev;
  explicit SliceScope(double flops) : prev(kapply_slice_flops()) { kapply_slice_flops() = flops; }
  ~SliceScope() { kapply_slice_flops() = prev; }
  SliceScope(const SliceScope &) = delete;
  SliceScope &operator=(const SliceScope &) = delete;
};
// stream-ordered device scratch: the allocator in force, else
// hipMallocAsync / hipFreeAsync (stream: a hipStream_t)
void *scratch_alloc(size_t bytes, void *stream);
void scratch_free(void *p, void *stream);

// ------------------------------------------------------------------ tree
struct Level {
  std::vector<int64_t> start;    // nbox + 1
  std::vector<int32_t> parent;   // nbox
  std::vector<int64_t> org;      // ostride * nbox (integer cube origins)
  std::vector<int32_t> blev;     // nbox
  std::vector<int32_t> nei_ptr, nei;
  std::vector<int32_t> int_ptr, intl;
  int32_t nbox() const { return (int32_t)parent.size(); }
};

// Allocator whose element construction without arguments leaves the
// element uninitialized, so that resizing a large buffer that is filled
// right after does not write it twice (the graph builder's adjacency).
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U> &) {}
  template <class U>
  void construct(U *p) noexcept {
    ::new ((void *)p) U;
  }
  template <class U, class... A>
  void construct(U *p, A &&...a) {
    ::new ((void *)p) U(std::forward<A>(a)...);
  }
};

struct Graph {
  std::vector<int32_t> vbox;     // active box per vertex
  std::vector<int32_t> vclass;   // neighbor-set class of the vertex's box set
  std::vector<int64_t> xadj;
  std::vector<int32_t, NoInitAlloc<int32_t>> adj;
  std::vector<int32_t> pa, pb, pv;  // pairs and their vertex
  std::vector<int32_t> color;
  int32_t ncolors = 0;
  bool colored = false;
  int64_t nv() const { return (int64_t)vbox.size(); }
};

struct DeviceTree;  // device copies, defined in the engine

struct Tree {
  int64_t n = 0;
  int dim = 0, kind = 0, adm = 0, leaf = 0;
  int kbits = 21;    // integer cell bits per coordinate (21 for d <= 3, 63 / d above)
  int ostride = 3;   // origin entries per box: max(3, dim)
  std::vector<double> pts;        // original order, n x dim row-major
  std::vector<int64_t> perm;      // tree position -> original index
  std::vector<Level> lev;
  std::vector<Graph> graphs;      // one per level + the leaf graph last
  // A forest holds independent instances side by side: instance i owns rows
  // [inst_off[i], inst_off[i+1]) in both orders, its boxes come before those
  // of instance i+1 at every level, and gvoff[g][i] is its first vertex in
  // graph g.  A single tree is a forest of one instance.
  std::vector<int64_t> inst_off;
  std::vector<std::vector<int64_t>> gvoff;
  // uniform H^1 stage-1 graphs, one per level (vertices = boxes with a
  // non-empty interaction list), built and colored on first use
  std::vector<Graph> ugraphs;
  bool uniform_built = false;
  std::shared_ptr<DeviceTree> dev;
  std::vector<std::shared_ptr<void>> keep;  // objects whose lifetime is the tree's
  int nlev() const { return (int)lev.size(); }
  int ninst() const { return inst_off.empty() ? 1 : (int)inst_off.size() - 1; }
  int L() const { return nlev() - 1; }
  Graph &leaf_graph() { return graphs.back(); }
  const Graph &leaf_graph() const { return graphs.back(); }
  int64_t box_size(int l, int b) const { return lev[l].start[b + 1] - lev[l].start[b]; }
  int32_t leaf_width() const;
};

hm_status build_tree(const double *pts, int64_t n, int dim, int leaf, int kind, int adm,
                     Tree &T);
// Independent trees over consecutive point ranges (counts[i] points each),
// merged level by level; shallower trees carry their leaves down to the
// deepest level, so level l of the forest is the union of the instances'
// level-l partitions.
hm_status build_forest(const double *pts, const int64_t *counts, int ninst, int dim, int leaf,
                       int kind, int adm, Tree &F);
// Builds and colors T.ugraphs (section on uniform H^1 compression,
// eq:unifh1constraints): box a wants Gaussian blocks on its interaction list
// and zeros on its neighbors; a and b conflict when a box active for one is
// a neighbor of the other.  Idempotent and serialized (one builder at a time).
void build_uniform_graphs(Tree &T);
int32_t dsatur(int64_t nv, const int64_t *xadj, const int32_t *adj, int32_t *color);
// Host worker threads: the CPUs this process may run on (its affinity
// mask), at most 16.
int host_threads();

// ------------------------------------------------------------------ sizes
int64_t hmatrix_device_bytes(const hm_hmatrix *H);
int64_t tree_device_bytes(const Tree &T);
int64_t compress_footprint(Tree &T, const hm_compress_opts &o);
int64_t matvec_footprint(const hm_hmatrix *H, int64_t nrhs, int dtype);
// frees the idle device blocks kept for reuse by H-matrices, trees and compressions
void trim_block_cache(int dev);
// hm_hmatrix_free / hm_tree_free for an object with no work in flight (its
// caller synchronized every stream that used it): its blocks go back at
// once instead of after a device-wide synchronization, which would wait
// for the work of every other stream (a compression of seconds)
void free_idle(hm_hmatrix *H);
void free_idle(hm_tree *T);

// ------------------------------------------------------------------ autotuner
struct KapplyShape {
  bool f32;
  int kernel, dim;
  int64_t ncols, n;
  bool forest;
  int64_t units;  // work units of a launch (row blocks, or forest items)
};
// Column-tile width of a kernel-apply launch: timed over the candidates on
// the first launch of a shape (each on a prefix of the work units), then
// cached.  launch(nt, units) enqueues one launch of the first `units` work
// units (0: all) on `stream` (hipStream_t); on return the output holds the
// full product.
int autotune_kapply(const KapplyShape &shape,
                    const std::function<void(int, int64_t)> &launch, void *stream);
std::string autotune_report();

}  // namespace hm

struct hm_tree {
  hm::Tree t;
};
