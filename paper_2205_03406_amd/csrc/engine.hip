// libhm engine: the C ABI of include/hm.h and the level pipeline of
// alg:h1_pseudocode on one GPU.
//
// Per sampled level l (coarsest first), on one stream:
//   1. draw [Omega | Psi] (N x 2*cpad, tree order; FP64, or FP32 in the mixed
//      path) -- Philox4x32-10 + Box-Muller, colored by the level's graph;
//   2. black box: [Y | Z] = [A Omega | A* Psi]; one call when A* = A;
//   3. peel: subtract the levels already compressed (grouped low-rank
//      products, deterministic, no atomics);
//   4. recover every admissible pair: C = G2^T Y_ab, pivoted QR bases for U
//      and V, coupling solve B, W = U B -- all FP64;
// then the leaf pass with identity test matrices.  Ranks live on the device
// (tolerance mode needs no host round trip); factor slots are sized for the
// largest rank the level can produce.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hm_internal.h"
#include "kernels.h"

namespace hm {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }
hm_status fail(hm_status code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(x)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      throw Error{HM_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};        \
  } while (0)

#define LAUNCH_CHECK()                                                                 \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess)                                                              \
      throw Error{HM_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)}; \
  } while (0)

// ------------------------------------------------------------------ device buffers
// Device blocks of H-matrices kept for reuse, per device: hipMalloc maps
// pages eagerly (about 10 us per MB) and freeing costs 20 us to 0.3 ms per
// buffer, milliseconds per compression for the few dozen buffers (a few
// hundred MB) an H-matrix holds.  A block comes back only once the device
// is idle (the H-matrix destructor synchronizes, and a block replaced while
// a compression runs waits for the device first), so a block taken from
// the cache has no work in flight.  At most 2 GiB per device is kept; the
// cache is emptied when hipMalloc fails.
struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, void *> free[64];  // block size -> block
  size_t held[64] = {};
};
BlockCache &block_cache() {
  static BlockCache c;
  return c;
}
constexpr size_t kCacheMax = size_t(2) << 30;
// a cached block of at least b bytes and at most 2b + 1 MB (its size in b),
// or nullptr
void *cache_take(int dev, size_t &b) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.free[dev].lower_bound(b);
  if (it == c.free[dev].end() || it->first > 2 * b + (size_t(1) << 20)) return nullptr;
  b = it->first;
  void *p = it->second;
  c.held[dev] -= b;
  c.free[dev].erase(it);
  return p;
}
void cache_put(int dev, void *p, size_t b) {
  BlockCache &c = block_cache();
  {
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.held[dev] + b <= kCacheMax) {
      c.free[dev].emplace(b, p);
      c.held[dev] += b;
      return;
    }
  }
  (void)hipFree(p);
}
void cache_drop(int dev) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto &e : c.free[dev]) (void)hipFree(e.second);
  c.free[dev].clear();
  c.held[dev] = 0;
}
// set while an H-matrix's members are destroyed after the device was synchronized
inline bool &release_synced() {
  thread_local bool f = false;
  return f;
}
// set while an owner whose every use its caller has already synchronized
// is destroyed (free_idle): nothing to wait for, however busy the device's
// other streams are
inline bool &release_idle() {
  thread_local bool f = false;
  return f;
}
// Declared as the first member of an owner of cached blocks (so destroyed
// last): the owner's destructor body calls begin(), which makes the owner's
// device current, waits until it is idle and lets the members that follow
// go back to the cache without waiting again; this member then ends that
// and restores the caller's device.
struct SyncedRelease {
  int cur = -1;
  void begin(int device) {
    (void)hipGetDevice(&cur);
    if (device >= 0 && device != cur) (void)hipSetDevice(device);
    if (!release_idle()) {
      (void)hipDeviceSynchronize();
      (void)hipGetLastError();
    }
    release_synced() = true;
  }
  // the same for buffers used on stream s only
  void begin_stream(hipStream_t s) {
    if (!release_idle()) {
      (void)hipStreamSynchronize(s);
      (void)hipGetLastError();
    }
    release_synced() = true;
  }
  ~SyncedRelease() {
    release_synced() = false;
    int d = -1;
    if (cur >= 0 && hipGetDevice(&d) == hipSuccess && d != cur) (void)hipSetDevice(cur);
  }
};

// The caller's allocator (hm_allocator) in force on this thread: set for
// the duration of an entry point that was given one (AllocScope); every
// device allocation made meanwhile goes through it.
double &kapply_slice_flops() {
  thread_local double f = 0.0;
  return f;
}

const hm_allocator *&alloc_scope() {
  thread_local const hm_allocator *a = nullptr;
  return a;
}
void *scope_alloc(const hm_allocator &a, size_t b, hipStream_t s) {
  void *p = a.alloc(a.ctx, b, (void *)s);
  if (!p) throw Error{HM_E_NOMEM, "allocator returned no block for " + std::to_string(b) + " bytes"};
  return p;
}
// stream-ordered scratch: the allocator in force, else hipMallocAsync
void *stream_alloc(size_t b, hipStream_t s) {
  if (b == 0) b = 64;
  if (const hm_allocator *a = alloc_scope()) return scope_alloc(*a, b, s);
  void *p = nullptr;
  if (hipMallocAsync(&p, b, s) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{HM_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed"};
  }
  return p;
}
void stream_free(void *p, hipStream_t s) {
  if (!p) return;
  if (const hm_allocator *a = alloc_scope())
    a->free(a->ctx, p, (void *)s);
  else
    (void)hipFreeAsync(p, s);
}
void *scratch_alloc(size_t bytes, void *stream) { return stream_alloc(bytes, (hipStream_t)stream); }
void scratch_free(void *p, void *stream) { stream_free(p, (hipStream_t)stream); }
// a stream-ordered block that goes back when it leaves scope (also on an
// error); the allocator scope must enclose it
struct StreamBlock {
  void *p = nullptr;
  hipStream_t s = nullptr;
  StreamBlock() = default;
  StreamBlock(size_t b, hipStream_t st) : s(st) { p = stream_alloc(b, st); }
  StreamBlock(const StreamBlock &) = delete;
  StreamBlock &operator=(const StreamBlock &) = delete;
  void take(size_t b, hipStream_t st) {
    s = st;
    p = stream_alloc(b, st);
  }
  ~StreamBlock() { stream_free(p, s); }
};

// Device buffer.  alloc(): plain hipMalloc / hipFree, for objects that
// outlive the call that makes them (trees).  cached(): the block cache above,
// for the buffers of H-matrices.  temp(): stream-
// ordered hipMallocAsync / hipFreeAsync on the stream of the work that uses
// it, so the scratch of one compression is freed without waiting on work
// that other streams (other requests) have in flight.  With a caller's
// allocator in force (alloc_scope) every form takes its block from it
// instead and returns it there, after the same waits.
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  hipStream_t st = nullptr;
  bool async = false;
  bool in_cache = false;  // from the block cache (cap bytes, device dev)
  bool stream_owned = false;  // returns once st is idle (else the device)
  size_t cap = 0;
  int dev = 0;
  hm_allocator al{};  // the caller's allocator the block came from (al.free set)
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept
      : p(o.p), bytes(o.bytes), st(o.st), async(o.async), in_cache(o.in_cache),
        stream_owned(o.stream_owned), cap(o.cap), dev(o.dev), al(o.al) {
    o.p = nullptr;
    o.bytes = 0;
    o.in_cache = false;
    o.al = hm_allocator{};
  }
  DBuf &operator=(DBuf &&o) noexcept {
    release();
    p = o.p;
    bytes = o.bytes;
    st = o.st;
    async = o.async;
    in_cache = o.in_cache;
    stream_owned = o.stream_owned;
    cap = o.cap;
    dev = o.dev;
    al = o.al;
    o.p = nullptr;
    o.bytes = 0;
    o.in_cache = false;
    o.al = hm_allocator{};
    return *this;
  }
  ~DBuf() { release(); }
  // a block from the allocator in force, if any
  bool from_scope(size_t b, hipStream_t s) {
    const hm_allocator *a = alloc_scope();
    if (!a) return false;
    p = scope_alloc(*a, b, s);
    al = *a;
    bytes = b;
    st = s;
    return true;
  }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 64;
    if (from_scope(b, nullptr)) {
      async = false;
      return;
    }
    if (hipMalloc(&p, b) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error{HM_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed"};
    }
    bytes = b;
    async = false;
  }
  // a cached block used on stream s only: it returns once s is idle, so
  // work of other streams is not waited on
  void scratch(size_t b, hipStream_t s) {
    cached(b);
    st = s;
    stream_owned = true;
  }
  void cached(size_t b) {
    release();
    if (b == 0) b = 64;
    b = (b + 255) / 256 * 256;
    if (from_scope(b, nullptr)) {
      async = false;
      return;
    }
    if (hipGetDevice(&dev) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{HM_E_DEVICE, "hipGetDevice failed"};
    }
    if (dev < 0 || dev >= 64) {  // beyond the cache's table: a plain allocation
      alloc(b);
      return;
    }
    size_t blk = b;
    p = cache_take(dev, blk);
    if (!p) {
      if (hipMalloc(&p, b) != hipSuccess) {
        (void)hipGetLastError();
        cache_drop(dev);
        if (hipMalloc(&p, b) != hipSuccess) {
          p = nullptr;
          (void)hipGetLastError();
          throw Error{HM_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed"};
        }
      }
      blk = b;
    }
    bytes = b;
    cap = blk;
    async = false;
    in_cache = true;
  }
  void temp(size_t b, hipStream_t s) {
    release();
    if (b == 0) b = 64;
    if (from_scope(b, s)) {
      async = true;
      return;
    }
    if (hipMallocAsync(&p, b, s) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error{HM_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed"};
    }
    bytes = b;
    st = s;
    async = true;
  }
  void release() {
    if (p && al.free) {
      // stream-ordered scratch goes back at once (the allocator orders its
      // reuse on that stream); other blocks once their work is done
      if (!async && !release_synced())
        (void)(stream_owned ? hipStreamSynchronize(st) : hipDeviceSynchronize());
      al.free(al.ctx, p, (void *)st);
      al = hm_allocator{};
    } else if (p && in_cache) {
      if (!release_synced()) (void)(stream_owned ? hipStreamSynchronize(st) : hipDeviceSynchronize());
      cache_put(dev, p, cap);
    } else if (p) {
      (void)(async ? hipFreeAsync(p, st) : hipFree(p));
    }
    p = nullptr;
    bytes = 0;
    in_cache = false;
    stream_owned = false;
  }
  template <class T>
  T *as() const {
    return (T *)p;
  }
};

template <class T>
void upload(DBuf &d, const std::vector<T> &v, hipStream_t s) {
  d.alloc(v.size() * sizeof(T));
  if (!v.empty())
    HIP_TRY(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// upload into a cached block (the buffers of H-matrices)
template <class T>
void upload_cached(DBuf &d, const std::vector<T> &v, hipStream_t s) {
  d.cached(v.size() * sizeof(T));
  if (!v.empty())
    HIP_TRY(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}


inline int64_t pad16(int64_t x) { return (x + 15) / 16 * 16; }

// ------------------------------------------------------------------ device tree
struct DeviceTree {
  SyncedRelease rel;  // first: destroyed last
  int device = -1;
  ~DeviceTree() { rel.begin(device); }
  DBuf pts;                    // dim x n, tree order
  DBuf perm;                   // n (tree -> original)
  std::vector<DBuf> rowbox;    // per level: box of every row
  std::vector<DBuf> start;     // per level: box starts
  DBuf inst_off;               // ninst + 1 row offsets of the instances
  DBuf kitems;                 // forest: full-width kernel-apply items
  int32_t nkitems = 0;
};

// Kernel-apply work items of a forest: every 64-row block of every
// instance, instances in decreasing size (the long contractions start
// first); width[i] = live columns of instance i.
std::vector<KItem> forest_items(const Tree &T, const std::vector<int32_t> &width) {
  std::vector<int> order(T.ninst());
  for (int i = 0; i < T.ninst(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return T.inst_off[a + 1] - T.inst_off[a] > T.inst_off[b + 1] - T.inst_off[b];
  });
  std::vector<KItem> it;
  for (int i : order) {
    const int64_t n = T.inst_off[i + 1] - T.inst_off[i];
    for (int64_t r0 = 0; r0 < n; r0 += 64)
      it.push_back(KItem{T.inst_off[i], (int32_t)n, (int32_t)r0, width[i], 0});
  }
  return it;
}

DeviceTree &device_tree(Tree &T, hipStream_t s) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (T.dev && T.dev->device == dev) return *T.dev;
  auto D = std::make_shared<DeviceTree>();
  D->device = dev;
  std::vector<double> soa((size_t)T.dim * T.n);
  for (int64_t i = 0; i < T.n; ++i)
    for (int d = 0; d < T.dim; ++d) soa[(size_t)d * T.n + i] = T.pts[T.perm[i] * T.dim + d];
  upload_cached(D->pts, soa, s);
  upload_cached(D->perm, T.perm, s);
  D->rowbox.resize(T.nlev());
  D->start.resize(T.nlev());
  for (int l = 0; l < T.nlev(); ++l) {
    std::vector<int32_t> rb(T.n);
    const Level &Lv = T.lev[l];
    for (int b = 0; b < Lv.nbox(); ++b)
      for (int64_t i = Lv.start[b]; i < Lv.start[b + 1]; ++i) rb[i] = b;
    upload_cached(D->rowbox[l], rb, s);
    upload_cached(D->start[l], Lv.start, s);
  }
  upload_cached(D->inst_off, T.inst_off.empty() ? std::vector<int64_t>{0, T.n} : T.inst_off, s);
  if (T.ninst() > 1) {
    std::vector<KItem> it = forest_items(T, std::vector<int32_t>(T.ninst(), INT32_MAX));
    upload_cached(D->kitems, it, s);
    D->nkitems = (int32_t)it.size();
  }
  HIP_TRY(hipStreamSynchronize(s));
  T.dev = D;
  return *D;
}

// ------------------------------------------------------------------ black boxes
struct KernelBB {
  Tree *tree;
  int kernel;
};

// Y = K X in tree order; block-diagonal over the instances of a forest.
// With a slice budget on this thread (kapply_slice_flops) a whole-operator
// apply runs as consecutive launches of row blocks, each about that many
// flops.
void kernel_apply_tree(const Tree &T, int kernel, int64_t ncols, bool f32, const void *X,
                       int64_t ldx, void *Y, int64_t ldy, hipStream_t s) {
  const DeviceTree &D = *T.dev;
  const bool forest = T.ninst() > 1;
  const int64_t units = forest ? D.nkitems : (T.n + 63) / 64;
  const double slice = kapply_slice_flops();
  autotune_kapply(KapplyShape{f32, kernel, T.dim, ncols, T.n, forest, units},
                  [&](int nt, int64_t part) {
                    if (forest) {
                      launch_kapply_forest(kernel, T.dim, T.n, D.pts.as<double>(),
                                           part > 0 ? (int32_t)part : D.nkitems,
                                           D.kitems.as<KItem>(), ncols, -1, nt, f32, X, ldx, Y,
                                           ldy, s);
                    } else if (part > 0 || !(slice > 0)) {
                      launch_kapply(kernel, T.dim, T.n, D.pts.as<double>(), ncols, nt, f32, X,
                                    ldx, Y, ldy, s, part * 64);
                    } else {
                      // about `slice` flops per launch, and at least 1024
                      // workgroups (4 per CU) so that a slice fills the device
                      const double per_blk = 2.0 * (double)T.n * 64.0 * (double)ncols;
                      const int ntw = nt > 0 ? nt : kapply_default_nt(ncols, f32, units);
                      const int64_t nct = (ncols + 16 * ntw - 1) / (16 * ntw);
                      const int64_t blks = std::max<int64_t>(
                          {(int64_t)1, (int64_t)(slice / std::max(per_blk, 1.0)),
                           (1024 + nct - 1) / std::max<int64_t>(nct, 1)});
                      // At most two slices queued at a time: the host waits for
                      // slice i - 1 before it enqueues slice i + 1.  A stream
                      // that shares this stream's hardware queue (more streams
                      // than queues) then waits behind two slices, not behind
                      // the whole apply, and the next slice still fills the
                      // tail of the one before.  Not under graph capture.
                      hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
                      (void)hipStreamIsCapturing(s, &cap);
                      (void)hipGetLastError();
                      hipEvent_t ev[2] = {nullptr, nullptr};
                      const bool pace = cap == hipStreamCaptureStatusNone &&
                                        hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) ==
                                            hipSuccess &&
                                        hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) ==
                                            hipSuccess;
                      (void)hipGetLastError();
                      int64_t i = 0;
                      for (int64_t b = 0; b < units; b += blks, ++i) {
                        if (pace && i >= 2) (void)hipEventSynchronize(ev[i & 1]);
                        launch_kapply(kernel, T.dim, T.n, D.pts.as<double>(), ncols, nt, f32, X,
                                      ldx, Y, ldy, s, blks * 64, b * 64);
                        if (pace) (void)hipEventRecord(ev[i & 1], s);
                      }
                      for (hipEvent_t e : ev)
                        if (e) (void)hipEventDestroy(e);
                    }
                  },
                  s);
}

int kernel_bb_apply(void *ctx, int /*transpose*/, int64_t n, int64_t ncols, int dtype,
                    const void *X, int64_t ldx, void *Y, int64_t ldy, void *stream) {
  KernelBB *k = (KernelBB *)ctx;
  if (!k || !k->tree || !k->tree->dev || n != k->tree->n) return 1;
  kernel_apply_tree(*k->tree, k->kernel, ncols, dtype == HM_F32, X, ldx, Y, ldy,
                    (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

struct DenseBB {
  const double *A;
  int64_t n, lda;
};

int dense_bb_apply(void *ctx, int transpose, int64_t n, int64_t ncols, int dtype, const void *X,
                   int64_t ldx, void *Y, int64_t ldy, void *stream) {
  DenseBB *d = (DenseBB *)ctx;
  if (!d || n != d->n || dtype != HM_F64) return 1;
  launch_dense_gemm(n, d->A, d->lda, transpose != 0, ncols, (const double *)X, ldx, (double *)Y,
                    ldy, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // namespace hm

// ------------------------------------------------------------------ the H-matrix
struct hm_hmatrix {
  hm::SyncedRelease rel;  // first: destroyed last
  hm_allocator al{};      // the caller's allocator its blocks came from (and its applies' scratch)
  struct Lv {
    int level = 0;
    int64_t np = 0;   // pairs
    int64_t g0 = 0;   // first global pair index
    std::vector<int32_t> pa, pb;
    std::vector<int64_t> offU, offV, offW, offB;
  };
  // Apply plan of one orientation (A, or A* with the roles of U and V swapped)
  struct Orient {
    hm::DBuf items, ppairs;              // projection work, levels in order
    hm::DBuf red;                        // pairs split over several segments
    std::vector<int32_t> red_upto;       // [li]: reduce items of the first li levels
    std::vector<int32_t> items_upto;     // [li]: items of the first li levels
    std::vector<int32_t> slots_upto;     // [li]: partial slots of the first li levels
    std::vector<hm::DBuf> chunks, entries;  // [li]: expand plan of the first li levels
    std::vector<int32_t> nch;
  };
  int device = 0;
  int64_t n = 0;
  int nlev = 0;
  int32_t r = 0, kmax = 0;
  int64_t np_total = 0;
  std::vector<std::vector<int64_t>> start;  // host box starts per level
  hm::DBuf perm;
  hm::DBuf U, V, W, B, Vf, Wf, D;
  hm::DBuf ranks;                  // [0, np): rank_u, [np, 2np): rank_v
  std::vector<int32_t> h_ranks;
  std::vector<Lv> lv;
  // leaf neighbor blocks
  std::vector<int32_t> na, nb;
  std::vector<int64_t> offD;
  hm::DBuf nchunks, nentries;
  hm::DBuf nchunksT, nentriesT;   // same chunks, entries of the adjoint
  int32_t nnch = 0;
  bool near_covers = false;        // the near chunks cover every row once
  int64_t max_np = 0;
  Orient oA, oT;
  // uniform format: the shared bases, one per box with a non-empty
  // interaction list (ubox[li], ascending), U_a in UB and V_a in VB at
  // uoff[li][v] (m x kmax, ld = m); brank [0, nvtot) U ranks, [nvtot, 2 nvtot)
  // V ranks, level li's vertices from uv0[li]
  int32_t format = HM_FORMAT_H1;
  hm::DBuf UB, VB, brank;
  // H^2: singular values (kmax per box) and transfers (kmax x kmax per box,
  // to its parent); UB / VB hold the bases implied by the nesting
  hm::DBuf SU, SV, TU, TV;
  // H^2 apply plan: boxes with long bases (whole, and 64-row chunks), per
  // level the upward sums (transfers of the children) and the downward sums
  // (couplings and the parent term) of the operator and of its adjoint
  struct H2Apply {
    hm::DBuf leaf, chunk;
    int32_t nleaf = 0, nchunk = 0;
    // [li]: boxes projected and expanded by the operator of the first li
    // levels (the level-truncated product of the peel): the boxes of level
    // li - 1 and the coarser ones without children holding bases
    std::vector<hm::DBuf> tleaf, tchunk;
    std::vector<int32_t> ntleaf, ntchunk;
    std::vector<hm::DBuf> up_j, up_t, dn_j, dn_t, dnt_j, dnt_t;
    std::vector<int32_t> nup, ndn;
    bool ready = false;
  } h2a;
  std::vector<std::vector<int32_t>> ubox;
  std::vector<std::vector<int64_t>> uoff;
  std::vector<int64_t> uv0;
  int64_t nvtot = 0;
  std::vector<int32_t> h_brank;
  hm_stats stats{};
  // the buffers return to the block cache once the device is idle
  ~hm_hmatrix() { rel.begin(device); }
};

namespace hm {

namespace {

constexpr int kSeg = 256;  // rows per projection segment of the applies' plans

// Low-rank product plans of both orientations (levels in order), into A and
// At.  Projection items group up to 128/kmax pairs that share a column box
// and cover one segment of `seg` rows of it (seg <= 0: the whole box); each
// pair owns one partial slot per segment.  The expand plan for the first li
// levels walks 64-row chunks of the finest of them and lists every pair
// whose row box (at its own level) contains the chunk; it is built for
// every li (prefixes, the peel's level-truncated products) or only for all
// levels (the applies of the finished matrix).
//   The applies of a finished H-matrix (few right-hand sides) take segments
// of 256 rows: parallel work over the rows of the large boxes of the coarse
// levels, the partials summed once (lr_reduce_kernel).  The peel (thousands
// of columns, parallel over column tiles) takes whole boxes: no partial
// slots to write, sum and read back, and fewer slots, so fewer column chunks.
void build_plans(const hm_hmatrix &H, const Tree &T, int32_t seg, bool prefixes,
                 hm_hmatrix::Orient &A, hm_hmatrix::Orient &At, hipStream_t s) {
  const int nlv = (int)H.lv.size();
  // pairs of one column box per projection item, at most 128 rank columns
  const int per_group = std::max(1, 128 / std::max(1, (int)H.kmax));
  for (int o = 0; o < 2; ++o) {
    const bool trans = o == 1;
    hm_hmatrix::Orient &O = trans ? At : A;
    std::vector<ProjItem> items;
    std::vector<ProjPair> pps;
    std::vector<ReduceItem> reds;
    O.red_upto.assign(1, 0);
    O.items_upto.assign(1, 0);
    O.slots_upto.assign(1, 0);
    std::vector<std::vector<int32_t>> slot_base(nlv), nseg(nlv);
    int32_t slots = 0;
    for (int li = 0; li < nlv; ++li) {
      const hm_hmatrix::Lv &L = H.lv[li];
      const Level &Lev = T.lev[L.level];
      const std::vector<int32_t> &colbox = trans ? L.pa : L.pb;
      const std::vector<int64_t> &roff = trans ? L.offW : L.offV;
      slot_base[li].resize(L.np);
      nseg[li].resize(L.np);
      for (int64_t p = 0; p < L.np; ++p) {
        const int64_t m = Lev.start[colbox[p] + 1] - Lev.start[colbox[p]];
        nseg[li][p] = seg > 0 ? (int32_t)((m + seg - 1) / seg) : 1;
        slot_base[li][p] = slots;
        if (nseg[li][p] > 1) reds.push_back(ReduceItem{slots, nseg[li][p]});
        slots += nseg[li][p];
      }
      O.red_upto.push_back((int32_t)reds.size());
      std::vector<int64_t> order(L.np);
      for (int64_t p = 0; p < L.np; ++p) order[p] = p;
      std::stable_sort(order.begin(), order.end(),
                       [&](int64_t a, int64_t b) { return colbox[a] < colbox[b]; });
      int64_t i = 0;
      while (i < L.np) {
        const int cb = colbox[order[i]];
        int64_t j = i;
        while (j < L.np && colbox[order[j]] == cb && j - i < per_group) ++j;
        const int32_t m = (int32_t)(Lev.start[cb + 1] - Lev.start[cb]);
        const int32_t sl = seg > 0 ? seg : std::max(m, 1);
        for (int32_t sg = 0; sg * sl < m; ++sg) {
          ProjItem it{Lev.start[cb] + (int64_t)sg * sl, std::min(sl, m - sg * sl), sg * sl,
                      m, (int32_t)(j - i), (int32_t)pps.size(), 0};
          for (int64_t q = i; q < j; ++q) {
            const int64_t p = order[q];
            pps.push_back(ProjPair{roff[p], (int32_t)(H.np_total + L.g0 + p), slot_base[li][p] + sg});
          }
          items.push_back(it);
        }
        i = j;
      }
      O.items_upto.push_back((int32_t)items.size());
      O.slots_upto.push_back(slots);
    }
    upload_cached(O.items, items, s);
    upload_cached(O.ppairs, pps, s);
    upload_cached(O.red, reds, s);
    HIP_TRY(hipStreamSynchronize(s));
    // expand plans
    O.chunks.clear();
    O.entries.clear();
    O.nch.assign(nlv + 1, 0);
    O.chunks.resize(nlv + 1);
    O.entries.resize(nlv + 1);
    // rows grouped by row box, per level
    std::vector<std::vector<int32_t>> rb_ptr(nlv), rb_idx(nlv);
    for (int li = 0; li < nlv; ++li) {
      const hm_hmatrix::Lv &L = H.lv[li];
      const int nb = T.lev[L.level].nbox();
      const std::vector<int32_t> &rowbox = trans ? L.pb : L.pa;
      rb_ptr[li].assign(nb + 1, 0);
      for (int64_t p = 0; p < L.np; ++p) rb_ptr[li][rowbox[p] + 1]++;
      for (int b = 0; b < nb; ++b) rb_ptr[li][b + 1] += rb_ptr[li][b];
      rb_idx[li].resize(L.np);
      std::vector<int32_t> fill(rb_ptr[li].begin(), rb_ptr[li].end() - 1);
      for (int64_t p = 0; p < L.np; ++p) rb_idx[li][fill[rowbox[p]]++] = (int32_t)p;
    }
    // (a tree with no sampled level has no plan: nlv = 0, no iteration)
    for (int le = prefixes ? 1 : std::max(nlv, 1); le <= nlv; ++le) {
      const int fl = H.lv[le - 1].level;
      const Level &F = T.lev[fl];
      std::vector<ExpandChunk> ch;
      std::vector<ExpandEntry> en;
      std::vector<int32_t> anc(le);
      for (int b = 0; b < F.nbox(); ++b) {
        // ancestors of b at the levels of the plan
        int box = b, lvl = fl;
        for (int li = le - 1; li >= 0; --li) {
          const int tl = H.lv[li].level;
          while (lvl > tl) box = T.lev[lvl--].parent[box];
          anc[li] = box;
        }
        const int32_t mb = (int32_t)(F.start[b + 1] - F.start[b]);
        for (int32_t off = 0; off < mb; off += 64) {
          ExpandChunk c{F.start[b] + off, std::min<int32_t>(64, mb - off), (int32_t)en.size(), 0, 0};
          for (int li = 0; li < le; ++li) {
            const hm_hmatrix::Lv &L = H.lv[li];
            const Level &Lev = T.lev[L.level];
            const int a = anc[li];
            const std::vector<int64_t> &loff = trans ? L.offV : L.offW;
            for (int32_t q = rb_ptr[li][a]; q < rb_ptr[li][a + 1]; ++q) {
              const int32_t p = rb_idx[li][q];
              en.push_back(ExpandEntry{loff[p], (int32_t)(Lev.start[a + 1] - Lev.start[a]),
                                       (int32_t)(c.row0 - Lev.start[a]),
                                       (int32_t)(H.np_total + L.g0 + p), slot_base[li][p],
                                       nseg[li][p], 0});
            }
          }
          c.last = (int32_t)en.size();
          if (c.last > c.first) ch.push_back(c);
        }
      }
      upload_cached(O.chunks[le], ch, s);
      upload_cached(O.entries[le], en, s);
      O.nch[le] = (int32_t)ch.size();
      HIP_TRY(hipStreamSynchronize(s));
    }
  }
}

// The peel's zero pattern of X and the scratch for the projection's tile
// flags (bytes; one per slot and 64-column tile of a column chunk)
struct PeelPattern {
  ColorPattern pat;
  uint8_t *flags;
  int64_t flag_cap;
};

// Y +=/-= (first li_end levels of H) X; T is scratch of tcap elements.
// pp: X is a colored test matrix with that zero pattern (peel plans only).
void apply_levels(const hm_hmatrix &H, size_t li_end, bool trans, bool f32, const void *X,
                  int64_t ldx, int64_t ncols, void *Y, int64_t ldy, double sign, void *T,
                  int64_t tcap, hipStream_t s, const hm_hmatrix::Orient *plans = nullptr,
                  const PeelPattern *pp = nullptr) {
  if (li_end == 0 || ncols <= 0) return;
  // plans: the two orientations' plans to use (the peel's), else the matrix's own
  const hm_hmatrix::Orient &O = plans ? plans[trans ? 1 : 0] : (trans ? H.oT : H.oA);
  if (O.items_upto.size() <= li_end || O.chunks.size() <= li_end || O.nch.size() <= li_end)
    throw Error{HM_E_STATE, "no per-pair apply plan for these levels"};
  const int32_t nitems = O.items_upto[li_end];
  const int64_t nslots = O.slots_upto[li_end];
  if (nitems == 0 || O.nch[li_end] == 0) return;
  const size_t es = f32 ? 4 : 8;
  const void *Rp = trans ? (f32 ? H.Wf.p : H.W.p) : (f32 ? H.Vf.p : H.V.p);
  const void *Lp = trans ? (f32 ? H.Vf.p : H.V.p) : (f32 ? H.Wf.p : H.W.p);
  int64_t cw = tcap / (nslots * H.kmax);
  if (cw < 1) throw Error{HM_E_NOMEM, "low-rank scratch too small"};
  cw = std::min<int64_t>(cw, ncols);
  if (cw < ncols && cw >= 64) cw = cw / 64 * 64;
  // a tile the projection leaves unwritten must not reach a reduction
  if (pp && O.red_upto[li_end] > 0)
    throw Error{HM_E_STATE, "zero-pattern projection on segmented plans"};
  for (int64_t c0 = 0; c0 < ncols; c0 += cw) {
    const int64_t w = std::min(cw, ncols - c0);
    const int64_t tstride = (int64_t)H.kmax * w;
    ColorPattern cp{};
    uint8_t *flags = nullptr;
    if (pp) {
      cp = pp->pat;
      cp.col0 += c0;
      flags = pp->flags;
      if (nslots * ((w + kLowRankTile - 1) / kLowRankTile) > pp->flag_cap)
        throw Error{HM_E_STATE, "projection flag scratch too small"};
    }
    launch_lr_project(nitems, O.items.as<ProjItem>(), O.ppairs.as<ProjPair>(), H.kmax, tstride,
                      H.ranks.as<int32_t>(), f32, Rp, (const char *)X + c0 * ldx * es, ldx, w, T,
                      pp ? &cp : nullptr, flags, s);
    // partials of pairs split over segments summed once, not per output chunk
    launch_lr_reduce(O.red_upto[li_end], O.red.as<ReduceItem>(), tstride, tstride, f32, T, s);
    LAUNCH_CHECK();
    launch_lr_expand(O.nch[li_end], O.chunks[li_end].as<ExpandChunk>(),
                     O.entries[li_end].as<ExpandEntry>(), H.kmax, tstride, H.ranks.as<int32_t>(),
                     f32, Lp, T, w, sign, (char *)Y + c0 * ldy * es, ldy, flags, s);
    LAUNCH_CHECK();
  }
}

// Partial projections of the low-rank products: every slot at full width,
// capped at 1 G elements (8 GB in FP64).  The products run over the columns
// in chunks of cap / (slots kmax), and every chunk reads the coarser levels'
// factors again, so a wide sample (thousands of columns) wants few chunks;
// the device holds 288 GB.
constexpr int64_t kTScratchCap = int64_t(1) << 30;

int64_t tscratch_elems(const hm_hmatrix &H, int64_t ncols) {
  const int64_t slots = std::max<int32_t>(
      H.oA.slots_upto.empty() ? 0 : H.oA.slots_upto.back(),
      H.oT.slots_upto.empty() ? 0 : H.oT.slots_upto.back());
  int64_t need = slots * H.kmax * std::max<int64_t>(ncols, 1);
  int64_t cap = kTScratchCap;
  int64_t minimum = slots * H.kmax * 64;
  return std::max<int64_t>(std::min(need, cap), std::max<int64_t>(minimum, 64));
}

// The H^2 part of Y += sign H X (or H* X) through the nested representation
// (alg:apply_h2_level_truncated): outgoing expansions of the boxes with
// long bases, upward pass, couplings and downward pass, expansion.  With
// le < the number of levels, the operator of the first le levels (the
// level-truncated product of the peel): its long bases are those of level
// le - 1 and of the coarser boxes without children holding bases.
// Expansions in QH / UH (nvtot x kmax x qcols each) when given, else in
// stream-ordered scratch; at most 256 columns at a time.
void h2_apply(const hm_hmatrix &H, size_t le, bool trans, bool f32, const void *X, int64_t ldx,
              int64_t ncols, void *Y, int64_t ldy, double sign, double *qh, double *uh,
              double *part, int64_t qcols, hipStream_t s) {
  const hm_hmatrix::H2Apply &P = H.h2a;
  const size_t nlv = H.lv.size();
  if (le == 0 || ncols <= 0) return;
  if (le > nlv) le = nlv;
  const int32_t kmax = H.kmax;
  const int64_t nb = H.nvtot;
  const int32_t *Ur = H.brank.as<int32_t>(), *Vr = Ur + nb;
  const int32_t *ro = trans ? Vr : Ur, *ri = trans ? Ur : Vr;  // incoming / outgoing ranks
  const double *Bout = trans ? H.UB.as<double>() : H.VB.as<double>();  // applied to x
  const double *Bin = trans ? H.VB.as<double>() : H.UB.as<double>();   // expands into y
  const double *Tup = trans ? H.TU.as<double>() : H.TV.as<double>();
  const double *Tdn = trans ? H.TV.as<double>() : H.TU.as<double>();
  const bool full = le == nlv;
  const H2Leaf *leaf = (full ? P.leaf : P.tleaf[le]).as<H2Leaf>();
  const H2Leaf *chunk = (full ? P.chunk : P.tchunk[le]).as<H2Leaf>();
  const int32_t nleaf = full ? P.nleaf : P.ntleaf[le];
  const int32_t nchunk = full ? P.nchunk : P.ntchunk[le];
  const size_t es = f32 ? 4 : 8;
  const bool own = qh == nullptr;
  const int64_t cw = own ? std::min<int64_t>(ncols, 256) : std::min<int64_t>(ncols, qcols);
  if (cw < 1) throw Error{HM_E_NOMEM, "H2 expansion scratch too small"};
  double *QH = qh, *UH = uh, *PT = part;
  StreamBlock oq, ou, op;
  if (own) {
    oq.take((size_t)std::max<int64_t>(nb * kmax * cw, 1) * 8, s);
    ou.take((size_t)std::max<int64_t>(nb * kmax * cw, 1) * 8, s);
    op.take((size_t)std::max<int64_t>((int64_t)nchunk * kmax * cw, 1) * 8, s);
    QH = (double *)oq.p;
    UH = (double *)ou.p;
    PT = (double *)op.p;
  }
  for (int64_t c0 = 0; c0 < ncols; c0 += cw) {
    const int64_t w = std::min(cw, ncols - c0);
    const char *Xc = (const char *)X + c0 * ldx * es;
    char *Yc = (char *)Y + c0 * ldy * es;
    launch_h2_project(nchunk, chunk, kmax, ri, Bout, f32, Xc, ldx, w, PT, w, s);
    launch_h2_reduce(nleaf, leaf, kmax, PT, QH, w, w, s);
    // upward: level li from its children on li + 1 (< le)
    for (size_t li = le - 1; li-- > 0;)
      launch_h2_sum(P.nup[li], P.up_j[li].as<H2Sum>(), P.up_t[li].as<H2Term>(), kmax, ri, ri,
                    Tup, Tup, QH, QH, QH, w, w, s);
    for (size_t li = 0; li < le; ++li)
      launch_h2_sum(P.ndn[li], (trans ? P.dnt_j[li] : P.dn_j[li]).as<H2Sum>(),
                    (trans ? P.dnt_t[li] : P.dn_t[li]).as<H2Term>(), kmax, ro, ri,
                    H.B.as<double>(), Tdn, QH, UH, UH, w, w, s);
    launch_h2_expand(nchunk, chunk, kmax, ro, Bin, UH, w, f32, w, Yc, ldy, sign, s);
    LAUNCH_CHECK();
  }
}

// Y = H X or H* X (rows in `order`); stream-ordered scratch.
void matvec_impl(const hm_hmatrix &H, bool trans, int64_t nrhs, bool f32, const void *X,
                 int64_t ldx, void *Y, int64_t ldy, int order, hipStream_t s) {
  // the H-matrix's allocator (if it was made with one) for the scratch
  AllocScope scope(H.al.alloc ? &H.al : nullptr);
  const size_t es = f32 ? 4 : 8;
  const int64_t n = H.n;
  const bool h2 = H.format == HM_FORMAT_H2 && H.h2a.ready;
  const int64_t tcap = h2 ? 0 : tscratch_elems(H, nrhs);
  StreamBlock tb, xb, yb;
  if (!h2) tb.take((size_t)tcap * es, s);
  void *Tb = tb.p, *xt = nullptr, *yt = nullptr;
  const bool orig = order != HM_ORDER_TREE;
  const void *Xt = X;
  void *Yt = Y;
  int64_t ldxt = ldx, ldyt = ldy;
  if (orig) {
    xb.take((size_t)n * nrhs * es, s);
    yb.take((size_t)n * nrhs * es, s);
    xt = xb.p;
    yt = yb.p;
    launch_permute_rows(n, nrhs, H.perm.as<int64_t>(), false, f32, X, ldx, xt, n, s);
    Xt = xt;
    Yt = yt;
    ldxt = ldyt = n;
  }
  // the near field writes Y first when it covers every row, else Y starts at 0
  if (!H.near_covers) launch_fill_cols(Yt, n, nrhs, ldyt, f32, s);
  launch_near_apply(H.nnch, (trans ? H.nchunksT : H.nchunks).as<ExpandChunk>(),
                    (trans ? H.nentriesT : H.nentries).as<NearEntry>(), f32, H.D.p, Xt, ldxt,
                    nrhs, Yt, ldyt, H.near_covers, s);
  LAUNCH_CHECK();
  if (h2)
    h2_apply(H, H.lv.size(), trans, f32, Xt, ldxt, nrhs, Yt, ldyt, 1.0, nullptr, nullptr, nullptr,
             0, s);
  else
    apply_levels(H, H.lv.size(), trans, f32, Xt, ldxt, nrhs, Yt, ldyt, 1.0, Tb, tcap, s);
  LAUNCH_CHECK();
  if (orig) {
    launch_permute_rows(n, nrhs, H.perm.as<int64_t>(), true, f32, yt, n, Y, ldy, s);
    LAUNCH_CHECK();
  }
}

// Y = H X or H* X (rows in `order`) with every scratch buffer carved out of
// buf (cap bytes, 256-aligned): the columns go through in blocks sized so
// that the block's order-conversion copies and the apply's expansions fit.
// Every byte of buf that a block reads is written earlier in that block.
void matvec_in(const hm_hmatrix &H, bool trans, int64_t nrhs, bool f32, const void *X,
               int64_t ldx, void *Y, int64_t ldy, int order, unsigned char *buf, size_t cap,
               hipStream_t s) {
  const size_t es = f32 ? 4 : 8;
  const int64_t n = H.n;
  const bool orig = order != HM_ORDER_TREE;
  const bool h2 = H.format == HM_FORMAT_H2 && H.h2a.ready;
  const int64_t nslots = std::max<int64_t>(
      H.oA.slots_upto.empty() ? 0 : H.oA.slots_upto.back(),
      H.oT.slots_upto.empty() ? 0 : H.oT.slots_upto.back());
  const size_t stage = orig ? (size_t)n * es : 0;  // per column, each of the two copies
  const size_t work = h2 ? (size_t)(2 * H.nvtot + H.h2a.nchunk) * H.kmax * 8
                         : (size_t)std::max<int64_t>(nslots, 1) * H.kmax * es;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t fixed = 8 * 256;  // alignment slack of the pieces
  const size_t per_col = 2 * stage + work;
  if (cap <= fixed || per_col > cap - fixed)
    throw Error{HM_E_ARG, "hm_matvec_static: one right-hand side needs " +
                              std::to_string(per_col + fixed) + " bytes of scratch, the static "
                              "scratch holds " + std::to_string(cap)};
  const int64_t cw = std::min<int64_t>(nrhs, (int64_t)((cap - fixed) / per_col));
  unsigned char *xt = buf, *yt = xt + up(stage * cw), *wk = yt + up(stage * cw);
  for (int64_t c0 = 0; c0 < nrhs; c0 += cw) {
    const int64_t w = std::min(cw, nrhs - c0);
    const void *Xc = (const char *)X + c0 * ldx * es;
    void *Yc = (char *)Y + c0 * ldy * es;
    const void *Xt = Xc;
    void *Yt = Yc;
    int64_t ldxt = ldx, ldyt = ldy;
    if (orig) {
      launch_permute_rows(n, w, H.perm.as<int64_t>(), false, f32, Xc, ldx, xt, n, s);
      Xt = xt;
      Yt = yt;
      ldxt = ldyt = n;
    }
    if (!H.near_covers) launch_fill_cols(Yt, n, w, ldyt, f32, s);
    launch_near_apply(H.nnch, (trans ? H.nchunksT : H.nchunks).as<ExpandChunk>(),
                      (trans ? H.nentriesT : H.nentries).as<NearEntry>(), f32, H.D.p, Xt, ldxt,
                      w, Yt, ldyt, H.near_covers, s);
    LAUNCH_CHECK();
    if (h2) {
      double *qh = (double *)wk;
      double *uh = (double *)(wk + up((size_t)H.nvtot * H.kmax * w * 8));
      double *pt = (double *)((unsigned char *)uh + up((size_t)H.nvtot * H.kmax * w * 8));
      h2_apply(H, H.lv.size(), trans, f32, Xt, ldxt, w, Yt, ldyt, 1.0, qh, uh, pt, w, s);
    } else {
      apply_levels(H, H.lv.size(), trans, f32, Xt, ldxt, w, Yt, ldyt, 1.0, wk,
                   std::max<int64_t>(nslots, 1) * H.kmax * w, s);
    }
    LAUNCH_CHECK();
    if (orig) {
      launch_permute_rows(n, w, H.perm.as<int64_t>(), true, f32, yt, n, Yc, ldy, s);
      LAUNCH_CHECK();
    }
  }
}

// ------------------------------------------------------------------ operator black boxes
// A compressed operator as a black box (hm_matvec / its adjoint).
struct HMatrixBB {
  const hm_hmatrix *H;
  int order;
};

int hmatrix_bb_apply(void *ctx, int transpose, int64_t n, int64_t ncols, int dtype, const void *X,
                     int64_t ldx, void *Y, int64_t ldy, void *stream) {
  HMatrixBB *b = (HMatrixBB *)ctx;
  if (!b || !b->H || n != b->H->n || (dtype != HM_F64 && dtype != HM_F32)) return 1;
  if (ncols <= 0) return 0;
  try {
    matvec_impl(*b->H, transpose != 0, ncols, dtype == HM_F32, X, ldx, Y, ldy, b->order,
                (hipStream_t)stream);
  } catch (const Error &e) {
    set_error(e.msg);
    return 2;
  }
  return 0;
}

// The product A B of two black boxes: Y = A (B X), Y = B* (A* X) for the
// adjoint, through a stream-ordered intermediate.
struct ProductBB {
  hm_blackbox A, B;
};

int product_bb_apply(void *ctx, int transpose, int64_t n, int64_t ncols, int dtype, const void *X,
                     int64_t ldx, void *Y, int64_t ldy, void *stream) {
  ProductBB *p = (ProductBB *)ctx;
  if (!p) return 1;
  if (ncols <= 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  const size_t es = dtype == HM_F32 ? 4 : 8;
  StreamBlock tb;
  try {
    tb.take((size_t)n * ncols * es, s);
  } catch (const Error &e) {
    set_error(e.msg);
    return 3;
  }
  void *tmp = tb.p;
  const hm_blackbox &first = transpose ? p->A : p->B;
  const hm_blackbox &second = transpose ? p->B : p->A;
  int rc = first.apply(first.ctx, transpose, n, ncols, dtype, X, ldx, tmp, n, stream);
  if (rc == 0) rc = second.apply(second.ctx, transpose, n, ncols, dtype, tmp, n, Y, ldy, stream);

  return rc;
}

struct Events {
  bool on = false;
  std::vector<std::pair<hipEvent_t, int>> marks;  // event, stage id
  hipStream_t s = nullptr;
  void mark(int stage) {
    if (!on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    marks.push_back({e, stage});
  }
  ~Events() {
    for (auto &m : marks) (void)hipEventDestroy(m.first);
  }
};

hm_status call_blackbox(const hm_blackbox &bb, int transpose, int64_t n, int64_t ncols, bool f32,
                        const void *X, int64_t ldx, void *Y, int64_t ldy, const DeviceTree &D,
                        DBuf &tmpx, DBuf &tmpy, hipStream_t s) {
  const int dtype = f32 ? HM_F32 : HM_F64;
  const size_t es = f32 ? 4 : 8;
  if (bb.order == HM_ORDER_TREE) {
    const int rc = bb.apply(bb.ctx, transpose, n, ncols, dtype, X, ldx, Y, ldy, (void *)s);
    if (rc != 0) throw Error{HM_E_CALLBACK, "black box returned " + std::to_string(rc)};
    return HM_OK;
  }
  const size_t need = (size_t)n * ncols * es;
  if (tmpx.bytes < need) tmpx.temp(need, s);
  if (tmpy.bytes < need) tmpy.temp(need, s);
  launch_permute_rows(n, ncols, D.perm.as<int64_t>(), true, f32, X, ldx, tmpx.p, n, s);
  LAUNCH_CHECK();
  const int rc = bb.apply(bb.ctx, transpose, n, ncols, dtype, tmpx.p, n, tmpy.p, n, (void *)s);
  if (rc != 0) throw Error{HM_E_CALLBACK, "black box returned " + std::to_string(rc)};
  launch_permute_rows(n, ncols, D.perm.as<int64_t>(), false, f32, tmpy.p, n, Y, ldy, s);
  LAUNCH_CHECK();
  return HM_OK;
}

double qr_flops(int64_t m, int64_t r, int64_t k) {
  double f = 2.0 * m * r;  // initial norms
  for (int64_t j = 0; j < k; ++j) f += 2.0 * (m - j) + 6.0 * (m - j) * (r - j - 1);
  for (int64_t j = 0; j < k; ++j) f += 4.0 * (m - j) * (k - j);
  return f;
}

// One compression.  setup() plans every launch and allocates every buffer;
// record() enqueues the whole device pipeline on a stream with no host round
// trip and no allocation, so once the autotuner has seen its shapes it can
// be captured into a HIP graph and replayed; finalize() reads the ranks
// back and fills the statistics.
struct Compression {
  SyncedRelease rel;           // first: destroyed last
  hipStream_t home = nullptr;  // the stream of the setup and the level work
  ~Compression() { rel.begin_stream(home); }
  Tree &T;
  hm_blackbox bb;
  hm_compress_opts o;
  bool persistent = false;  // buffers outlive the call (a plan): plain allocations
  int p = 10, kfix = 0, r = 0;
  int32_t kmax = 0;
  bool mixed = false;
  size_t es = 8;
  int64_t n = 0;
  DeviceTree *D = nullptr;
  std::unique_ptr<hm_hmatrix> H;
  std::vector<int> levels;
  int64_t np_total = 0, szU = 0, szV = 0, szB = 0, szD = 0;
  int32_t mw = 0;
  int64_t cmax = 0, leaf_cols = 0, wcols = 0, tcap = 0, cmax_np = 0;
  DBuf Xb, Yb, tmpx, tmpy, Tb, work, core, scratch, sat, flag, floor_u, floor_v;
  DBuf tflags, leaf_act;     // projection tile flags; leaf colors of every leaf box
  int64_t tflag_cap = 0;
  // host copies of the peel's zero patterns (the work count of finalize):
  // per level its (box, color) activity and color count (empty: the level's
  // peel runs dense), and the leaf pass's
  std::vector<std::vector<uint8_t>> h_act;
  std::vector<int32_t> h_act_nc;
  std::vector<uint8_t> h_leaf_act;
  struct LevelJobs {
    DBuf act, ju, jv, jc, kit;
    DBuf order;  // pairs by block size, largest first (the fused recovery's work list)
    int32_t nkit = 0;
  };
  DBuf counters;  // one work counter per level of the fused recovery
  hm_hmatrix::Orient peel_plans[2];  // the peel's low-rank product plans (A, A*)
  int recover_grid = 1024;
  std::vector<LevelJobs> jobs_of;
  int ni = 1;
  KernelBB *kbb = nullptr;
  bool direct = false;
  DBuf dib, dic, dkit, dr0, dc0, dma, dmb, doff;  // leaf pass lists
  int32_t nib = 0, nkit_leaf = 0;
  int64_t cols_A = 0, cols_At = 0;
  // uniform format (see hm_compress_opts.format)
  bool uniform = false;
  struct UniformJobs {
    DBuf act;          // stage-1 active (box, color) flags
    DBuf ju;           // stage-1 QR jobs, one per vertex
    DBuf slot;         // stage-2 (box, color) -> vertex + 1
    DBuf uoff;         // basis offsets per vertex
    DBuf mix, terms;   // combination jobs (row chunks) and their terms
    DBuf jv;           // row-basis QR jobs on S
    DBuf uc;           // per-pair coupling jobs
    DBuf kit1, kit2;   // forest kernel-apply items of the two stages
    // H^2: norm jobs of the raw samples (mixed floors), augmentation jobs of
    // the two stages, transfers and nesting of the previous level into this one
    DBuf jn, augu, augv, tr, nest;
    int32_t nv = 0, nmix = 0, nkit1 = 0, nkit2 = 0, naug = 0, ntr = 0, nnest = 0;
  };
  std::vector<UniformJobs> ujobs_of;
  DBuf Sb, usat;
  DBuf h2q, h2u, h2p;  // H^2: expansions of the level-truncated products, chunk partials
  int64_t h2cols = 0;  // columns they hold
  bool h2 = false;  // H^2: uniform stages with augmented SVD bases, nested
  void setup_uniform(hipStream_t s);
  void record_uniform_level(size_t li, hipStream_t s, Events &ev);
  void setup_h2(hipStream_t s);
  void build_h2_apply(const std::vector<std::vector<int32_t>> &vid, hipStream_t s);
  void record_h2_level(size_t li, hipStream_t s, Events &ev);
  void fp32_copies(size_t li, hipStream_t s);
  int inst_of_row(int64_t row) const {
    if (ni <= 1) return 0;
    return (int)(std::upper_bound(T.inst_off.begin(), T.inst_off.end(), row) -
                 T.inst_off.begin()) - 1;
  }

  hm_allocator al{};  // copy of the caller's allocator (o.allocator points here)
  Compression(Tree &t, const hm_blackbox &b, const hm_compress_opts &opt)
      : T(t), bb(b), o(opt) {
    if (opt.allocator && opt.allocator->alloc && opt.allocator->free) {
      al = *opt.allocator;
      o.allocator = &al;
    } else {
      o.allocator = nullptr;
    }
  }

  // scratch of one compression: cached blocks owned by its stream (the
  // compression waits for the stream before it ends), plain allocations for
  // a plan, whose captured launches keep them
  void buf(DBuf &d, size_t bytes, hipStream_t s) {
    if (persistent)
      d.alloc(bytes);
    else
      d.scratch(bytes, s);
  }
  template <class V>
  void put(DBuf &d, const std::vector<V> &v, hipStream_t s) {
    if (persistent) {
      upload(d, v, s);
    } else {
      d.scratch(v.size() * sizeof(V), s);
      if (!v.empty())
        HIP_TRY(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, s));
    }
  }
  // live colors of each instance in graph g
  std::vector<int32_t> inst_colors(int g) const {
    std::vector<int32_t> w(ni, 0);
    const Graph &Gg = T.graphs[g];
    for (int i = 0; i < ni; ++i)
      for (int64_t v = T.gvoff[g][i]; v < T.gvoff[g][i + 1]; ++v)
        w[i] = std::max(w[i], Gg.color[v] + 1);
    return w;
  }
  hm_status setup(hipStream_t s);
  void record(hipStream_t s, Events &ev);
  hm_status finalize(hipStream_t s, Events &ev,
                     std::chrono::steady_clock::time_point t_host0);
};

hm_status Compression::setup(hipStream_t s) {
  home = s;
  // ---------------- options
  if (T.n <= 0) return fail(HM_E_ARG, "empty tree");
  for (const Graph &G : T.graphs)
    if (!G.colored && G.nv() > 0) return fail(HM_E_STATE, "tree is not colored (hm_tree_color)");
  p = o.oversample > 0 ? o.oversample : 10;
  kfix = o.rank > 0 ? o.rank : 0;
  if (kfix == 0 && !(o.tol > 0)) return fail(HM_E_ARG, "need rank > 0 or tol > 0");
  r = o.r > 0 ? o.r : (kfix > 0 ? kfix + p : 0);
  if (r <= 0) return fail(HM_E_ARG, "tolerance mode needs r > 0");
  if (r > 64) return fail(HM_E_ARG, "r must be <= 64");
  if (kfix == 0 && r - p < 1) return fail(HM_E_ARG, "r - p must be >= 1 in tolerance mode");
  mixed = o.prec == HM_PREC_MIXED;
  if (mixed && !(bb.dtypes & (1 << HM_F32))) return fail(HM_E_ARG, "black box has no FP32 apply");
  if (!mixed && !(bb.dtypes & (1 << HM_F64))) return fail(HM_E_ARG, "black box has no FP64 apply");
  if (!bb.apply) return fail(HM_E_ARG, "black box without apply");
  if (o.format != HM_FORMAT_H1 && o.format != HM_FORMAT_UNIFORM_H1 && o.format != HM_FORMAT_H2)
    return fail(HM_E_ARG, "unknown format");
  uniform = o.format == HM_FORMAT_UNIFORM_H1 || o.format == HM_FORMAT_H2;
  h2 = o.format == HM_FORMAT_H2;
  if (uniform && mixed && !(bb.dtypes & (1 << HM_F64)))
    return fail(HM_E_ARG, "the uniform and H2 formats apply A* in FP64: black box has no FP64 apply");
  kmax = kfix > 0 ? std::min(kfix, r) : r - p;
  es = mixed ? 4 : 8;
  n = T.n;
  if (uniform) build_uniform_graphs(T);

  D = &device_tree(T, s);
  H = std::make_unique<hm_hmatrix>();
  if (o.allocator) H->al = al;
  HIP_TRY(hipGetDevice(&H->device));
  H->n = n;
  H->nlev = T.nlev();
  H->r = r;
  H->kmax = kmax;
  for (const Level &Lv : T.lev) H->start.push_back(Lv.start);
  H->perm.cached(n * sizeof(int64_t));
  HIP_TRY(hipMemcpyAsync(H->perm.p, D->perm.p, n * sizeof(int64_t), hipMemcpyDeviceToDevice, s));

  // ---------------- layout of the factor pools
  for (int l = 1; l < T.nlev(); ++l)
    if (!T.graphs[l].pa.empty()) levels.push_back(l);
  for (int l : levels) {
    const Graph &G = T.graphs[l];
    const Level &Lv = T.lev[l];
    hm_hmatrix::Lv L;
    L.level = l;
    L.np = (int64_t)G.pa.size();
    L.g0 = np_total;
    L.pa = G.pa;
    L.pb = G.pb;
    for (int64_t q = 0; q < L.np; ++q) {
      const int64_t ma = Lv.start[G.pa[q] + 1] - Lv.start[G.pa[q]];
      const int64_t mb = Lv.start[G.pb[q] + 1] - Lv.start[G.pb[q]];
      L.offU.push_back(szU);
      L.offW.push_back(szU);
      szU += ma * kmax;
      L.offV.push_back(szV);
      szV += mb * kmax;
      L.offB.push_back(szB);
      szB += (int64_t)kmax * kmax;
    }
    np_total += L.np;
    H->max_np = std::max(H->max_np, L.np);
    H->lv.push_back(std::move(L));
  }
  H->np_total = np_total;
  // H^2 applies through its passes: no per-pair copies of the bases, no
  // products W = U B, no FP32 copies (export reads the bases themselves)
  H->U.cached(h2 ? 0 : szU * 8);
  H->W.cached(h2 ? 0 : szU * 8);
  H->V.cached(h2 ? 0 : szV * 8);
  H->B.cached(szB * 8);
  H->Wf.cached(h2 ? 0 : szU * 4);
  H->Vf.cached(h2 ? 0 : szV * 4);
  H->ranks.cached(2 * np_total * sizeof(int32_t));
  // H^2 applies through its passes.  The matrix keeps the applies' plans;
  // the peel's (whole boxes, every prefix of levels) live with the compression.
  if (!h2) {
    build_plans(*H, T, kSeg, false, H->oA, H->oT, s);
    build_plans(*H, T, 0, true, peel_plans[0], peel_plans[1], s);
  }

  // leaf neighbor blocks
  const Graph &GL = T.leaf_graph();
  const Level &LL = T.lev[T.L()];
  {
    // the near kernel takes at most kNearCols columns per entry: wider
    // neighbor boxes are split into column pieces
    constexpr int32_t kNearCols = 128;
    std::vector<ExpandChunk> ch;
    std::vector<NearEntry> en;
    std::vector<size_t> eq;  // pair of each entry
    H->na = GL.pa;
    H->nb = GL.pb;
    for (size_t q = 0; q < GL.pa.size(); ++q) {
      H->offD.push_back(szD);
      szD += T.box_size(T.L(), GL.pa[q]) * T.box_size(T.L(), GL.pb[q]);
    }
    size_t i = 0;
    while (i < GL.pa.size()) {
      size_t j = i;
      while (j < GL.pa.size() && GL.pa[j] == GL.pa[i]) ++j;
      const int a = GL.pa[i];
      const int32_t m = (int32_t)T.box_size(T.L(), a);
      for (int32_t off = 0; off < m; off += 64) {
        ExpandChunk c{LL.start[a] + off, std::min<int32_t>(64, m - off), (int32_t)en.size(), 0, 0};
        for (size_t q = i; q < j; ++q) {
          const int32_t mb = (int32_t)T.box_size(T.L(), GL.pb[q]);
          for (int32_t k0 = 0; k0 < mb; k0 += kNearCols) {
            en.push_back(NearEntry{H->offD[q] + (int64_t)k0 * m, LL.start[GL.pb[q]] + k0, m,
                                   std::min(kNearCols, mb - k0), off, 0});
            eq.push_back(q);
          }
        }
        c.last = (int32_t)en.size();
        ch.push_back(c);
      }
      i = j;
    }
    upload_cached(H->nchunks, ch, s);
    upload_cached(H->nentries, en, s);
    H->nnch = (int32_t)ch.size();
    // the adjoint's near field: block (a, b) of H* is D_(b,a)^T (neighbor
    // pairs come in both orders)
    std::unordered_map<int64_t, size_t> qidx;
    qidx.reserve(GL.pa.size() * 2);
    for (size_t q = 0; q < GL.pa.size(); ++q) qidx[(int64_t)GL.pa[q] * LL.nbox() + GL.pb[q]] = q;
    std::vector<NearEntry> enT;
    for (ExpandChunk &c : ch) {
      const int32_t first = (int32_t)enT.size();
      for (int32_t e = c.first; e < c.last; ++e) {
        const size_t q = eq[e];  // the entry's pair (a, b)
        const int a = GL.pa[q], b = GL.pb[q];
        const auto it = qidx.find((int64_t)b * LL.nbox() + a);
        if (it == qidx.end()) throw Error{HM_E_STATE, "neighbor pairs are not symmetric"};
        const int32_t mb = (int32_t)T.box_size(T.L(), b);
        const int32_t k0 = (int32_t)(en[e].xrow0 - LL.start[b]);  // column piece of b
        enT.push_back(NearEntry{H->offD[it->second] + k0, LL.start[b] + k0, mb, en[e].mb,
                                en[e].off, 1});
      }
      c.first = first;
      c.last = (int32_t)enT.size();
    }
    upload_cached(H->nchunksT, ch, s);
    upload_cached(H->nentriesT, enT, s);
    // every row has a near block (a box is its own neighbor): the near
    // field can open an apply by writing Y
    int64_t covered = 0;
    for (const ExpandChunk &c : ch) covered += c.nrows;
    H->near_covers = covered == T.n;
    H->D.cached(szD * 8);
    HIP_TRY(hipStreamSynchronize(s));
  }

  // ---------------- working buffers
  for (int l : levels) cmax = std::max<int64_t>(cmax, pad16((int64_t)T.graphs[l].ncolors * r));
  mw = T.leaf_width();
  leaf_cols = pad16((int64_t)GL.ncolors * mw);
  wcols = std::max<int64_t>(2 * cmax, leaf_cols);
  size_t wbytes = (size_t)n * wcols * es, tes = es;
  if (uniform) {
    // the two stages run one after the other through the same buffers;
    // stage 2 always runs in FP64 (its samples are summed, see
    // record_uniform_level)
    wcols = leaf_cols;
    int64_t w2 = 0;
    for (int l : levels) {
      wcols = std::max(wcols, pad16((int64_t)T.ugraphs[l].ncolors * r));
      w2 = std::max(w2, pad16((int64_t)T.graphs[l].ncolors * kmax));
    }
    wbytes = std::max((size_t)n * wcols * es, (size_t)n * w2 * 8);
    wcols = std::max(wcols, w2);
    tes = 8;
  }
  buf(Xb, wbytes, s);
  buf(Yb, wbytes, s);
  {
    // partial projections of the peel: one slot per pair (whole boxes)
    const int64_t slots = std::max<int64_t>(
        peel_plans[0].slots_upto.empty() ? 0 : peel_plans[0].slots_upto.back(),
        peel_plans[1].slots_upto.empty() ? 0 : peel_plans[1].slots_upto.back());
    const int64_t need = slots * kmax * std::max<int64_t>(wcols, 1);
    tcap = std::max<int64_t>(std::min(need, kTScratchCap), std::max<int64_t>(slots * kmax * 64, 64));
  }
  buf(Tb, (size_t)tcap * tes, s);
  {
    // one flag per slot and 64-column tile: a chunk of w columns uses
    // slots * ceil(w / 64) <= tcap / (kmax 64) + slots
    const int64_t slots = std::max<int64_t>(
        peel_plans[0].slots_upto.empty() ? 0 : peel_plans[0].slots_upto.back(),
        peel_plans[1].slots_upto.empty() ? 0 : peel_plans[1].slots_upto.back());
    tflag_cap = tcap / ((int64_t)std::max(kmax, 1) * kLowRankTile) + slots + 64;
    buf(tflags, (size_t)tflag_cap, s);
  }
  int64_t wmax = 0;
  for (size_t li = 0; li < H->lv.size(); ++li) {
    const hm_hmatrix::Lv &L = H->lv[li];
    const Level &Lv = T.lev[L.level];
    int64_t rows = 0;
    for (int64_t q = 0; q < L.np; ++q)
      rows += (Lv.start[L.pa[q] + 1] - Lv.start[L.pa[q]]) + (Lv.start[L.pb[q] + 1] - Lv.start[L.pb[q]]);
    wmax = std::max(wmax, rows * r);
    cmax_np = std::max(cmax_np, L.np);
  }
  buf(work, (size_t)std::max<int64_t>(wmax, 1) * 8, s);
  buf(core, (size_t)std::max<int64_t>(cmax_np, 1) * r * r * 8, s);
  buf(scratch, (size_t)std::max<int64_t>(cmax_np, 1) * r * r * 8, s);
  buf(sat, (size_t)std::max<int64_t>(2 * np_total, 1) * 4, s);
  buf(flag, 64, s);
  // mixed path: per-block noise floors of the FP32 samples (see record)
  if (mixed) {
    buf(floor_u, (size_t)std::max<int64_t>(cmax_np, 1) * 8, s);
    buf(floor_v, (size_t)std::max<int64_t>(cmax_np, 1) * 8, s);
  }
  // a black box in the original point order works through two permuted
  // copies of the samples
  if (bb.order != HM_ORDER_TREE) {
    buf(tmpx, wbytes, s);
    buf(tmpy, wbytes, s);
  }

  // ---------------- forest: the library's own kernel black box on this
  // forest is called directly with the per-instance live widths: colors an
  // instance does not use are zero columns in its rows, and their tiles are
  // skipped
  ni = T.ninst();
  kbb = bb.apply == kernel_bb_apply ? (KernelBB *)bb.ctx : nullptr;
  direct = kbb && kbb->tree == &T && ni > 1;

  // ---------------- every job list of every level, uploaded once up front
  if (h2) {
    // the SVD workspace holds every basis box of a level (at most n rows) x r
    if ((int64_t)work.bytes < n * r * 8) buf(work, (size_t)n * r * 8, s);
    setup_h2(s);
  } else if (uniform) {
    setup_uniform(s);
  }
  jobs_of.resize(H->lv.size());
  if (!uniform) {
    h_act.assign(H->lv.size(), {});
    h_act_nc.assign(H->lv.size(), 0);
  }
  for (size_t li = 0; !uniform && li < H->lv.size(); ++li) {
    hm_hmatrix::Lv &L = H->lv[li];
    const Graph &G = T.graphs[L.level];
    const Level &Lv = T.lev[L.level];
    const int64_t cpad = pad16((int64_t)G.ncolors * r);
    std::vector<uint8_t> act((size_t)Lv.nbox() * G.ncolors, 0);
    for (int64_t v = 0; v < G.nv(); ++v) act[(size_t)G.vbox[v] * G.ncolors + G.color[v]] = 1;
    h_act[li] = act;
    h_act_nc[li] = G.ncolors;
    std::unordered_map<int64_t, int64_t> pidx;
    pidx.reserve(L.np * 2);
    for (int64_t q = 0; q < L.np; ++q) pidx[(int64_t)L.pa[q] * Lv.nbox() + L.pb[q]] = q;
    std::vector<QrJob> ju(L.np), jv(L.np);
    std::vector<CoreJob> jc(L.np);
    int64_t wofs = 0;
    for (int64_t q = 0; q < L.np; ++q) {
      const int a = L.pa[q], b = L.pb[q];
      const int64_t cu = G.color[G.pv[q]];
      const int64_t cv = G.color[G.pv[pidx.at((int64_t)b * Lv.nbox() + a)]];
      const int32_t ma = (int32_t)(Lv.start[a + 1] - Lv.start[a]);
      const int32_t mb = (int32_t)(Lv.start[b + 1] - Lv.start[b]);
      ju[q] = QrJob{Lv.start[a], cu * r, L.offU[q], wofs, ma, 0};
      wofs += (int64_t)ma * r;
      jv[q] = QrJob{Lv.start[b], cpad + cv * r, L.offV[q], wofs, mb, 0};
      wofs += (int64_t)mb * r;
      jc[q] = CoreJob{Lv.start[a], Lv.start[b], cu * r, cpad + cv * r, L.offU[q], L.offV[q],
                      L.offW[q], L.offB[q], q * r * r, ma, mb,
                      (int32_t)(L.g0 + q), (int32_t)(np_total + L.g0 + q)};
    }
    if (direct) {
      std::vector<int32_t> w = inst_colors(L.level);
      for (int32_t &x : w) x *= r;
      std::vector<KItem> kit = forest_items(T, w);
      put(jobs_of[li].kit, kit, s);
      jobs_of[li].nkit = (int32_t)kit.size();
    }
    // the fused recovery takes the largest blocks first, so that the
    // workgroups finish together
    std::vector<int32_t> order(L.np);
    for (int64_t q = 0; q < L.np; ++q) order[q] = (int32_t)q;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
      return ju[x].m + jv[x].m > ju[y].m + jv[y].m;
    });
    put(jobs_of[li].act, act, s);
    put(jobs_of[li].ju, ju, s);
    put(jobs_of[li].jv, jv, s);
    put(jobs_of[li].jc, jc, s);
    put(jobs_of[li].order, order, s);
    HIP_TRY(hipStreamSynchronize(s));  // the host vectors die here
  }
  if (!uniform) {
    buf(counters, (size_t)std::max<size_t>(H->lv.size(), 1) * 4, s);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, H->device) ==
            hipSuccess &&
        cus > 0)
      recover_grid = 16 * cus;  // as many as fit resident; the rest find the list empty
    (void)hipGetLastError();
  }

  // ---------------- leaf pass lists
  {
    std::vector<int32_t> ib, ic;
    for (int64_t v = 0; v < GL.nv(); ++v) {
      ib.push_back(GL.vbox[v]);
      ic.push_back(GL.color[v]);
    }
    // one item per (box, color) is enough; duplicates write the same ones
    put(dib, ib, s);
    put(dic, ic, s);
    nib = (int32_t)ib.size();
    // the identity blocks' zero pattern: leaf box b is active in color c
    std::vector<uint8_t> la((size_t)std::max<int64_t>((int64_t)LL.nbox() * GL.ncolors, 1), 0);
    for (int64_t v = 0; v < GL.nv(); ++v) la[(size_t)GL.vbox[v] * GL.ncolors + GL.color[v]] = 1;
    put(leaf_act, la, s);
    h_leaf_act = la;
    std::vector<KItem> kit;
    if (direct) {
      std::vector<int32_t> w = inst_colors(T.nlev());
      for (int32_t &x : w) x *= mw;
      kit = forest_items(T, w);
      put(dkit, kit, s);
    }
    nkit_leaf = (int32_t)kit.size();
    std::vector<int64_t> r0(GL.pa.size()), c0(GL.pa.size());
    std::vector<int32_t> ma(GL.pa.size()), mb(GL.pa.size());
    for (size_t q = 0; q < GL.pa.size(); ++q) {
      r0[q] = LL.start[GL.pa[q]];
      ma[q] = (int32_t)T.box_size(T.L(), GL.pa[q]);
      mb[q] = (int32_t)T.box_size(T.L(), GL.pb[q]);
      c0[q] = (int64_t)GL.color[GL.pv[q]] * mw;
    }
    put(dr0, r0, s);
    put(dc0, c0, s);
    put(dma, ma, s);
    put(dmb, mb, s);
    put(doff, H->offD, s);
    HIP_TRY(hipStreamSynchronize(s));
  }
  return HM_OK;
}

// Bases, job lists and buffers of the uniform format (one vertex per box
// with a non-empty interaction list; the same boxes are the row and the
// column boxes of the level's pairs).
void Compression::setup_uniform(hipStream_t s) {
  H->format = HM_FORMAT_UNIFORM_H1;
  const size_t nlv = H->lv.size();
  int64_t szb = 0;
  H->ubox.resize(nlv);
  H->uoff.resize(nlv);
  H->uv0.resize(nlv);
  for (size_t li = 0; li < nlv; ++li) {
    const int l = H->lv[li].level;
    const Graph &UG = T.ugraphs[l];
    H->uv0[li] = H->nvtot;
    H->ubox[li] = UG.vbox;
    for (int64_t v = 0; v < UG.nv(); ++v) {
      H->uoff[li].push_back(szb);
      szb += T.box_size(l, UG.vbox[v]) * kmax;
    }
    H->nvtot += UG.nv();
  }
  H->UB.cached((size_t)std::max<int64_t>(szb, 1) * 8);
  H->VB.cached((size_t)std::max<int64_t>(szb, 1) * 8);
  H->brank.cached((size_t)std::max<int64_t>(2 * H->nvtot, 1) * 4);
  buf(Sb, (size_t)n * kmax * 8, s);
  buf(usat, (size_t)std::max<int64_t>(2 * H->nvtot, 1) * 4, s);

  ujobs_of.resize(nlv);
  h_act.assign(nlv, {});
  h_act_nc.assign(nlv, 0);
  for (size_t li = 0; li < nlv; ++li) {
    const hm_hmatrix::Lv &L = H->lv[li];
    const int l = L.level;
    const Graph &G = T.graphs[l], &UG = T.ugraphs[l];
    const Level &Lv = T.lev[l];
    const int nb = Lv.nbox();
    UniformJobs &J = ujobs_of[li];
    J.nv = (int32_t)UG.nv();
    std::vector<int32_t> vid(nb, -1);
    for (int64_t v = 0; v < UG.nv(); ++v) vid[UG.vbox[v]] = (int32_t)v;
    // stage 1: active flags and QR jobs
    std::vector<uint8_t> act((size_t)nb * std::max(UG.ncolors, 1), 0);
    std::vector<QrJob> ju(UG.nv()), jv(UG.nv());
    int64_t wofs = 0;
    for (int64_t v = 0; v < UG.nv(); ++v) {
      const int a = UG.vbox[v], c = UG.color[v];
      for (int32_t t = Lv.int_ptr[a]; t < Lv.int_ptr[a + 1]; ++t)
        act[(size_t)Lv.intl[t] * UG.ncolors + c] = 1;
      const int32_t m = (int32_t)T.box_size(l, a);
      ju[v] = QrJob{Lv.start[a], (int64_t)c * r, H->uoff[li][v], wofs, m, 0};
      jv[v] = QrJob{Lv.start[a], 0, H->uoff[li][v], wofs, m, 0};
      wofs += (int64_t)m * r;
    }
    // stage 2: the pair graph's (box, color) slots hold the box's basis
    std::vector<int32_t> slot((size_t)nb * std::max(G.ncolors, 1), 0);
    for (int64_t v = 0; v < G.nv(); ++v) {
      const int a = G.vbox[v];
      if (vid[a] < 0) throw Error{HM_E_STATE, "pair-graph box without a uniform basis"};
      slot[(size_t)a * G.ncolors + G.color[v]] = vid[a] + 1;
    }
    std::unordered_map<int64_t, int64_t> pidx;
    pidx.reserve(L.np * 2);
    for (int64_t q = 0; q < L.np; ++q) pidx[(int64_t)L.pa[q] * nb + L.pb[q]] = q;
    auto color_of = [&](int a, int b) {  // color of the pair (a, b)'s vertex
      return (int64_t)G.color[G.pv[pidx.at((int64_t)a * nb + b)]];
    };
    // combination jobs: 256-row chunks of every vertex box b, terms over a in int(b)
    std::vector<MixJob> mix;
    std::vector<MixTerm> terms;
    for (int64_t v = 0; v < UG.nv(); ++v) {
      const int b = UG.vbox[v];
      const int32_t t0 = (int32_t)terms.size();
      for (int32_t t = Lv.int_ptr[b]; t < Lv.int_ptr[b + 1]; ++t) {
        const int a = Lv.intl[t];
        const int inst = inst_of_row(Lv.start[a]);
        const int64_t base = ni > 1 ? T.inst_off[inst] : 0;
        terms.push_back(MixTerm{color_of(b, a) * kmax, (uint32_t)(Lv.start[a] - base),
                                (uint32_t)inst});
      }
      const int32_t t1 = (int32_t)terms.size();
      const int64_t m = T.box_size(l, b);
      for (int64_t r0 = 0; r0 < m; r0 += 256)
        mix.push_back(MixJob{Lv.start[b] + r0, (int32_t)std::min<int64_t>(256, m - r0), t0, t1, 0});
    }
    // per-pair coupling jobs
    std::vector<UCJob> uc(L.np);
    for (int64_t q = 0; q < L.np; ++q) {
      const int a = L.pa[q], b = L.pb[q];
      uc[q] = UCJob{Lv.start[b], color_of(b, a) * kmax, H->uoff[li][vid[a]], H->uoff[li][vid[b]],
                    L.offU[q], L.offV[q], L.offW[q], L.offB[q],
                    (int32_t)T.box_size(l, a), (int32_t)T.box_size(l, b), vid[a], vid[b],
                    (int32_t)(L.g0 + q), (int32_t)(np_total + L.g0 + q)};
    }
    if (direct) {
      std::vector<int32_t> wu(ni, 0);
      for (int64_t v = 0; v < UG.nv(); ++v) {
        const int i = inst_of_row(Lv.start[UG.vbox[v]]);
        wu[i] = std::max(wu[i], UG.color[v] + 1);
      }
      for (int32_t &x : wu) x *= r;
      std::vector<KItem> k1 = forest_items(T, wu);
      std::vector<int32_t> w2 = inst_colors(l);
      for (int32_t &x : w2) x *= kmax;
      std::vector<KItem> k2 = forest_items(T, w2);
      put(J.kit1, k1, s);
      put(J.kit2, k2, s);
      J.nkit1 = (int32_t)k1.size();
      J.nkit2 = (int32_t)k2.size();
    }
    J.nmix = (int32_t)mix.size();
    h_act[li] = act;
    h_act_nc[li] = UG.ncolors;
    put(J.act, act, s);
    put(J.ju, ju, s);
    put(J.jv, jv, s);
    put(J.slot, slot, s);
    put(J.uoff, H->uoff[li], s);
    put(J.mix, mix, s);
    put(J.terms, terms, s);
    put(J.uc, uc, s);
    HIP_TRY(hipStreamSynchronize(s));  // the host vectors die here
  }
}

// H^2: bases on every level of the sampled range for each box whose far
// field is not empty (an interaction list, or a parent with a basis); the
// parent's long basis augments the samples, transfer matrices nest each
// level into the next, and after every level the bases of all coarser
// levels are rebuilt from the finest ones through the transfers, with
// their pairs' apply factors, so the per-pair apply of the level-truncated
// matrix is the nested (H^2) one.
void Compression::setup_h2(hipStream_t s) {
  H->format = HM_FORMAT_H2;
  const size_t nlv = H->lv.size();
  for (size_t li = 1; li < nlv; ++li)
    if (H->lv[li].level != H->lv[li - 1].level + 1)
      throw Error{HM_E_ARG, "H2 format: a level between the first and the last sampled level "
                            "has no admissible pair"};
  // each instance's last sampled level: its boxes inherit bases only up to
  // it (a forest carries a shallow instance's leaves further down, and the
  // instance compressed alone has no bases there)
  std::vector<int> inst_last(ni, -1);
  for (size_t li = 0; li < nlv; ++li) {
    const hm_hmatrix::Lv &L = H->lv[li];
    for (int64_t q = 0; q < L.np; ++q) {
      const int i = inst_of_row(T.lev[L.level].start[L.pa[q]]);
      inst_last[i] = std::max(inst_last[i], L.level);
    }
  }
  int64_t szb = 0;
  H->ubox.resize(nlv);
  H->uoff.resize(nlv);
  H->uv0.resize(nlv);
  std::vector<std::vector<int32_t>> vid(nlv);
  for (size_t li = 0; li < nlv; ++li) {
    const int l = H->lv[li].level;
    const Level &Lv = T.lev[l];
    vid[li].assign(Lv.nbox(), -1);
    H->uv0[li] = H->nvtot;
    for (int a = 0; a < Lv.nbox(); ++a) {
      const bool inherit = li > 0 && vid[li - 1][Lv.parent[a]] >= 0 &&
                           l <= inst_last[inst_of_row(Lv.start[a])];
      if (Lv.int_ptr[a + 1] > Lv.int_ptr[a] || inherit) {
        vid[li][a] = (int32_t)H->ubox[li].size();
        H->ubox[li].push_back(a);
        H->uoff[li].push_back(szb);
        szb += T.box_size(l, a) * kmax;
      }
    }
    H->nvtot += (int64_t)H->ubox[li].size();
  }
  const int64_t nb = H->nvtot;
  H->UB.cached((size_t)std::max<int64_t>(szb, 1) * 8);
  H->VB.cached((size_t)std::max<int64_t>(szb, 1) * 8);
  H->brank.cached((size_t)std::max<int64_t>(2 * nb, 1) * 4);
  H->SU.cached((size_t)std::max<int64_t>(nb * kmax, 1) * 8);
  H->SV.cached((size_t)std::max<int64_t>(nb * kmax, 1) * 8);
  H->TU.cached((size_t)std::max<int64_t>(nb * kmax * kmax, 1) * 8);
  H->TV.cached((size_t)std::max<int64_t>(nb * kmax * kmax, 1) * 8);
  // expansion scratch of the peel's level-truncated products, at most 64 MB each
  h2cols = std::min<int64_t>(256, std::max<int64_t>(16, (int64_t(64) << 20) /
                                                            std::max<int64_t>(nb * kmax * 8, 1)));
  buf(h2q, (size_t)std::max<int64_t>(nb * kmax * h2cols, 1) * 8, s);
  buf(h2u, (size_t)std::max<int64_t>(nb * kmax * h2cols, 1) * 8, s);
  buf(Sb, (size_t)n * r * 8, s);
  buf(usat, (size_t)std::max<int64_t>(2 * nb, 1) * 4, s);
  if (mixed) {
    const size_t nbl = [&] {
      size_t x = 1;
      for (const auto &u : H->ubox) x = std::max(x, u.size());
      return x;
    }();
    buf(floor_u, nbl * 8, s);
  }

  ujobs_of.resize(nlv);
  h_act.assign(nlv, {});
  h_act_nc.assign(nlv, 0);
  for (size_t li = 0; li < nlv; ++li) {
    hm_hmatrix::Lv &L = H->lv[li];  // offU, offV point into the box bases (no pair copies)
    const int l = L.level;
    const Graph &G = T.graphs[l], &UG = T.ugraphs[l];
    const Level &Lv = T.lev[l];
    const int nbx = Lv.nbox();
    UniformJobs &J = ujobs_of[li];
    const std::vector<int32_t> &hb = H->ubox[li];
    J.nv = (int32_t)hb.size();
    const int64_t v0 = H->uv0[li];
    std::vector<int32_t> ucol(nbx, -1);  // stage-1 color of a vertex box
    for (int64_t v = 0; v < UG.nv(); ++v) ucol[UG.vbox[v]] = UG.color[v];
    std::vector<uint8_t> act((size_t)nbx * std::max(UG.ncolors, 1), 0);
    for (int64_t v = 0; v < UG.nv(); ++v)
      for (int32_t t = Lv.int_ptr[UG.vbox[v]]; t < Lv.int_ptr[UG.vbox[v] + 1]; ++t)
        act[(size_t)Lv.intl[t] * UG.ncolors + UG.color[v]] = 1;
    std::vector<QrJob> jn(hb.size()), jsu(hb.size()), jsv(hb.size());
    std::vector<AugJob> au, av;
    int64_t wofs = 0;
    for (size_t v = 0; v < hb.size(); ++v) {
      const int a = hb[v];
      const int32_t m = (int32_t)T.box_size(l, a);
      const bool vert = ucol[a] >= 0;
      jn[v] = QrJob{Lv.start[a], vert ? (int64_t)ucol[a] * r : 0, 0, 0, vert ? m : 0, 0};
      jsu[v] = QrJob{Lv.start[a], 0, H->uoff[li][v], wofs, m, 0};
      jsv[v] = jsu[v];
      wofs += (int64_t)m * r;
      const int inst = inst_of_row(Lv.start[a]);
      const int64_t base = ni > 1 ? T.inst_off[inst] : 0;
      int32_t pi = -1;
      int64_t poff = -1, pstart = 0;
      int32_t pld = 0;
      if (li > 0) {
        const int tau = Lv.parent[a];
        const int32_t tv = vid[li - 1][tau];
        if (tv >= 0) {
          pi = (int32_t)(H->uv0[li - 1] + tv);
          pstart = T.lev[l - 1].start[tau];
          poff = H->uoff[li - 1][tv] + (Lv.start[a] - pstart);
          pld = (int32_t)T.box_size(l - 1, tau);
        }
      }
      for (int64_t c0 = 0; c0 < m; c0 += 256) {
        const int32_t cm = (int32_t)std::min<int64_t>(256, m - c0);
        au.push_back(AugJob{Lv.start[a] + c0, vert ? (int64_t)ucol[a] * r : -1,
                            poff >= 0 ? poff + c0 : -1, cm, pld, pi,
                            (uint32_t)(Lv.start[a] - base), (uint32_t)inst, 0});
        av.push_back(AugJob{Lv.start[a] + c0, vert ? 0 : -1, poff >= 0 ? poff + c0 : -1, cm, pld,
                            pi, (uint32_t)(Lv.start[a] - base), (uint32_t)inst, 0});
      }
    }
    std::vector<int32_t> slot((size_t)nbx * std::max(G.ncolors, 1), 0);
    for (int64_t v = 0; v < G.nv(); ++v) {
      const int a = G.vbox[v];
      if (vid[li][a] < 0) throw Error{HM_E_STATE, "pair-graph box without a basis"};
      slot[(size_t)a * G.ncolors + G.color[v]] = vid[li][a] + 1;
    }
    std::unordered_map<int64_t, int64_t> pidx;
    pidx.reserve(L.np * 2);
    for (int64_t q = 0; q < L.np; ++q) pidx[(int64_t)L.pa[q] * nbx + L.pb[q]] = q;
    auto color_of = [&](int a, int b) {
      return (int64_t)G.color[G.pv[pidx.at((int64_t)a * nbx + b)]];
    };
    std::vector<MixJob> mix;
    std::vector<MixTerm> terms;
    for (int b : hb) {
      if (Lv.int_ptr[b + 1] == Lv.int_ptr[b]) continue;
      const int32_t t0 = (int32_t)terms.size();
      for (int32_t t = Lv.int_ptr[b]; t < Lv.int_ptr[b + 1]; ++t) {
        const int a = Lv.intl[t];
        const int inst = inst_of_row(Lv.start[a]);
        const int64_t base = ni > 1 ? T.inst_off[inst] : 0;
        terms.push_back(MixTerm{color_of(b, a) * kmax, (uint32_t)(Lv.start[a] - base),
                                (uint32_t)inst});
      }
      const int32_t t1 = (int32_t)terms.size();
      const int64_t m = T.box_size(l, b);
      for (int64_t r0 = 0; r0 < m; r0 += 256)
        mix.push_back(MixJob{Lv.start[b] + r0, (int32_t)std::min<int64_t>(256, m - r0), t0, t1, 0});
    }
    std::vector<UCJob> uc(L.np);
    for (int64_t q = 0; q < L.np; ++q) {
      const int a = L.pa[q], b = L.pb[q];
      uc[q] = UCJob{Lv.start[b], color_of(b, a) * kmax, H->uoff[li][vid[li][a]],
                    H->uoff[li][vid[li][b]], L.offU[q], L.offV[q], L.offW[q], L.offB[q],
                    (int32_t)T.box_size(l, a), (int32_t)T.box_size(l, b), vid[li][a], vid[li][b],
                    (int32_t)(L.g0 + q), (int32_t)(np_total + L.g0 + q)};
      // no pair copies: a pair's bases are read where the boxes keep them
      L.offU[q] = H->uoff[li][vid[li][a]];
      L.offV[q] = H->uoff[li][vid[li][b]];
    }
    // transfers and nesting of the previous level into this one
    std::vector<TransferJob> tr;
    std::vector<NestJob> ne;
    if (li > 0) {
      for (size_t v = 0; v < hb.size(); ++v) {
        const int a = hb[v];
        const int tau = Lv.parent[a];
        const int32_t tv = vid[li - 1][tau];
        if (tv < 0) continue;
        const int64_t ga = v0 + (int64_t)v, gt = H->uv0[li - 1] + tv;
        const int64_t rowin = Lv.start[a] - T.lev[l - 1].start[tau];
        const int32_t ma = (int32_t)T.box_size(l, a), mt = (int32_t)T.box_size(l - 1, tau);
        tr.push_back(TransferJob{H->uoff[li][v], H->uoff[li - 1][tv] + rowin,
                                 ga * kmax * kmax, ma, mt, (int32_t)ga, (int32_t)gt});
        for (int64_t c0 = 0; c0 < ma; c0 += 256)
          ne.push_back(NestJob{H->uoff[li - 1][tv] + rowin + c0, H->uoff[li][v] + c0,
                               ga * kmax * kmax, (int32_t)std::min<int64_t>(256, ma - c0), mt,
                               ma, (int32_t)ga, (int32_t)gt, 0});
      }
    }
    if (direct) {
      std::vector<int32_t> wu(ni, 0);
      for (int64_t v = 0; v < UG.nv(); ++v) {
        const int i = inst_of_row(Lv.start[UG.vbox[v]]);
        wu[i] = std::max(wu[i], UG.color[v] + 1);
      }
      for (int32_t &x : wu) x *= r;
      std::vector<KItem> k1 = forest_items(T, wu);
      std::vector<int32_t> w2 = inst_colors(l);
      for (int32_t &x : w2) x *= kmax;
      std::vector<KItem> k2 = forest_items(T, w2);
      put(J.kit1, k1, s);
      put(J.kit2, k2, s);
      J.nkit1 = (int32_t)k1.size();
      J.nkit2 = (int32_t)k2.size();
    }
    J.nmix = (int32_t)mix.size();
    J.naug = (int32_t)au.size();
    J.ntr = (int32_t)tr.size();
    J.nnest = (int32_t)ne.size();
    put(J.act, act, s);
    put(J.ju, jsu, s);
    put(J.jv, jsv, s);
    put(J.jn, jn, s);
    put(J.augu, au, s);
    put(J.augv, av, s);
    put(J.slot, slot, s);
    put(J.uoff, H->uoff[li], s);
    put(J.mix, mix, s);
    put(J.terms, terms, s);
    put(J.uc, uc, s);
    put(J.tr, tr, s);
    put(J.nest, ne, s);
    HIP_TRY(hipStreamSynchronize(s));
  }
  build_h2_apply(vid, s);
  // chunk partials of the outgoing expansions, for the largest chunk list
  int64_t maxc = H->h2a.nchunk;
  for (int32_t c : H->h2a.ntchunk) maxc = std::max<int64_t>(maxc, c);
  buf(h2p, (size_t)std::max<int64_t>(maxc * kmax * h2cols, 1) * 8, s);
}

// The H^2 apply plan (alg:apply_h2_level_truncated) from the basis boxes.
void Compression::build_h2_apply(const std::vector<std::vector<int32_t>> &vid, hipStream_t s) {
  hm_hmatrix::H2Apply &P = H->h2a;
  const size_t nlv = H->lv.size();
  const int64_t km2 = (int64_t)kmax * kmax;
  std::vector<H2Leaf> leaf, chunk;
  // per level: every basis box as a leaf record, and whether it has children with bases
  std::vector<std::vector<H2Leaf>> all_of(nlv);
  std::vector<std::vector<uint8_t>> haskids(nlv);
  P.up_j.resize(nlv);
  P.up_t.resize(nlv);
  P.dn_j.resize(nlv);
  P.dn_t.resize(nlv);
  P.dnt_j.resize(nlv);
  P.dnt_t.resize(nlv);
  P.nup.assign(nlv, 0);
  P.ndn.assign(nlv, 0);
  for (size_t li = 0; li < nlv; ++li) {
    const hm_hmatrix::Lv &L = H->lv[li];
    const int l = L.level;
    const Level &Lv = T.lev[l];
    const std::vector<int32_t> &hb = H->ubox[li];
    const int64_t v0 = H->uv0[li];
    // children with bases of each basis box
    std::vector<std::vector<int32_t>> kids(hb.size());
    if (li + 1 < nlv) {
      const Level &Ln = T.lev[H->lv[li + 1].level];
      for (size_t c = 0; c < H->ubox[li + 1].size(); ++c) {
        const int a = H->ubox[li + 1][c];
        const int32_t pv = vid[li][Ln.parent[a]];
        if (pv >= 0) kids[pv].push_back((int32_t)(H->uv0[li + 1] + c));
      }
    }
    std::unordered_map<int64_t, int64_t> pidx;
    pidx.reserve(L.np * 2);
    for (int64_t q = 0; q < L.np; ++q) pidx[(int64_t)L.pa[q] * Lv.nbox() + L.pb[q]] = q;
    std::vector<H2Sum> uj, dj, dtj;
    std::vector<H2Term> ut, dt, dtt;
    haskids[li].assign(hb.size(), 0);
    for (size_t v = 0; v < hb.size(); ++v) {
      const int a = hb[v];
      const int32_t g = (int32_t)(v0 + v);
      all_of[li].push_back(H2Leaf{Lv.start[a], H->uoff[li][v], (int32_t)T.box_size(l, a), g, 0, 0});
      if (kids[v].empty()) {
        const int32_t m = (int32_t)T.box_size(l, a);
        leaf.push_back(H2Leaf{Lv.start[a], H->uoff[li][v], m, g, 0, (int32_t)chunk.size()});
        for (int32_t r0 = 0; r0 < m; r0 += 64)
          chunk.push_back(H2Leaf{Lv.start[a], H->uoff[li][v], m, g, r0, 0});
      } else {
        haskids[li][v] = 1;
        const int32_t t0 = (int32_t)ut.size();
        for (int32_t c : kids[v]) ut.push_back(H2Term{c * km2, c, 0, 1});
        uj.push_back(H2Sum{g, t0, (int32_t)ut.size(), 0});
      }
      // downward: couplings of the level, then the parent's incoming expansion
      const int32_t d0 = (int32_t)dt.size(), e0 = (int32_t)dtt.size();
      for (int32_t t = Lv.int_ptr[a]; t < Lv.int_ptr[a + 1]; ++t) {
        const int b = Lv.intl[t];
        const int32_t gb = (int32_t)(v0 + vid[li][b]);
        dt.push_back(H2Term{L.offB[pidx.at((int64_t)a * Lv.nbox() + b)], gb, 0, 0});
        dtt.push_back(H2Term{L.offB[pidx.at((int64_t)b * Lv.nbox() + a)], gb, 0, 1});
      }
      if (li > 0) {
        const int32_t pv = vid[li - 1][Lv.parent[a]];
        if (pv >= 0) {
          const int32_t gp = (int32_t)(H->uv0[li - 1] + pv);
          dt.push_back(H2Term{(int64_t)g * km2, gp, 1, 0});
          dtt.push_back(H2Term{(int64_t)g * km2, gp, 1, 0});
        }
      }
      dj.push_back(H2Sum{g, d0, (int32_t)dt.size(), 0});
      dtj.push_back(H2Sum{g, e0, (int32_t)dtt.size(), 0});
    }
    upload_cached(P.up_j[li], uj, s);
    upload_cached(P.up_t[li], ut, s);
    upload_cached(P.dn_j[li], dj, s);
    upload_cached(P.dn_t[li], dt, s);
    upload_cached(P.dnt_j[li], dtj, s);
    upload_cached(P.dnt_t[li], dtt, s);
    P.nup[li] = (int32_t)uj.size();
    P.ndn[li] = (int32_t)dj.size();
    HIP_TRY(hipStreamSynchronize(s));
  }
  upload_cached(P.leaf, leaf, s);
  upload_cached(P.chunk, chunk, s);
  P.nleaf = (int32_t)leaf.size();
  P.nchunk = (int32_t)chunk.size();
  // the level-truncated operators of the peel (first li levels, li < nlv)
  P.tleaf.resize(nlv);
  P.tchunk.resize(nlv);
  P.ntleaf.assign(nlv, 0);
  P.ntchunk.assign(nlv, 0);
  for (size_t le = 1; le < nlv; ++le) {
    std::vector<H2Leaf> tl, tc;
    for (size_t li = 0; li < le; ++li)
      for (size_t v = 0; v < all_of[li].size(); ++v) {
        if (li + 1 < le && haskids[li][v]) continue;
        H2Leaf b = all_of[li][v];
        b.c0 = (int32_t)tc.size();
        tl.push_back(b);
        for (int32_t r0 = 0; r0 < b.m; r0 += 64)
          tc.push_back(H2Leaf{b.row0, b.boff, b.m, b.g, r0, 0});
      }
    upload_cached(P.tleaf[le], tl, s);
    upload_cached(P.tchunk[le], tc, s);
    P.ntleaf[le] = (int32_t)tl.size();
    P.ntchunk[le] = (int32_t)tc.size();
  }
  HIP_TRY(hipStreamSynchronize(s));
  P.ready = true;
}

void Compression::record_h2_level(size_t li, hipStream_t s, Events &ev) {
  const DeviceTree &Dv = *D;
  hm_hmatrix::Lv &L = H->lv[li];
  const int l = L.level;
  const Graph &G = T.graphs[l], &UG = T.ugraphs[l];
  UniformJobs &J = ujobs_of[li];
  const int64_t v0 = H->uv0[li], nb = H->nvtot;
  int32_t *rk = H->brank.as<int32_t>();
  const int64_t c1 = (int64_t)UG.ncolors * r, c1pad = pad16(c1);
  const int64_t c2 = (int64_t)G.ncolors * kmax, c2pad = pad16(c2);
  void *X = Xb.p, *Y = Yb.p;
  auto apply_bb = [&](int trans, int64_t cols, const DBuf &kit, int32_t nkit, bool f32) {
    if (direct) {
      autotune_kapply(KapplyShape{f32, kbb->kernel, T.dim, cols, n, true, nkit},
                      [&](int nt, int64_t part) {
                        launch_kapply_forest(kbb->kernel, T.dim, n, Dv.pts.as<double>(),
                                             part > 0 ? (int32_t)part : nkit, kit.as<KItem>(),
                                             cols, -1, nt, f32, X, n, Y, n, s);
                      },
                      s);
      LAUNCH_CHECK();
    } else {
      call_blackbox(bb, bb.symmetric ? 0 : trans, n, cols, f32, X, n, Y, n, Dv, tmpx, tmpy, s);
    }
  };
  constexpr double kNoiseGamma = 8.0;
  const bool gamma = (o.flags & HM_FLAG_MIX_GAMMA) != 0;  // extension: weighted combination
  // ---------------- stage 1: augmented samples, SVD column bases
  if (UG.nv() > 0) {
    ev.mark(0);
    launch_testmat(n, Dv.rowbox[l].as<int32_t>(), J.act.as<uint8_t>(), UG.ncolors, r, l, 2,
                   o.seed, Dv.inst_off.as<int64_t>(), ni, mixed, X, n, c1pad, s);
    LAUNCH_CHECK();
    ev.mark(1);
    apply_bb(0, c1pad, J.kit1, J.nkit1, mixed);
    cols_A += c1;
    if (mixed) {
      launch_block_norms(J.nv, J.jn.as<QrJob>(), r, kNoiseGamma * 0x1p-24 / std::sqrt((double)r),
                         true, Y, n, floor_u.as<double>(), s);
      LAUNCH_CHECK();
    }
    ev.mark(2);
    h2_apply(*H, li, false, mixed, X, n, c1pad, Y, n, -1.0, h2q.as<double>(), h2u.as<double>(),
             h2p.as<double>(), h2cols, s);
    launch_check_finite(n, c1pad, mixed, Y, n, flag.as<int32_t>(), s);
    LAUNCH_CHECK();
  }
  ev.mark(3);
  launch_h2_sample(J.naug, J.augu.as<AugJob>(), r, l, 2, o.seed, mixed, Y, n, H->UB.as<double>(),
                   rk, H->SU.as<double>(), kmax, Sb.as<double>(), n, s);
  launch_svd_basis(J.nv, J.ju.as<QrJob>(), r, kfix, o.tol, kfix > 0 ? kfix : r - p,
                   mixed ? floor_u.as<double>() : nullptr, Sb.as<double>(), n, work.as<double>(),
                   H->UB.as<double>(), H->SU.as<double>() + v0 * kmax, kmax, rk + v0,
                   usat.as<int32_t>() + v0, s);
  LAUNCH_CHECK();
  // ---------------- stage 2: Z, sums, augmented SVD row bases; FP64 in both
  // precisions, as in the uniform format (the samples are summed)
  if (G.nv() > 0) {
    ev.mark(0);
    launch_basis_testmat(n, Dv.rowbox[l].as<int32_t>(), Dv.start[l].as<int64_t>(),
                         J.slot.as<int32_t>(), G.ncolors, kmax, H->UB.as<double>(),
                         J.uoff.as<int64_t>(), rk + v0, false, X, n, c2pad, s);
    LAUNCH_CHECK();
    ev.mark(1);
    apply_bb(1, c2pad, J.kit2, J.nkit2, false);
    cols_At += c2;
    ev.mark(2);
    h2_apply(*H, li, true, false, X, n, c2pad, Y, n, -1.0, h2q.as<double>(), h2u.as<double>(),
             h2p.as<double>(), h2cols, s);
    launch_check_finite(n, c2pad, false, Y, n, flag.as<int32_t>(), s);
    LAUNCH_CHECK();
  }
  ev.mark(3);
  launch_mix_sum(J.nmix, J.mix.as<MixJob>(), J.terms.as<MixTerm>(), kmax, l, o.seed, gamma, false, Y, n,
                 Sb.as<double>(), n, s);
  launch_h2_sample(J.naug, J.augv.as<AugJob>(), kmax, l, 3, o.seed, false, Sb.p, n,
                   H->VB.as<double>(), rk + nb, H->SV.as<double>(), kmax, Sb.as<double>(), n, s);
  launch_svd_basis(J.nv, J.jv.as<QrJob>(), kmax, kfix, o.tol, kmax, nullptr, Sb.as<double>(), n,
                   work.as<double>(), H->VB.as<double>(), H->SV.as<double>() + v0 * kmax, kmax,
                   rk + nb + v0, usat.as<int32_t>() + nb + v0, s);
  LAUNCH_CHECK();
  ev.mark(4);
  // couplings and the pair copies of the bases (the exported blocks); the
  // products W = U B only serve the per-pair apply plan, which H^2 does not use
  launch_ucoupling((int32_t)L.np, J.uc.as<UCJob>(), kmax, false, Y, n, H->UB.as<double>(),
                   H->VB.as<double>(), rk + v0, rk + nb + v0, nullptr, nullptr,
                   H->B.as<double>(), nullptr, H->ranks.as<int32_t>(), true, s);
  LAUNCH_CHECK();
  // ---------------- nest the previous level; after the last level rebuild the
  // bases the nesting implies on every coarser level (for export: the peel and
  // the apply read only long bases and transfers, and a transfer is taken
  // from the parent's basis as computed, before any rebuild)
  if (li > 0) {
    const UniformJobs &Jc = J;
    launch_transfer(Jc.ntr, Jc.tr.as<TransferJob>(), kmax, H->UB.as<double>(), rk,
                    H->TU.as<double>(), s);
    launch_transfer(Jc.ntr, Jc.tr.as<TransferJob>(), kmax, H->VB.as<double>(), rk + nb,
                    H->TV.as<double>(), s);
    LAUNCH_CHECK();
    for (size_t lj = li + 1 == H->lv.size() ? li : 0; lj-- > 0;) {
      // level lj's bases from level lj + 1's through the transfers of lj + 1's boxes
      const UniformJobs &Jn = ujobs_of[lj + 1];
      launch_nest(Jn.nnest, Jn.nest.as<NestJob>(), kmax, H->UB.as<double>(), H->TU.as<double>(),
                  rk, H->UB.as<double>(), s);
      launch_nest(Jn.nnest, Jn.nest.as<NestJob>(), kmax, H->VB.as<double>(), H->TV.as<double>(),
                  rk + nb, H->VB.as<double>(), s);
      LAUNCH_CHECK();
    }
  }
}

// One uniform level: stage 1 (column bases), stage 2 (row bases, couplings).
void Compression::record_uniform_level(size_t li, hipStream_t s, Events &ev) {
  const DeviceTree &Dv = *D;
  hm_hmatrix::Lv &L = H->lv[li];
  const int l = L.level;
  const Graph &G = T.graphs[l], &UG = T.ugraphs[l];
  UniformJobs &J = ujobs_of[li];
  const int64_t v0 = H->uv0[li];
  int32_t *urank = H->brank.as<int32_t>() + v0;
  int32_t *vrank = H->brank.as<int32_t>() + H->nvtot + v0;
  const int64_t c1 = (int64_t)UG.ncolors * r, c1pad = pad16(c1);
  const int64_t c2 = (int64_t)G.ncolors * kmax, c2pad = pad16(c2);
  void *X = Xb.p, *Y = Yb.p;
  // black box on the first `cols` columns of X into Y (A, or A* when trans)
  auto apply_bb = [&](int trans, int64_t cols, const DBuf &kit, int32_t nkit, bool f32) {
    if (direct) {
      autotune_kapply(KapplyShape{f32, kbb->kernel, T.dim, cols, n, true, nkit},
                      [&](int nt, int64_t part) {
                        launch_kapply_forest(kbb->kernel, T.dim, n, Dv.pts.as<double>(),
                                             part > 0 ? (int32_t)part : nkit, kit.as<KItem>(),
                                             cols, -1, nt, f32, X, n, Y, n, s);
                      },
                      s);
      LAUNCH_CHECK();
    } else {
      call_blackbox(bb, bb.symmetric ? 0 : trans, n, cols, f32, X, n, Y, n, Dv, tmpx, tmpy, s);
    }
  };
  constexpr double kNoiseGamma = 8.0;  // see the mixed floor of record()
  const bool gamma = (o.flags & HM_FLAG_MIX_GAMMA) != 0;  // extension: weighted combination
  // ---------------- stage 1: Y = (A - A^(l)) Omega, U_a = qr(Y(I_a, block))
  ev.mark(0);
  launch_testmat(n, Dv.rowbox[l].as<int32_t>(), J.act.as<uint8_t>(), UG.ncolors, r, l, 2, o.seed,
                 Dv.inst_off.as<int64_t>(), ni, mixed, X, n, c1pad, s);
  LAUNCH_CHECK();
  ev.mark(1);
  apply_bb(0, c1pad, J.kit1, J.nkit1, mixed);
  cols_A += c1;
  if (mixed) {
    launch_block_norms(J.nv, J.ju.as<QrJob>(), r, kNoiseGamma * 0x1p-24 / std::sqrt((double)r),
                       true, Y, n, floor_u.as<double>(), s);
    LAUNCH_CHECK();
  }
  ev.mark(2);
  const PeelPattern pp1{ColorPattern{Dv.rowbox[l].as<int32_t>(), Dv.start[l].as<int64_t>(),
                                     J.act.as<uint8_t>(), UG.ncolors, r, 0},
                        tflags.as<uint8_t>(), tflag_cap};
  apply_levels(*H, li, false, mixed, X, n, c1pad, Y, n, -1.0, Tb.p, tcap, s, peel_plans, &pp1);
  launch_check_finite(n, c1pad, mixed, Y, n, flag.as<int32_t>(), s);
  LAUNCH_CHECK();
  ev.mark(3);
  launch_pivqr(J.nv, J.ju.as<QrJob>(), r, kfix, o.tol, kfix > 0 ? kfix : r - p,
               mixed ? floor_u.as<double>() : nullptr, mixed, Y, n, work.as<double>(),
               H->UB.as<double>(), urank, usat.as<int32_t>() + v0, s);
  LAUNCH_CHECK();
  // ---------------- stage 2: Z = (A - A^(l))* Psi(U), V_b = qr(sum_a Z_ba).
  // FP64 in both precisions: the sum adds column j of every term, and where
  // the terms cancel, the directions V_b must keep fall below the rounding
  // of an FP32 sample (a mixed stage 2 measured 2.5e-4 against 5e-7).
  ev.mark(0);
  launch_basis_testmat(n, Dv.rowbox[l].as<int32_t>(), Dv.start[l].as<int64_t>(),
                       J.slot.as<int32_t>(), G.ncolors, kmax, H->UB.as<double>(),
                       J.uoff.as<int64_t>(), urank, false, X, n, c2pad, s);
  LAUNCH_CHECK();
  ev.mark(1);
  apply_bb(1, c2pad, J.kit2, J.nkit2, false);
  cols_At += c2;
  ev.mark(2);
  apply_levels(*H, li, true, false, X, n, c2pad, Y, n, -1.0, Tb.p, tcap, s, peel_plans);
  launch_check_finite(n, c2pad, false, Y, n, flag.as<int32_t>(), s);
  LAUNCH_CHECK();
  ev.mark(3);
  launch_mix_sum(J.nmix, J.mix.as<MixJob>(), J.terms.as<MixTerm>(), kmax, l, o.seed, gamma, false, Y, n,
                 Sb.as<double>(), n, s);
  launch_pivqr(J.nv, J.jv.as<QrJob>(), kmax, kfix, o.tol, kmax, nullptr, false, Sb.p, n,
               work.as<double>(), H->VB.as<double>(), vrank, usat.as<int32_t>() + H->nvtot + v0, s);
  LAUNCH_CHECK();
  ev.mark(4);
  launch_ucoupling((int32_t)L.np, J.uc.as<UCJob>(), kmax, false, Y, n, H->UB.as<double>(),
                   H->VB.as<double>(), urank, vrank, H->U.as<double>(), H->V.as<double>(),
                   H->B.as<double>(), H->W.as<double>(), H->ranks.as<int32_t>(), true, s);
  LAUNCH_CHECK();
}

// FP32 copies of level li's apply factors
void Compression::fp32_copies(size_t li, hipStream_t s) {
  const hm_hmatrix::Lv &L = H->lv[li];
  const int64_t u0 = L.offU.empty() ? 0 : L.offU[0];
  const int64_t u1 = li + 1 < H->lv.size() ? H->lv[li + 1].offU[0] : szU;
  const int64_t v0 = L.offV.empty() ? 0 : L.offV[0];
  const int64_t v1 = li + 1 < H->lv.size() ? H->lv[li + 1].offV[0] : szV;
  launch_convert(u1 - u0, 1, false, H->W.as<double>() + u0, u1 - u0, H->Wf.as<float>() + u0,
                 u1 - u0, s);
  launch_convert(v1 - v0, 1, false, H->V.as<double>() + v0, v1 - v0, H->Vf.as<float>() + v0,
                 v1 - v0, s);
  LAUNCH_CHECK();
}

void Compression::record(hipStream_t s, Events &ev) {
  const DeviceTree &Dv = *D;
  const Graph &GL = T.leaf_graph();
  // state every run starts from (fill kernels, no memset: capturable)
  if (!h2) launch_fill(H->W.p, szU, false, 0.0, s);
  if (!h2) launch_fill(H->V.p, szV, false, 0.0, s);
  launch_fill(H->ranks.p, 2 * np_total, true, 0.0, s);  // int32 zeros share the float bit pattern
  launch_fill(sat.p, std::max<int64_t>(2 * np_total, 1), true, 0.0, s);
  launch_fill(flag.p, 1, true, 0.0, s);
  if (!uniform) launch_fill(counters.p, std::max<int64_t>((int64_t)H->lv.size(), 1), true, 0.0, s);
  LAUNCH_CHECK();
  cols_A = cols_At = 0;
  // ---------------- the level loop (no host round trips)
  if (uniform) launch_fill(usat.p, std::max<int64_t>(2 * H->nvtot, 1), true, 0.0, s);
  for (size_t li = 0; li < H->lv.size(); ++li) {
    hm_hmatrix::Lv &L = H->lv[li];
    if (uniform) {
      if (h2) {
        record_h2_level(li, s, ev);
      } else {
        record_uniform_level(li, s, ev);
        fp32_copies(li, s);
      }
      ev.mark(5);
      continue;
    }
    const int l = L.level;
    const Graph &G = T.graphs[l];
    const int64_t c = (int64_t)G.ncolors * r;
    const int64_t cpad = pad16(c);
    void *Om = Xb.p;
    void *Ps = (char *)Xb.p + (size_t)cpad * n * es;
    void *Yl = Yb.p;
    void *Zl = (char *)Yb.p + (size_t)cpad * n * es;
    DBuf &dact = jobs_of[li].act;
    ev.mark(0);
    launch_testmat(n, Dv.rowbox[l].as<int32_t>(), dact.as<uint8_t>(), G.ncolors, r, l, 0, o.seed,
                   Dv.inst_off.as<int64_t>(), ni, mixed, Om, n, cpad, s);
    launch_testmat(n, Dv.rowbox[l].as<int32_t>(), dact.as<uint8_t>(), G.ncolors, r, l, 1, o.seed,
                   Dv.inst_off.as<int64_t>(), ni, mixed, Ps, n, cpad, s);
    LAUNCH_CHECK();
    ev.mark(1);
    if (direct) {
      autotune_kapply(KapplyShape{mixed, kbb->kernel, T.dim, 2 * cpad, n, true, jobs_of[li].nkit},
                      [&](int nt, int64_t part) {
                        launch_kapply_forest(kbb->kernel, T.dim, n, Dv.pts.as<double>(),
                                             part > 0 ? (int32_t)part : jobs_of[li].nkit,
                                             jobs_of[li].kit.as<KItem>(), 2 * cpad, cpad, nt,
                                             mixed, Om, n, Yl, n, s);
                      },
                      s);
      LAUNCH_CHECK();
    } else if (bb.symmetric) {
      call_blackbox(bb, 0, n, 2 * cpad, mixed, Om, n, Yl, n, Dv, tmpx, tmpy, s);
    } else {
      call_blackbox(bb, 0, n, cpad, mixed, Om, n, Yl, n, Dv, tmpx, tmpy, s);
      call_blackbox(bb, 1, n, cpad, mixed, Ps, n, Zl, n, Dv, tmpx, tmpy, s);
    }
    cols_A += c;
    cols_At += c;
    // Mixed path: a sample block computed in FP32 carries rounding noise of
    // about 3 u32 ||block||_F before the peel (measured for the compensated
    // FP32 kernel apply, independent of N).  Rank decisions below
    // kNoiseGamma u32 ||raw block||_F / sqrt(r) would be decided by that
    // noise and drive every such block to the rank cap, so the pivoted QR
    // stops there as well.
    if (mixed) {
      constexpr double kNoiseGamma = 8.0;
      const double scale = kNoiseGamma * 0x1p-24 / std::sqrt((double)r);
      launch_block_norms((int32_t)L.np, jobs_of[li].ju.as<QrJob>(), r, scale, true, Yb.p, n,
                         floor_u.as<double>(), s);
      launch_block_norms((int32_t)L.np, jobs_of[li].jv.as<QrJob>(), r, scale, true, Yb.p, n,
                         floor_v.as<double>(), s);
      LAUNCH_CHECK();
    }
    ev.mark(2);
    // Omega and Psi share the zero pattern of the level's colors
    const PeelPattern pp{ColorPattern{Dv.rowbox[l].as<int32_t>(), Dv.start[l].as<int64_t>(),
                                      dact.as<uint8_t>(), G.ncolors, r, 0},
                         tflags.as<uint8_t>(), tflag_cap};
    apply_levels(*H, li, false, mixed, Om, n, cpad, Yl, n, -1.0, Tb.p, tcap, s, peel_plans, &pp);
    apply_levels(*H, li, true, mixed, Ps, n, cpad, Zl, n, -1.0, Tb.p, tcap, s, peel_plans, &pp);
    launch_check_finite(n, 2 * cpad, mixed, Yb.p, n, flag.as<int32_t>(), s);
    LAUNCH_CHECK();
    ev.mark(3);
    // per pair: core, the pivoted QRs of the Y and Z blocks, the coupling
    // solve and W = U B, in one persistent launch over the level's pairs
    // (the QR stage's time includes the solves)
    RecoverArgs ra{};
    ra.jc = jobs_of[li].jc.as<CoreJob>();
    ra.ju = jobs_of[li].ju.as<QrJob>();
    ra.jv = jobs_of[li].jv.as<QrJob>();
    ra.order = jobs_of[li].order.as<int32_t>();
    ra.counter = counters.as<int32_t>() + li;
    ra.njobs = (int32_t)L.np;
    ra.r = r;
    ra.kmax = kmax;
    ra.rank_fixed = kfix;
    ra.cap = kfix > 0 ? kfix : r - p;
    ra.tol = o.tol;
    ra.ld = n;
    ra.floor_u = mixed ? floor_u.as<double>() : nullptr;
    ra.floor_v = mixed ? floor_v.as<double>() : nullptr;
    ra.work = work.as<double>();
    ra.U = H->U.as<double>();
    ra.V = H->V.as<double>();
    ra.core = core.as<double>();
    ra.scratch = scratch.as<double>();
    ra.B = H->B.as<double>();
    ra.W = H->W.as<double>();
    ra.ranks = H->ranks.as<int32_t>();
    ra.ranks_u = H->ranks.as<int32_t>() + L.g0;
    ra.ranks_v = H->ranks.as<int32_t>() + np_total + L.g0;
    ra.sat_u = sat.as<int32_t>() + L.g0;
    ra.sat_v = sat.as<int32_t>() + np_total + L.g0;
    launch_recover(ra, recover_grid, mixed, Xb.p, Xb.p, Yb.p, s);
    LAUNCH_CHECK();
    ev.mark(4);
    fp32_copies(li, s);
    ev.mark(5);
  }

  // ---------------- leaf pass
  ev.mark(0);
  launch_leaf_identity(n, nib, dib.as<int32_t>(), dic.as<int32_t>(),
                       Dv.start[T.L()].as<int64_t>(), mw, mixed, Xb.p, n, leaf_cols, s);
  LAUNCH_CHECK();
  ev.mark(1);
  if (direct) {
    autotune_kapply(KapplyShape{mixed, kbb->kernel, T.dim, leaf_cols, n, true,
                                (int64_t)nkit_leaf},
                    [&](int nt, int64_t part) {
                      launch_kapply_forest(kbb->kernel, T.dim, n, Dv.pts.as<double>(),
                                           part > 0 ? (int32_t)part : nkit_leaf,
                                           dkit.as<KItem>(), leaf_cols, -1, nt, mixed, Xb.p, n,
                                           Yb.p, n, s);
                    },
                    s);
    LAUNCH_CHECK();
  } else {
    call_blackbox(bb, 0, n, leaf_cols, mixed, Xb.p, n, Yb.p, n, Dv, tmpx, tmpy, s);
  }
  cols_A += (int64_t)GL.ncolors * mw;
  ev.mark(2);
  if (h2) {
    h2_apply(*H, H->lv.size(), false, mixed, Xb.p, n, leaf_cols, Yb.p, n, -1.0, h2q.as<double>(),
             h2u.as<double>(), h2p.as<double>(), h2cols, s);
  } else {
    // the identity blocks: color c is zero on the leaf boxes not active in it
    const PeelPattern pl{ColorPattern{Dv.rowbox[T.L()].as<int32_t>(),
                                      Dv.start[T.L()].as<int64_t>(), leaf_act.as<uint8_t>(),
                                      GL.ncolors, mw, 0},
                         tflags.as<uint8_t>(), tflag_cap};
    apply_levels(*H, H->lv.size(), false, mixed, Xb.p, n, leaf_cols, Yb.p, n, -1.0, Tb.p, tcap,
                 s, peel_plans, &pl);
  }
  launch_check_finite(n, leaf_cols, mixed, Yb.p, n, flag.as<int32_t>(), s);
  LAUNCH_CHECK();
  ev.mark(3);
  launch_extract_near((int32_t)GL.pa.size(), dr0.as<int64_t>(), dma.as<int32_t>(),
                      dc0.as<int64_t>(), dmb.as<int32_t>(), doff.as<int64_t>(), mixed, Yb.p, n,
                      H->D.as<double>(), s);
  LAUNCH_CHECK();
  ev.mark(5);
}

hm_status Compression::finalize(hipStream_t s, Events &ev,
                                std::chrono::steady_clock::time_point t_host0) {
  const Graph &GL = T.leaf_graph();
  const Level &LL = T.lev[T.L()];
  // ---------------- results back on the host
  H->h_ranks.resize(2 * np_total);
  std::vector<int32_t> hsat(2 * np_total);
  int32_t hflag = 0;
  if (np_total) {
    HIP_TRY(hipMemcpyAsync(H->h_ranks.data(), H->ranks.p, 2 * np_total * 4,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hsat.data(), sat.p, 2 * np_total * 4, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipMemcpyAsync(&hflag, flag.p, 4, hipMemcpyDeviceToHost, s));
  std::vector<int32_t> husat;
  if (uniform && H->nvtot) {
    H->h_brank.resize(2 * H->nvtot);
    husat.resize(2 * H->nvtot);
    HIP_TRY(hipMemcpyAsync(H->h_brank.data(), H->brank.p, 2 * H->nvtot * 4,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(husat.data(), usat.p, 2 * H->nvtot * 4, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (hflag) return fail(HM_E_NUMERIC, "NaN or Inf in the black-box samples");

  // ---------------- statistics
  hm_stats &st = H->stats;
  st = hm_stats{};
  st.nlevels = T.nlev();
  st.r = r;
  st.n = n;
  st.cols_A = cols_A;
  st.cols_At = cols_At;
  for (int l : levels)
    if (l < 32) st.colors[l] = T.graphs[l].ncolors;
  st.leaf_colors = GL.ncolors;
  st.leaf_width = mw;
  st.npairs = np_total;
  st.nnear = (int64_t)GL.pa.size();
  double fpeel = 0, fqr = 0, fsolve = 0;
  int64_t nfloats = szD;
  // algorithmic work is counted per instance: instance i applies its own
  // operator to its own live columns and peels its own factors
  // apply_cost[li][i]: flops per column of instance i's level-li factors
  std::vector<std::vector<double>> apply_cost_of(H->lv.size(), std::vector<double>(ni, 0.0));
  for (size_t li = 0; li < H->lv.size(); ++li) {
    const hm_hmatrix::Lv &L = H->lv[li];
    const Level &Lv = T.lev[L.level];
    std::vector<double> &apply_cost = apply_cost_of[li];
    for (int64_t q = 0; q < L.np; ++q) {
      const int64_t ma = Lv.start[L.pa[q] + 1] - Lv.start[L.pa[q]];
      const int64_t mb = Lv.start[L.pb[q] + 1] - Lv.start[L.pb[q]];
      const int ku = H->h_ranks[L.g0 + q], kv = H->h_ranks[np_total + L.g0 + q];
      st.max_rank = std::max(st.max_rank, std::max(ku, kv));
      st.saturated += hsat[L.g0 + q] + hsat[np_total + L.g0 + q];
      apply_cost[ni > 1 ? inst_of_row(Lv.start[L.pa[q]]) : 0] += 2.0 * kv * (ma + mb);
      if (uniform) {
        // coupling B = Z_blk^T V_b and W = U_a B; bases counted per box below
        nfloats += (int64_t)ku * kv;
        fsolve += 2.0 * mb * ku * kv + 2.0 * ma * ku * kv;
        continue;
      }
      nfloats += ma * ku + (int64_t)ku * kv + mb * kv;
      fqr += qr_flops(ma, r, ku) + qr_flops(mb, r, kv);
      fsolve += 2.0 * ma * r * r + 2.0 * ma * r * ku + 2.0 * mb * r * kv + 4.0 * r * ku * ku +
                4.0 * r * kv * kv + 2.0 * r * r * (ku + kv) + 2.0 * ma * ku * kv;
    }
    if (uniform) {
      st.format = h2 ? HM_FORMAT_H2 : HM_FORMAT_UNIFORM_H1;
      if (L.level < 32) st.ucolors[L.level] = T.ugraphs[L.level].ncolors;
      const int64_t v0 = H->uv0[li];
      // H^2: basis index of each box of the previous level (transfers), and
      // the boxes with a basis on the next level below them (a box without
      // one keeps its long bases)
      std::vector<int32_t> pv;
      if (h2 && li > 0) {
        pv.assign(T.lev[H->lv[li - 1].level].nbox(), -1);
        for (size_t v = 0; v < H->ubox[li - 1].size(); ++v) pv[H->ubox[li - 1][v]] = (int32_t)v;
      }
      std::vector<uint8_t> parent_of_basis(Lv.nbox(), 0);
      if (h2 && li + 1 < H->lv.size()) {
        const Level &Ln = T.lev[H->lv[li + 1].level];
        for (int c : H->ubox[li + 1]) parent_of_basis[Ln.parent[c]] = 1;
      }
      for (size_t v = 0; v < H->ubox[li].size(); ++v) {
        const int a = H->ubox[li][v];
        const int64_t m = Lv.start[a + 1] - Lv.start[a];
        const int ku = H->h_brank[v0 + v], kv = H->h_brank[H->nvtot + v0 + v];
        st.saturated += husat[v0 + v];
        if (!h2 || !parent_of_basis[a]) nfloats += m * (ku + kv);
        if (h2 && li > 0 && pv[Lv.parent[a]] >= 0) {
          const int64_t g = H->uv0[li - 1] + pv[Lv.parent[a]];
          nfloats += (int64_t)ku * H->h_brank[g] + (int64_t)kv * H->h_brank[H->nvtot + g];
          // transfers, and the nested bases rebuilt on every coarser level
          fsolve += 2.0 * m * (ku * H->h_brank[g] + kv * H->h_brank[H->nvtot + g]) *
                    (1.0 + (double)(H->lv.size() - li));
        }
        if (h2) {
          // QR, Jacobi sweeps (about 10), basis formation; the augmentation
          fqr += 2.0 * qr_flops(m, r, r) + 20.0 * r * r * r;
          fsolve += 4.0 * m * kmax * r;
        } else {
          fqr += qr_flops(m, r, ku) + qr_flops(m, kmax, kv);
        }
        // the combination sum_a Z_ba Gamma_a
        fsolve += 2.0 * m * kmax * kmax * (T.lev[L.level].int_ptr[a + 1] - T.lev[L.level].int_ptr[a]);
      }
    }
  }
  double fbb = 0, bpeel = 0;
  {
    const double es1 = mixed ? 4.0 : 8.0;
    // Work of a peel through a zero pattern: sampled level ls whose test
    // matrix has color blocks of colw columns, block c nonzero only on the
    // boxes active in c (act, nc colors), minus the operator of levels
    // [0, li_end) in one orientation.  A pair projects only the active
    // blocks inside its column box (2 k rows colw flops each; an identity
    // block has one nonzero per row: 2 k rows) and expands only the colors
    // whose projection is nonzero (2 k |row box| colw each).  Bytes: each
    // nonzero block of X read once, each Y element some pair updates read
    // and written once, each factor of a pair with a nonzero projection
    // read once.
    auto pattern_peel = [&](size_t li_end, bool trans, const std::vector<uint8_t> &act, int nc,
                            int64_t colw, int ls, bool identity, double &flops, double &bytes) {
      if (li_end == 0 || nc <= 0) return;
      const Level &LS = T.lev[ls];
      const int words = (nc + 63) / 64;
      std::vector<uint8_t> xread(act.size(), 0);
      std::vector<std::vector<uint64_t>> rows_live(li_end);  // per level: colors on each row box
      for (size_t li = 0; li < li_end; ++li) {
        const hm_hmatrix::Lv &L = H->lv[li];
        const Level &Lv = T.lev[L.level];
        rows_live[li].assign((size_t)Lv.nbox() * words, 0);
        std::unordered_map<int, std::vector<std::pair<int, int64_t>>> colors_of;  // column box
        for (int64_t q = 0; q < L.np; ++q) {
          const int cb = trans ? L.pa[q] : L.pb[q], rb = trans ? L.pb[q] : L.pa[q];
          const int kv = H->h_ranks[np_total + L.g0 + q];
          if (kv == 0) continue;
          auto it = colors_of.find(cb);
          if (it == colors_of.end()) {
            std::vector<int64_t> rows(nc, 0);
            const int64_t s0 = Lv.start[cb], s1 = Lv.start[cb + 1];
            int b = (int)(std::upper_bound(LS.start.begin(), LS.start.end(), s0) -
                          LS.start.begin()) - 1;
            for (b = std::max(b, 0); b < LS.nbox() && LS.start[b] < s1; ++b) {
              const int64_t m = LS.start[b + 1] - LS.start[b];
              if (m == 0) continue;
              for (int c = 0; c < nc; ++c)
                if (act[(size_t)b * nc + c]) {
                  rows[c] += m;
                  xread[(size_t)b * nc + c] = 1;
                }
            }
            std::vector<std::pair<int, int64_t>> v;
            for (int c = 0; c < nc; ++c)
              if (rows[c] > 0) v.emplace_back(c, rows[c]);
            it = colors_of.emplace(cb, std::move(v)).first;
          }
          if (it->second.empty()) continue;
          const int64_t ma = Lv.start[rb + 1] - Lv.start[rb];
          const int64_t mb = Lv.start[cb + 1] - Lv.start[cb];
          for (const auto &cr : it->second) {
            flops += 2.0 * kv * (identity ? (double)cr.second : (double)cr.second * colw);
            flops += 2.0 * kv * (double)ma * colw;
            rows_live[li][(size_t)rb * words + cr.first / 64] |= uint64_t(1) << (cr.first % 64);
          }
          bytes += es1 * kv * (double)(ma + mb);
        }
      }
      for (size_t e = 0; e < xread.size(); ++e)
        if (xread[e]) bytes += es1 * (double)(LS.start[e / nc + 1] - LS.start[e / nc]) * colw;
      // Y: each box of the finest included level, the colors of its ancestors' pairs
      const int fine = H->lv[li_end - 1].level;
      const Level &LF = T.lev[fine];
      std::vector<uint64_t> u(words);
      for (int a = 0; a < LF.nbox(); ++a) {
        std::fill(u.begin(), u.end(), 0);
        for (size_t li = 0; li < li_end; ++li) {
          int b = a;
          for (int l = fine; l > H->lv[li].level; --l) b = T.lev[l].parent[b];
          for (int w = 0; w < words; ++w) u[w] |= rows_live[li][(size_t)b * words + w];
        }
        int64_t cnt = 0;
        for (int w = 0; w < words; ++w) cnt += __builtin_popcountll(u[w]);
        bytes += 2.0 * es1 * (double)(LF.start[a + 1] - LF.start[a]) * cnt * colw;
      }
    };
    // Dense peel bytes (a level without a pattern: H^2, the uniform
    // format's stage 2): X read and Y read and written once (es bytes per
    // element; stage 2 in FP64), every coarser factor read once (V and
    // W = U B, prev / 2 elements).
    std::vector<double> prev(ni, 0.0);
    for (size_t li = 0; li < H->lv.size(); ++li) {
      const int l = H->lv[li].level;
      const std::vector<int32_t> w = inst_colors(l);
      std::vector<int32_t> wu(ni, 0);
      if (uniform) {
        const Graph &UG = T.ugraphs[l];
        for (int64_t v = 0; v < UG.nv(); ++v) {
          const int i = inst_of_row(T.lev[l].start[UG.vbox[v]]);
          wu[i] = std::max(wu[i], UG.color[v] + 1);
        }
      }
      const bool pat = li < h_act.size() && !h_act[li].empty();
      for (int i = 0; i < ni; ++i) {
        // columns of the Y and Z passes
        const double c = uniform ? (double)wu[i] * r + (double)w[i] * kmax : 2.0 * w[i] * r;
        const double ni_rows = (double)(T.inst_off[i + 1] - T.inst_off[i]);
        fbb += 2.0 * ni_rows * ni_rows * c;
        if (pat) {
          if (uniform && prev[i] > 0) {
            // stage 2 (A*) runs dense
            fpeel += (double)w[i] * kmax * prev[i];
            bpeel += 3.0 * ni_rows * (double)w[i] * kmax * 8.0 + 8.0 * prev[i] / 2.0;
          }
          continue;
        }
        fpeel += c * prev[i];
        if (prev[i] > 0) {
          const double sbytes = uniform ? (double)wu[i] * r * es1 + (double)w[i] * kmax * 8.0
                                        : c * es1;
          bpeel += 3.0 * ni_rows * sbytes + (uniform ? es1 + 8.0 : es1) * prev[i] / 2.0;
        }
      }
      if (pat) {
        // A (both formats) and A* (H^1) through the level's pattern
        pattern_peel(li, false, h_act[li], h_act_nc[li], r, l, false, fpeel, bpeel);
        if (!uniform) pattern_peel(li, true, h_act[li], h_act_nc[li], r, l, false, fpeel, bpeel);
      }
      for (int i = 0; i < ni; ++i) prev[i] += apply_cost_of[li][i];
    }
    // leaf pass: an instance's identity blocks are as wide as its own
    // largest leaf
    const std::vector<int32_t> wl = inst_colors(T.nlev());
    std::vector<int64_t> mwi(ni, 0);
    for (int b = 0; b < LL.nbox(); ++b) {
      const int i = ni > 1 ? inst_of_row(LL.start[b]) : 0;
      mwi[i] = std::max(mwi[i], LL.start[b + 1] - LL.start[b]);
    }
    for (int i = 0; i < ni; ++i) {
      const double ni_rows = (double)(T.inst_off[i + 1] - T.inst_off[i]);
      fbb += 2.0 * ni_rows * ni_rows * (double)wl[i] * mwi[i];
      if (!h2) continue;
      fpeel += (double)wl[i] * mwi[i] * prev[i];
      if (prev[i] > 0) bpeel += 3.0 * ni_rows * (double)wl[i] * mwi[i] * es1 + es1 * prev[i] / 2.0;
    }
    if (!h2)
      pattern_peel(H->lv.size(), false, h_leaf_act, GL.ncolors, mw, T.L(), true, fpeel, bpeel);
  }
  st.nfloats = nfloats;
  st.flops_blackbox = fbb;
  st.flops_peel = fpeel;
  st.flops_qr = fqr;
  st.flops_solve = fsolve;
  st.bytes_peel = bpeel;
  if (ev.on && !ev.marks.empty()) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (size_t i = 0; i + 1 < ev.marks.size(); ++i) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, ev.marks[i].first, ev.marks[i + 1].first);
      acc[ev.marks[i].second] += ms;
    }
    st.ms_blackbox = acc[1];
    st.ms_peel = acc[2];
    st.ms_qr = acc[3];
    st.ms_solve = acc[4];
    st.ms_other = acc[0] + acc[5];
  }
  st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host0).count();
  return HM_OK;
}

hm_status compress_impl(Tree &T, const hm_blackbox &bb, const hm_compress_opts &o,
                        hipStream_t s, hm_hmatrix **out) {
  auto t_host0 = std::chrono::steady_clock::now();
  AllocScope scope(o.allocator);
  Compression C(T, bb, o);
  hm_status st = C.setup(s);
  if (st != HM_OK) return st;
  Events ev;
  ev.on = (o.flags & HM_FLAG_TIMING) != 0;
  ev.s = s;
  C.record(s, ev);
  st = C.finalize(s, ev, t_host0);
  if (st != HM_OK) return st;
  *out = C.H.release();
  return HM_OK;
}

}  // namespace

// Device bytes an H-matrix holds (factor pools, near blocks, apply plans).
int64_t hmatrix_device_bytes(const hm_hmatrix *H) {
  int64_t b = H->perm.bytes + H->U.bytes + H->V.bytes + H->W.bytes + H->B.bytes + H->Vf.bytes +
              H->Wf.bytes + H->D.bytes + H->ranks.bytes + H->nchunks.bytes + H->nentries.bytes +
              H->nchunksT.bytes + H->nentriesT.bytes + H->UB.bytes + H->VB.bytes + H->brank.bytes +
              H->SU.bytes + H->SV.bytes + H->TU.bytes + H->TV.bytes + H->h2a.leaf.bytes +
              H->h2a.chunk.bytes;
  for (const auto *v : {&H->h2a.up_j, &H->h2a.up_t, &H->h2a.dn_j, &H->h2a.dn_t, &H->h2a.dnt_j,
                        &H->h2a.dnt_t})
    for (const DBuf &d : *v) b += d.bytes;
  for (const hm_hmatrix::Orient *O : {&H->oA, &H->oT}) {
    b += O->items.bytes + O->ppairs.bytes + O->red.bytes;
    for (const DBuf &d : O->chunks) b += d.bytes;
    for (const DBuf &d : O->entries) b += d.bytes;
  }
  return b;
}

// Device bytes of T's device copy (device_tree: coordinates, permutation,
// per-level row boxes and box starts, instance offsets, forest items), each
// block rounded as the block cache rounds it.
int64_t tree_device_bytes(const Tree &T) {
  auto blk = [](int64_t b) { return (std::max<int64_t>(b, 64) + 255) / 256 * 256; };
  int64_t b = blk((int64_t)T.dim * T.n * 8) + blk(T.n * 8) + blk((int64_t)(T.ninst() + 1) * 8);
  for (int l = 0; l < T.nlev(); ++l)
    b += blk(T.n * 4) + blk((int64_t)(T.lev[l].nbox() + 1) * 8);
  if (T.ninst() > 1) b += blk((T.n / 64 + T.ninst()) * (int64_t)sizeof(KItem));
  return b;
}

// Device bytes of the low-rank plans build_plans makes for T's sampled
// levels (both orientations; every prefix of levels when `prefixes`), from
// the same loops without building them, each list rounded as the block cache
// rounds it.
static int64_t plan_bytes(const Tree &T, int64_t kmax, int32_t seg, bool prefixes) {
  auto blk = [](int64_t b) { return (std::max<int64_t>(b, 64) + 255) / 256 * 256; };
  std::vector<int> levels;
  for (int l = 1; l < T.nlev(); ++l)
    if (!T.graphs[l].pa.empty()) levels.push_back(l);
  const int nlv = (int)levels.size();
  const int64_t per_group = std::max<int64_t>(1, 128 / std::max<int64_t>(1, kmax));
  int64_t bytes = 0;
  for (int o = 0; o < 2; ++o) {
    const bool trans = o == 1;
    int64_t nitems = 0, npps = 0, nred = 0;
    std::vector<std::vector<int32_t>> cnt(nlv);  // pairs per row box
    for (int li = 0; li < nlv; ++li) {
      const Graph &G = T.graphs[levels[li]];
      const Level &Lev = T.lev[levels[li]];
      const std::vector<int32_t> &colbox = trans ? G.pa : G.pb;
      std::vector<int64_t> per(Lev.nbox(), 0);
      for (int32_t b : colbox) per[b]++;
      for (int b = 0; b < Lev.nbox(); ++b) {
        const int64_t m = Lev.start[b + 1] - Lev.start[b];
        if (!per[b] || m <= 0) continue;
        const int64_t nsg = seg > 0 ? (m + seg - 1) / seg : 1;
        nitems += (per[b] + per_group - 1) / per_group * nsg;
        npps += per[b] * nsg;
        if (nsg > 1) nred += per[b];
      }
      cnt[li].assign(Lev.nbox(), 0);
      for (int32_t a : trans ? G.pb : G.pa) cnt[li][a]++;
    }
    bytes += blk(nitems * (int64_t)sizeof(ProjItem)) + blk(npps * (int64_t)sizeof(ProjPair)) +
             blk(nred * (int64_t)sizeof(ReduceItem));
    for (int le = prefixes ? 1 : std::max(nlv, 1); le <= nlv; ++le) {
      const int fl = levels[le - 1];
      const Level &F = T.lev[fl];
      int64_t nch = 0, nen = 0;
      for (int b = 0; b < F.nbox(); ++b) {
        int box = b, lvl = fl;
        int64_t per_chunk = 0;
        for (int li = le - 1; li >= 0; --li) {
          while (lvl > levels[li]) box = T.lev[lvl--].parent[box];
          per_chunk += cnt[li][box];
        }
        const int64_t chunks = (F.start[b + 1] - F.start[b] + 63) / 64;
        if (per_chunk > 0) {
          nch += chunks;
          nen += chunks * per_chunk;
        }
      }
      bytes += blk(nch * (int64_t)sizeof(ExpandChunk)) + blk(nen * (int64_t)sizeof(ExpandEntry));
    }
  }
  return bytes;
}

// Device bytes of the other work lists of a compression of T: the leaf near
// field's plans (both orientations), the per-level job lists of the
// recovery and its color-activity table, the leaf pass lists, and for H^2
// the pass lists (upward and downward sums of every level, the long bases
// and their 64-row chunks for the full operator and every level-truncated
// one); upper bounds where a list's length depends on ranks.
static int64_t list_bytes(const Tree &T, const hm_compress_opts &o) {
  auto blk = [](int64_t b) { return (std::max<int64_t>(b, 64) + 255) / 256 * 256; };
  const Graph &GL = T.leaf_graph();
  const Level &LL = T.lev[T.L()];
  int64_t b = 0;
  {
    int64_t nch = 0, nen = 0;
    std::vector<int64_t> cols(LL.nbox(), 0);
    for (size_t q = 0; q < GL.pa.size(); ++q) cols[GL.pa[q]] += (T.box_size(T.L(), GL.pb[q]) + 127) / 128;
    for (int a = 0; a < LL.nbox(); ++a) {
      if (!cols[a]) continue;
      const int64_t chunks = (T.box_size(T.L(), a) + 63) / 64;
      nch += chunks;
      nen += chunks * cols[a];
    }
    b += 2 * (blk(nch * (int64_t)sizeof(ExpandChunk)) + blk(nen * (int64_t)sizeof(NearEntry)));
    const int64_t npl = (int64_t)GL.pa.size();
    b += 2 * blk(GL.nv() * 4) + blk((int64_t)LL.nbox() * GL.ncolors) + 3 * blk(npl * 8) +
         2 * blk(npl * 4) + (T.ninst() > 1 ? blk((T.n / 64 + T.ninst()) * (int64_t)sizeof(KItem)) : 0);
  }
  int64_t nb = 0, np = 0, nlv = 0;
  for (int l = 1; l < T.nlev(); ++l) {
    const Graph &G = T.graphs[l];
    if (G.pa.empty()) continue;
    const int64_t npl = (int64_t)G.pa.size(), nbl = T.lev[l].nbox();
    b += 2 * blk(npl * (int64_t)sizeof(QrJob)) + blk(npl * (int64_t)sizeof(CoreJob)) +
         blk(npl * 4) + blk(nbl * G.ncolors) +
         (T.ninst() > 1 ? blk((T.n / 64 + T.ninst()) * (int64_t)sizeof(KItem)) : 0);
    if (o.format != HM_FORMAT_H1) {
      // the shared-basis formats' lists (build_uniform_graphs ran): stage-1
      // activity and QR jobs, stage-2 slots, basis offsets, the combination
      // jobs (256-row pieces) and terms, the coupling jobs; H^2 adds the
      // norm jobs, the augmentation jobs, the transfers and the nesting
      const int64_t pieces = nbl + T.n / 256 + 1;
      b += blk(nbl * std::max(T.ugraphs[l].ncolors, 1)) + 3 * blk(nbl * (int64_t)sizeof(QrJob)) +
           blk(nbl * std::max(G.ncolors, 1) * 4) + blk(nbl * 8) +
           blk(pieces * (int64_t)sizeof(MixJob)) + blk(npl * (int64_t)sizeof(MixTerm)) +
           blk(npl * (int64_t)sizeof(UCJob));
      if (o.format == HM_FORMAT_H2)
        b += 2 * blk(pieces * (int64_t)sizeof(AugJob)) + blk(nbl * (int64_t)sizeof(TransferJob)) +
             blk(nbl * (int64_t)sizeof(NestJob));
      if (T.ninst() > 1) b += 2 * blk((T.n / 64 + T.ninst()) * (int64_t)sizeof(KItem));
    }
    nb += nbl;
    np += npl;
    ++nlv;
  }
  if (o.format == HM_FORMAT_H2) {
    const int64_t rec = (nb + T.n / 64 + nb) * (int64_t)sizeof(H2Leaf);
    b += nlv * (3 * blk(nb * (int64_t)sizeof(H2Sum)) + 3 * blk((np + 2 * nb) * (int64_t)sizeof(H2Term)));
    b += (nlv + 1) * 2 * blk(rec);
  }
  return b + 4096;
}

// Peak device bytes of one compression of T with a black box in tree order
// (factor pools at the largest rank, sample and scratch buffers, plans and
// work lists, and T's device copy when T has none on this device yet), from
// the same sizes compress_impl allocates; the server's admission estimate.
int64_t compress_footprint(Tree &T, const hm_compress_opts &o) {
  const int p = o.oversample > 0 ? o.oversample : 10;
  const int kfix = o.rank > 0 ? o.rank : 0;
  const int r = o.r > 0 ? o.r : (kfix > 0 ? kfix + p : 0);
  if (r <= 0) return 0;
  const int64_t kmax = kfix > 0 ? std::min(kfix, r) : r - p;
  const bool mixed = o.prec == HM_PREC_MIXED;
  const int64_t es = mixed ? 4 : 8;
  const int64_t n = T.n;
  const bool uniform = o.format != HM_FORMAT_H1, h2 = o.format == HM_FORMAT_H2;
  if (uniform) build_uniform_graphs(T);
  int64_t szU = 0, szV = 0, np = 0, nb = 0, nlv = 0, cmax = 0, wmax = 0, cmax_np = 0;
  int64_t w1 = 0, w2 = 0;  // shared-basis formats: widest stage-1 and stage-2 samples
  for (int l = 1; l < T.nlev(); ++l) {
    const Graph &G = T.graphs[l];
    if (G.pa.empty()) continue;
    const Level &Lv = T.lev[l];
    int64_t rows = 0;
    for (size_t q = 0; q < G.pa.size(); ++q) {
      const int64_t ma = Lv.start[G.pa[q] + 1] - Lv.start[G.pa[q]];
      const int64_t mb = Lv.start[G.pb[q] + 1] - Lv.start[G.pb[q]];
      szU += ma * kmax;
      szV += mb * kmax;
      rows += ma + mb;
    }
    np += (int64_t)G.pa.size();
    nb += Lv.nbox();
    ++nlv;
    cmax = std::max<int64_t>(cmax, pad16((int64_t)G.ncolors * r));
    wmax = std::max(wmax, rows * r);
    cmax_np = std::max<int64_t>(cmax_np, (int64_t)G.pa.size());
    if (uniform) {
      w1 = std::max(w1, pad16((int64_t)T.ugraphs[l].ncolors * r));
      w2 = std::max(w2, pad16((int64_t)G.ncolors * kmax));
    }
  }
  const Graph &GL = T.leaf_graph();
  int64_t szD = 0;
  for (size_t q = 0; q < GL.pa.size(); ++q)
    szD += T.box_size(T.L(), GL.pa[q]) * T.box_size(T.L(), GL.pb[q]);
  const int64_t leaf_cols = pad16((int64_t)GL.ncolors * T.leaf_width());
  // factor pools: per-pair bases, their products and FP32 copies (not kept
  // by H^2), couplings, leaf blocks, ranks, permutation
  const int64_t pools = (h2 ? 0 : szU * (8 + 8 + 4) + szV * (8 + 4)) + np * kmax * kmax * 8 +
                        szD * 8 + np * 8 + n * 8;
  // the two sample buffers (the shared-basis formats' stage 2 in FP64) and
  // the peel's partial projections: one slot per pair and sample column,
  // capped (H^2 peels through its passes and keeps no slots)
  int64_t wcols = std::max<int64_t>(2 * cmax, leaf_cols), xbytes = n * wcols * es, tes = es;
  if (uniform) {
    w1 = std::max(w1, leaf_cols);
    xbytes = std::max(n * w1 * es, n * w2 * 8);
    wcols = std::max(w1, w2);
    tes = 8;
  }
  const int64_t slots = h2 ? 0 : np;
  const int64_t tcap = std::max(std::min<int64_t>(slots * kmax * std::max<int64_t>(wcols, 1), kTScratchCap),
                                std::max<int64_t>(slots * kmax * 64, 64));
  const int64_t tflags = tcap / std::max<int64_t>(kmax * kLowRankTile, 1) + slots + 64;
  int64_t work = std::max<int64_t>(wmax, 1) * 8;
  if (h2) work = std::max(work, n * r * 8);
  const int64_t scratch = 2 * xbytes + tcap * tes + tflags + work +
                          2 * std::max<int64_t>(cmax_np, 1) * r * r * 8 + 2 * np * 4 + 64 +
                          (mixed ? 2 * cmax_np * 8 : 0) + nlv * 4;
  int64_t uni = 0;
  if (h2) {
    // per level: implied bases U and V (a level's boxes cover at most n
    // rows), singular values and transfers of every box; basis ranks and
    // saturation flags; the augmented sample; the expansion scratch of the
    // peel (two nb x kmax x h2cols blocks, capped at 64 MB each, and the
    // chunk partials: at most one 64-row chunk per box plus n / 64)
    for (int l = 1; l < T.nlev(); ++l)
      if (!T.graphs[l].pa.empty())
        uni += 2 * n * kmax * 8 + 2 * T.lev[l].nbox() * (kmax + kmax * kmax) * 8;
    uni += 16 * nb + n * r * 8 + (mixed ? nb * 8 : 0);
    const int64_t h2cols = std::min<int64_t>(
        256, std::max<int64_t>(16, (int64_t(64) << 20) / std::max<int64_t>(nb * kmax * 8, 1)));
    uni += 2 * nb * kmax * h2cols * 8 + (nb + n / 64 + 1) * kmax * h2cols * 8;
  } else if (uniform) {
    // shared bases U and V of every level, their ranks and saturation
    // flags, the combination buffer
    uni += nlv * 2 * n * kmax * 8 + 16 * nb + n * kmax * 8;
  }
  const int64_t plans =
      (h2 ? 0 : plan_bytes(T, kmax, kSeg, false) + plan_bytes(T, kmax, 0, true)) + list_bytes(T, o);
  int dev = -1;
  const int64_t tree = T.dev && hipGetDevice(&dev) == hipSuccess && T.dev->device == dev
                           ? 0
                           : tree_device_bytes(T);
  return pools + scratch + plans + uni + tree;
}

// Device bytes of one hm_matvec call (scratch and order conversion).
int64_t matvec_footprint(const hm_hmatrix *H, int64_t nrhs, int dtype) {
  const int64_t es = dtype == HM_F32 ? 4 : 8;
  int64_t b = tscratch_elems(*H, nrhs) * es + 2 * H->n * nrhs * es;
  if (H->format == HM_FORMAT_H2 && H->h2a.ready) {
    // the passes' expansions (h2_apply's own scratch, 256 columns at a time)
    const int64_t cw = std::min<int64_t>(std::max<int64_t>(nrhs, 1), 256);
    b += (2 * H->nvtot + H->h2a.nchunk) * H->kmax * cw * 8;
  }
  return b;
}

// Frees the idle blocks the block cache keeps for device dev.
void trim_block_cache(int dev) {
  if (dev >= 0 && dev < 64) cache_drop(dev);
}

}  // namespace hm

// ------------------------------------------------------------------ plans
// A compression whose device pipeline is captured once into a HIP graph and
// replayed: every execution draws the same test matrices, applies the black
// box again and recovers a new H-matrix into the same buffers.
struct hm_plan {
  std::unique_ptr<hm::Compression> C;
  hipStream_t cs = nullptr;  // capture stream (the null stream cannot be captured)
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  int64_t nodes = 0;
  ~hm_plan() {
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

// ================================================================== C ABI
using namespace hm;

#define API_BEGIN try {
#define API_END                                              \
  }                                                          \
  catch (const hm::Error &e) {                               \
    return fail(e.code, e.msg);                              \
  }                                                          \
  catch (const std::bad_alloc &) {                           \
    return fail(HM_E_NOMEM, "host allocation failed");       \
  }                                                          \
  catch (const std::exception &e) {                          \
    return fail(HM_E_ARG, e.what());                         \
  }

namespace hm {
namespace {
struct IdleRelease {
  IdleRelease() { release_idle() = true; }
  ~IdleRelease() { release_idle() = false; }
};
}  // namespace
void free_idle(hm_hmatrix *H) {
  IdleRelease g;
  delete H;
}
void free_idle(hm_tree *T) {
  IdleRelease g;
  delete T;
}
}  // namespace hm

extern "C" {

const char *hm_last_error(void) { return g_last_error.c_str(); }

const char *hm_autotune_table(void) {
  static thread_local std::string snap;
  snap = autotune_report();
  return snap.c_str();
}

hm_status hm_build_tree(const double *points, int64_t n, int dim, int leaf_size, int tree_kind,
                        int adm, hm_tree **out) {
  API_BEGIN
  if (!points || !out || n <= 0 || dim < 1 || dim > 8 || leaf_size < 1)
    return fail(HM_E_ARG, "hm_build_tree: bad argument");
  if (tree_kind != HM_TREE_GEOMETRIC && tree_kind != HM_TREE_INDEX_BINARY)
    return fail(HM_E_ARG, "hm_build_tree: bad tree kind");
  if (adm != HM_ADM_STRONG && adm != HM_ADM_WEAK) return fail(HM_E_ARG, "hm_build_tree: bad adm");
  if (tree_kind == HM_TREE_INDEX_BINARY && adm != HM_ADM_WEAK)
    return fail(HM_E_ARG, "hm_build_tree: the index-halving tree needs weak admissibility");
  for (int64_t i = 0; i < n * dim; ++i)
    if (!std::isfinite(points[i])) return fail(HM_E_ARG, "hm_build_tree: non-finite point");
  auto t = std::make_unique<hm_tree>();
  hm_status st = build_tree(points, n, dim, leaf_size, tree_kind, adm, t->t);
  if (st != HM_OK) return st;
  *out = t.release();
  return HM_OK;
  API_END
}

hm_status hm_build_forest(const double *points, const int64_t *counts, int32_t ninst, int dim,
                          int leaf_size, int tree_kind, int adm, hm_tree **out) {
  API_BEGIN
  if (!points || !counts || !out || ninst < 1 || dim < 1 || dim > 8 || leaf_size < 1)
    return fail(HM_E_ARG, "hm_build_forest: bad argument");
  if (tree_kind != HM_TREE_GEOMETRIC && tree_kind != HM_TREE_INDEX_BINARY)
    return fail(HM_E_ARG, "hm_build_forest: bad tree kind");
  if (adm != HM_ADM_STRONG && adm != HM_ADM_WEAK) return fail(HM_E_ARG, "hm_build_forest: bad adm");
  if (tree_kind == HM_TREE_INDEX_BINARY && adm != HM_ADM_WEAK)
    return fail(HM_E_ARG, "hm_build_forest: the index-halving tree needs weak admissibility");
  int64_t n = 0;
  for (int32_t i = 0; i < ninst; ++i) {
    if (counts[i] < 1) return fail(HM_E_ARG, "hm_build_forest: empty instance");
    n += counts[i];
  }
  if (n > INT32_MAX) return fail(HM_E_ARG, "hm_build_forest: more than 2^31 - 1 points");
  for (int64_t i = 0; i < n * dim; ++i)
    if (!std::isfinite(points[i])) return fail(HM_E_ARG, "hm_build_forest: non-finite point");
  auto t = std::make_unique<hm_tree>();
  hm_status st = build_forest(points, counts, ninst, dim, leaf_size, tree_kind, adm, t->t);
  if (st != HM_OK) return st;
  *out = t.release();
  return HM_OK;
  API_END
}

hm_status hm_tree_instances(const hm_tree *tree, int32_t *ninst, int64_t *offsets) {
  if (!tree || !ninst) return fail(HM_E_ARG, "null argument");
  *ninst = tree->t.ninst();
  if (offsets) {
    if (tree->t.inst_off.empty()) {
      offsets[0] = 0;
      offsets[1] = tree->t.n;
    } else {
      std::memcpy(offsets, tree->t.inst_off.data(), tree->t.inst_off.size() * 8);
    }
  }
  return HM_OK;
}

void hm_tree_free(hm_tree *tree) { delete tree; }

hm_status hm_tree_info(const hm_tree *tree, int32_t *nlevels, int64_t *n, int32_t *dim) {
  if (!tree) return fail(HM_E_ARG, "null tree");
  if (nlevels) *nlevels = tree->t.nlev();
  if (n) *n = tree->t.n;
  if (dim) *dim = tree->t.dim;
  return HM_OK;
}

hm_status hm_tree_perm(const hm_tree *tree, int64_t *perm) {
  if (!tree || !perm) return fail(HM_E_ARG, "null argument");
  std::memcpy(perm, tree->t.perm.data(), tree->t.n * sizeof(int64_t));
  return HM_OK;
}

hm_status hm_tree_level(const hm_tree *tree, int level, int32_t *nbox, int64_t *start,
                        int32_t *parent, int64_t *org, int32_t *blev) {
  if (!tree || level < 0 || level >= tree->t.nlev()) return fail(HM_E_ARG, "bad level");
  const Level &Lv = tree->t.lev[level];
  if (nbox) *nbox = Lv.nbox();
  if (start) std::memcpy(start, Lv.start.data(), Lv.start.size() * 8);
  if (parent) std::memcpy(parent, Lv.parent.data(), Lv.parent.size() * 4);
  if (org) std::memcpy(org, Lv.org.data(), Lv.org.size() * 8);
  if (blev) std::memcpy(blev, Lv.blev.data(), Lv.blev.size() * 4);
  return HM_OK;
}

hm_status hm_tree_list(const hm_tree *tree, int level, int which, int64_t *nnz, int32_t *ptr,
                       int32_t *idx) {
  if (!tree || level < 0 || level >= tree->t.nlev()) return fail(HM_E_ARG, "bad level");
  if (which != HM_LIST_NEIGHBOR && which != HM_LIST_INTERACTION) return fail(HM_E_ARG, "bad list");
  const Level &Lv = tree->t.lev[level];
  const std::vector<int32_t> &p = which == HM_LIST_NEIGHBOR ? Lv.nei_ptr : Lv.int_ptr;
  const std::vector<int32_t> &x = which == HM_LIST_NEIGHBOR ? Lv.nei : Lv.intl;
  if (nnz) *nnz = (int64_t)x.size();
  if (ptr) std::memcpy(ptr, p.data(), p.size() * 4);
  if (idx) std::memcpy(idx, x.data(), x.size() * 4);
  return HM_OK;
}

static const Graph *graph_of(const hm_tree *tree, int level) {
  if (!tree) return nullptr;
  if (level == -1) return &tree->t.leaf_graph();
  if (level < 0 || level >= tree->t.nlev()) return nullptr;
  return &tree->t.graphs[level];
}

hm_status hm_incompat_graph(const hm_tree *tree, int level, int64_t *nv, int64_t *nadj,
                            const int64_t **xadj, const int32_t **adj, const int32_t **vbox,
                            int64_t *npairs, const int32_t **pair_a, const int32_t **pair_b,
                            const int32_t **pair_v) {
  const Graph *G = graph_of(tree, level);
  if (!G) return fail(HM_E_ARG, "bad level");
  if (nv) *nv = G->nv();
  if (nadj) *nadj = (int64_t)G->adj.size();
  if (xadj) *xadj = G->xadj.data();
  if (adj) *adj = G->adj.data();
  if (vbox) *vbox = G->vbox.data();
  if (npairs) *npairs = (int64_t)G->pa.size();
  if (pair_a) *pair_a = G->pa.data();
  if (pair_b) *pair_b = G->pb.data();
  if (pair_v) *pair_v = G->pv.data();
  return HM_OK;
}

hm_status hm_uniform_graph(hm_tree *tree, int level, int64_t *nv, int64_t *nadj,
                           const int64_t **xadj, const int32_t **adj, const int32_t **vbox,
                           int32_t *ncolors, const int32_t **color) {
  API_BEGIN
  if (!tree || level < 0 || level >= tree->t.nlev()) return fail(HM_E_ARG, "bad level");
  build_uniform_graphs(tree->t);
  const Graph &G = tree->t.ugraphs[level];
  if (nv) *nv = G.nv();
  if (nadj) *nadj = (int64_t)G.adj.size();
  if (xadj) *xadj = G.xadj.data();
  if (adj) *adj = G.adj.data();
  if (vbox) *vbox = G.vbox.data();
  if (ncolors) *ncolors = G.ncolors;
  if (color) *color = G.color.data();
  return HM_OK;
  API_END
}

hm_status hm_color(int64_t nv, const int64_t *xadj, const int32_t *adj, int32_t *color,
                   int32_t *ncolors) {
  API_BEGIN
  if (nv < 0 || (nv > 0 && (!xadj || !color))) return fail(HM_E_ARG, "hm_color: bad argument");
  if (nv > 0 && xadj[nv] > 0 && !adj) return fail(HM_E_ARG, "hm_color: null adjacency");
  for (int64_t v = 0; v < nv; ++v)
    for (int64_t t = xadj[v]; t < xadj[v + 1]; ++t)
      if (adj[t] < 0 || adj[t] >= nv || adj[t] == v) return fail(HM_E_ARG, "hm_color: bad edge");
  const int32_t nc = dsatur(nv, xadj, adj, color);
  if (ncolors) *ncolors = nc;
  return HM_OK;
  API_END
}

hm_status hm_tree_color(hm_tree *tree) {
  API_BEGIN
  if (!tree) return fail(HM_E_ARG, "null tree");
  Tree &T = tree->t;
  // One DSatur run per (graph, instance): the instances of a forest are
  // disconnected components, and DSatur restricted to one component takes
  // the same choices as on the whole graph (saturation and degree are
  // component-local, ties go to the lower id, which keeps its order), so
  // coloring them apart gives the same colors.  Large jobs run on a pool.
  struct Job {
    Graph *G;
    int64_t v0, v1;
  };
  std::vector<Job> jobs;
  int64_t total = 0;
  for (size_t g = 0; g < T.graphs.size(); ++g) {
    Graph &G = T.graphs[g];
    G.color.assign(G.nv(), 0);
    G.ncolors = 0;
    for (int i = 0; i < T.ninst(); ++i) {
      const int64_t v0 = T.gvoff[g][i], v1 = T.gvoff[g][i + 1];
      if (v1 > v0) {
        jobs.push_back(Job{&G, v0, v1});
        total += G.xadj[v1] - G.xadj[v0];
      }
    }
  }
  std::vector<int32_t> ncol(jobs.size(), 0);
  auto run = [&](size_t j) {
    const Job &J = jobs[j];
    const Graph &G = *J.G;
    const int64_t nv = J.v1 - J.v0;
    if (J.v0 == 0) {
      ncol[j] = dsatur(nv, G.xadj.data(), G.adj.data(), J.G->color.data());
      return;
    }
    std::vector<int64_t> xa(nv + 1);
    for (int64_t v = 0; v <= nv; ++v) xa[v] = G.xadj[J.v0 + v] - G.xadj[J.v0];
    std::vector<int32_t> ad(G.adj.begin() + G.xadj[J.v0], G.adj.begin() + G.xadj[J.v1]);
    for (int32_t &u : ad) u -= (int32_t)J.v0;
    ncol[j] = dsatur(nv, xa.data(), ad.data(), J.G->color.data() + J.v0);
  };
  if (total < (int64_t(1) << 20) || jobs.size() == 1) {
    for (size_t j = 0; j < jobs.size(); ++j) run(j);
  } else {
    std::vector<size_t> order(jobs.size());
    for (size_t j = 0; j < jobs.size(); ++j) order[j] = j;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
      return jobs[a].G->xadj[jobs[a].v1] - jobs[a].G->xadj[jobs[a].v0] >
             jobs[b].G->xadj[jobs[b].v1] - jobs[b].G->xadj[jobs[b].v0];
    });
    std::atomic<size_t> next{0};
    const int nth = std::max(1, std::min<int>((int)jobs.size(), host_threads()));
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&] {
        for (size_t q = next++; q < order.size(); q = next++) run(order[q]);
      });
    for (auto &t : th) t.join();
  }
  for (size_t j = 0; j < jobs.size(); ++j)
    jobs[j].G->ncolors = std::max(jobs[j].G->ncolors, ncol[j]);
  for (Graph &G : T.graphs) G.colored = true;
  return HM_OK;
  API_END
}

hm_status hm_tree_set_colors(hm_tree *tree, int level, const int32_t *color) {
  API_BEGIN
  Graph *G = const_cast<Graph *>(graph_of(tree, level));
  if (!G || (!color && G->nv() > 0)) return fail(HM_E_ARG, "bad argument");
  int32_t nc = 0;
  for (int64_t v = 0; v < G->nv(); ++v) {
    if (color[v] < 0) return fail(HM_E_ARG, "negative color");
    nc = std::max(nc, color[v] + 1);
    for (int64_t t = G->xadj[v]; t < G->xadj[v + 1]; ++t)
      if (color[G->adj[t]] == color[v]) return fail(HM_E_ARG, "coloring is not valid");
  }
  G->color.assign(color, color + G->nv());
  G->ncolors = nc;
  G->colored = true;
  return HM_OK;
  API_END
}

hm_status hm_tree_colors(const hm_tree *tree, int level, int32_t *ncolors, const int32_t **color) {
  const Graph *G = graph_of(tree, level);
  if (!G) return fail(HM_E_ARG, "bad level");
  if (!G->colored) return fail(HM_E_STATE, "graph not colored");
  if (ncolors) *ncolors = G->ncolors;
  if (color) *color = G->color.data();
  return HM_OK;
}

hm_status hm_kernel_blackbox(hm_tree *tree, int kernel, hm_blackbox *out) {
  API_BEGIN
  if (!tree || !out) return fail(HM_E_ARG, "null argument");
  if (kernel != HM_KERNEL_LOG && kernel != HM_KERNEL_INV_R) return fail(HM_E_ARG, "bad kernel");
  if (tree->t.dim > 3) return fail(HM_E_ARG, "the kernel black box takes 1 to 3 dimensions");
  auto k = std::make_shared<KernelBB>();
  k->tree = &tree->t;
  k->kernel = kernel;
  tree->t.keep.push_back(k);
  out->apply = kernel_bb_apply;
  out->ctx = k.get();
  out->order = HM_ORDER_TREE;
  out->symmetric = 1;
  out->dtypes = (1 << HM_F64) | (1 << HM_F32);
  device_tree(tree->t, nullptr);
  return HM_OK;
  API_END
}

hm_status hm_mfma_rate(int dtype, void *stream, double *tflops) {
  API_BEGIN
  if (!tflops || (dtype != HM_F64 && dtype != HM_F32)) return fail(HM_E_ARG, "hm_mfma_rate: bad argument");
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  try {
    *tflops = hm::measure_mfma_rate(dtype == HM_F32, cus, (hipStream_t)stream);
  } catch (const std::runtime_error &e) {
    return fail(HM_E_DEVICE, e.what());
  }
  return HM_OK;
  API_END
}

hm_status hm_kernel_apply(hm_tree *tree, int kernel, int64_t ncols, int dtype, const void *X,
                          int64_t ldx, void *Y, int64_t ldy, int order, void *stream) {
  API_BEGIN
  if (!tree || !X || !Y || ncols < 0 || ldx < tree->t.n || ldy < tree->t.n)
    return fail(HM_E_ARG, "hm_kernel_apply: bad argument");
  if (kernel != HM_KERNEL_LOG && kernel != HM_KERNEL_INV_R) return fail(HM_E_ARG, "bad kernel");
  if (dtype != HM_F64 && dtype != HM_F32) return fail(HM_E_ARG, "bad dtype");
  if (tree->t.dim > 3) return fail(HM_E_ARG, "the kernel apply takes 1 to 3 dimensions");
  hipStream_t s = (hipStream_t)stream;
  DeviceTree &D = device_tree(tree->t, s);
  const bool f32 = dtype == HM_F32;
  const int64_t n = tree->t.n;
  if (order == HM_ORDER_TREE) {
    kernel_apply_tree(tree->t, kernel, ncols, f32, X, ldx, Y, ldy, s);
    LAUNCH_CHECK();
    return HM_OK;
  }
  const size_t es = f32 ? 4 : 8;
  DBuf tx, ty;
  tx.alloc((size_t)n * std::max<int64_t>(ncols, 1) * es);
  ty.alloc((size_t)n * std::max<int64_t>(ncols, 1) * es);
  launch_permute_rows(n, ncols, D.perm.as<int64_t>(), false, f32, X, ldx, tx.p, n, s);
  kernel_apply_tree(tree->t, kernel, ncols, f32, tx.p, n, ty.p, n, s);
  launch_permute_rows(n, ncols, D.perm.as<int64_t>(), true, f32, ty.p, n, Y, ldy, s);
  LAUNCH_CHECK();
  HIP_TRY(hipStreamSynchronize(s));
  return HM_OK;
  API_END
}

hm_status hm_dense_blackbox(const double *A, int64_t n, int64_t lda, int order, hm_blackbox *out) {
  if (!A || !out || n <= 0 || lda < n) return fail(HM_E_ARG, "hm_dense_blackbox: bad argument");
  DenseBB *d = new (std::nothrow) DenseBB{A, n, lda};
  if (!d) return fail(HM_E_NOMEM, "host allocation failed");
  out->apply = dense_bb_apply;
  out->ctx = d;
  out->order = order == HM_ORDER_TREE ? HM_ORDER_TREE : HM_ORDER_ORIGINAL;
  out->symmetric = 0;
  out->dtypes = 1 << HM_F64;
  return HM_OK;
}

hm_status hm_hmatrix_blackbox(const hm_hmatrix *H, int order, hm_blackbox *out) {
  if (!H || !out) return fail(HM_E_ARG, "hm_hmatrix_blackbox: bad argument");
  HMatrixBB *b = new (std::nothrow) HMatrixBB{H, order == HM_ORDER_TREE ? HM_ORDER_TREE
                                                                       : HM_ORDER_ORIGINAL};
  if (!b) return fail(HM_E_NOMEM, "host allocation failed");
  out->apply = hmatrix_bb_apply;
  out->ctx = b;
  out->order = b->order;
  out->symmetric = 0;
  out->dtypes = (1 << HM_F64) | (1 << HM_F32);
  return HM_OK;
}

hm_status hm_product_blackbox(const hm_blackbox *A, const hm_blackbox *B, hm_blackbox *out) {
  if (!A || !B || !out || !A->apply || !B->apply)
    return fail(HM_E_ARG, "hm_product_blackbox: bad argument");
  if (A->order != B->order) return fail(HM_E_ARG, "the two black boxes take different orders");
  if (!(A->dtypes & B->dtypes)) return fail(HM_E_ARG, "the two black boxes share no dtype");
  ProductBB *p = new (std::nothrow) ProductBB{*A, *B};
  if (!p) return fail(HM_E_NOMEM, "host allocation failed");
  out->apply = product_bb_apply;
  out->ctx = p;
  out->order = A->order;
  // (A A)* = A A when A* = A
  out->symmetric = A->symmetric && B->symmetric && A->apply == B->apply && A->ctx == B->ctx;
  out->dtypes = A->dtypes & B->dtypes;
  return HM_OK;
}

void hm_blackbox_free(hm_blackbox *bb) {
  if (!bb) return;
  if (bb->apply == hmatrix_bb_apply)
    delete (HMatrixBB *)bb->ctx;
  else if (bb->apply == product_bb_apply)
    delete (ProductBB *)bb->ctx;
  else if (bb->apply == dense_bb_apply)
    delete (DenseBB *)bb->ctx;
  else
    return;  // the kernel black box belongs to its tree
  bb->ctx = nullptr;
}

void hm_dense_blackbox_free(hm_blackbox *bb) {
  if (bb && bb->apply == dense_bb_apply) {
    delete (DenseBB *)bb->ctx;
    bb->ctx = nullptr;
    bb->apply = nullptr;
  }
}

hm_status hm_compress(hm_tree *tree, const hm_blackbox *bb, const hm_compress_opts *opts,
                      void *stream, hm_hmatrix **out) {
  API_BEGIN
  if (!tree || !bb || !opts || !out) return fail(HM_E_ARG, "hm_compress: null argument");
  if (opts->max_retries < 0) return fail(HM_E_ARG, "hm_compress: max_retries < 0");
  // tolerance mode: a block whose rank reached r - p may be truncated above
  // the tolerance; retry with 8 more columns per test matrix, then report
  hm_compress_opts o = *opts;
  for (int attempt = 0;; ++attempt) {
    hm_hmatrix *H = nullptr;
    const hm_status st = compress_impl(tree->t, *bb, o, (hipStream_t)stream, &H);
    if (st != HM_OK) return st;
    const bool sat = o.rank <= 0 && H->stats.saturated > 0;
    const int r_used = H->stats.r;
    if (!sat || attempt >= o.max_retries || r_used + 8 > 64) {
      if (sat && (o.flags & HM_FLAG_STRICT)) {
        delete H;
        return fail(HM_E_SATURATED, "tolerance not reached within r - p columns");
      }
      H->stats.retries = attempt;
      *out = H;
      return HM_OK;
    }
    delete H;
    o.r = r_used + 8;
  }
  API_END
}

void hm_hmatrix_free(hm_hmatrix *H) { delete H; }

hm_status hm_compress_plan(hm_tree *tree, const hm_blackbox *bb, const hm_compress_opts *opts,
                           void *stream, hm_plan **out) {
  API_BEGIN
  if (!tree || !bb || !opts || !out) return fail(HM_E_ARG, "hm_compress_plan: null argument");
  hipStream_t s = (hipStream_t)stream;
  AllocScope scope(opts->allocator);
  auto P = std::make_unique<hm_plan>();
  P->C = std::make_unique<Compression>(tree->t, *bb, *opts);
  P->C->persistent = true;
  P->C->o.flags &= ~HM_FLAG_TIMING;
  hm_status st = P->C->setup(s);
  if (st != HM_OK) return st;
  // one eager run validates the pipeline and settles the autotuner, so the
  // captured launches are exactly the ones an eager compression makes
  Events ev;
  ev.s = s;
  P->C->record(s, ev);
  st = P->C->finalize(s, ev, std::chrono::steady_clock::now());
  if (st != HM_OK) return st;
  HIP_TRY(hipStreamCreateWithFlags(&P->cs, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(P->cs, hipStreamCaptureModeThreadLocal));
  try {
    ev.s = P->cs;
    P->C->record(P->cs, ev);
  } catch (...) {
    hipGraph_t bad = nullptr;
    (void)hipStreamEndCapture(P->cs, &bad);
    if (bad) (void)hipGraphDestroy(bad);
    (void)hipGetLastError();
    throw;
  }
  if (hipStreamEndCapture(P->cs, &P->g) != hipSuccess || !P->g) {
    (void)hipGetLastError();
    return fail(HM_E_DEVICE, "hm_compress_plan: the pipeline could not be captured "
                             "(the black box must only enqueue work on the given stream)");
  }
  HIP_TRY(hipGraphInstantiate(&P->ge, P->g, nullptr, nullptr, 0));
  size_t nn = 0;
  (void)hipGraphGetNodes(P->g, nullptr, &nn);
  P->nodes = (int64_t)nn;
  *out = P.release();
  return HM_OK;
  API_END
}

hm_status hm_plan_execute(hm_plan *plan, void *stream) {
  API_BEGIN
  if (!plan) return fail(HM_E_ARG, "null plan");
  hipStream_t s = (hipStream_t)stream;
  AllocScope scope(plan->C->o.allocator);
  const auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(hipGraphLaunch(plan->ge, s));
  Events ev;
  ev.s = s;
  return plan->C->finalize(s, ev, t0);
  API_END
}

hm_status hm_plan_hmatrix(const hm_plan *plan, const hm_hmatrix **H, int64_t *graph_nodes) {
  if (!plan) return fail(HM_E_ARG, "null plan");
  if (H) *H = plan->C->H.get();
  if (graph_nodes) *graph_nodes = plan->nodes;
  return HM_OK;
}

void hm_plan_free(hm_plan *plan) { delete plan; }

hm_status hm_matvec(const hm_hmatrix *H, int64_t nrhs, int dtype, const void *X, int64_t ldx,
                    void *Y, int64_t ldy, int order, void *stream) {
  return hm_matvec_op(H, 0, nrhs, dtype, X, ldx, Y, ldy, order, stream);
}

hm_status hm_matvec_op(const hm_hmatrix *H, int trans, int64_t nrhs, int dtype, const void *X,
                       int64_t ldx, void *Y, int64_t ldy, int order, void *stream) {
  API_BEGIN
  if (!H || !X || !Y || nrhs < 0 || ldx < H->n || ldy < H->n)
    return fail(HM_E_ARG, "hm_matvec: bad argument");
  if (dtype != HM_F64 && dtype != HM_F32) return fail(HM_E_ARG, "bad dtype");
  if (nrhs == 0) return HM_OK;
  matvec_impl(*H, trans != 0, nrhs, dtype == HM_F32, X, ldx, Y, ldy, order, (hipStream_t)stream);
  return HM_OK;
  API_END
}

// Scratch of hm_matvec_static, for callers that cannot allocate: a static
// device array, one copy per device from the code object's load until the
// process ends.  Host code reaches it only through the address
// hipGetSymbolAddress returns on each device (static_scratch_address).
static __device__ __align__(256) unsigned char scratch[HM_STATIC_SCRATCH_BYTES];

// The device address of `scratch` on the current device, looked up on the
// first call on that device (with it current) and kept.
static unsigned char *static_scratch_address() {
  static std::mutex mu;
  static unsigned char *addr[64] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    throw hm::Error{HM_E_DEVICE, "hm_matvec_static: no current device (or device id >= 64)"};
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw hm::Error{HM_E_DEVICE, std::string("hm_matvec_static: hipGetSymbolAddress: ") +
                                       hipGetErrorString(e)};
    }
    addr[dev] = (unsigned char *)p;
  }
  return addr[dev];
}

hm_status hm_matvec_static(const hm_hmatrix *H, int trans, int64_t nrhs, int dtype, const void *X,
                           int64_t ldx, void *Y, int64_t ldy, int order, void *stream) {
  API_BEGIN
  if (!H || !X || !Y || nrhs < 0 || ldx < H->n || ldy < H->n)
    return fail(HM_E_ARG, "hm_matvec_static: bad argument");
  if (dtype != HM_F64 && dtype != HM_F32) return fail(HM_E_ARG, "bad dtype");
  if (nrhs == 0) return HM_OK;
  unsigned char *buf = static_scratch_address();
  matvec_in(*H, trans != 0, nrhs, dtype == HM_F32, X, ldx, Y, ldy, order, buf,
            HM_STATIC_SCRATCH_BYTES, (hipStream_t)stream);
  return HM_OK;
  API_END
}

hm_status hm_test_matrix(const hm_tree *tree, int level, int pass, int32_t r, uint64_t seed,
                         int dtype, void *out, int64_t ld, void *stream) {
  API_BEGIN
  if (!tree || !out || level < 0 || level >= tree->t.nlev() || r <= 0 || ld < tree->t.n ||
      pass < 0 || pass > 2 || (dtype != HM_F64 && dtype != HM_F32))
    return fail(HM_E_ARG, "hm_test_matrix: bad argument");
  Tree &T = const_cast<Tree &>(tree->t);
  if (pass == 2) build_uniform_graphs(T);
  const Graph &G = pass == 2 ? T.ugraphs[level] : T.graphs[level];
  if (!G.colored && G.nv() > 0) return fail(HM_E_STATE, "graph not colored");
  hipStream_t s = (hipStream_t)stream;
  DeviceTree &D = device_tree(T, s);
  const Level &Lv = T.lev[level];
  std::vector<uint8_t> act((size_t)Lv.nbox() * std::max(G.ncolors, 1), 0);
  for (int64_t v = 0; v < G.nv(); ++v) {
    if (pass == 2) {  // uniform stage 1: Gaussian on the vertex box's interaction list
      const int a = G.vbox[v];
      for (int32_t t = Lv.int_ptr[a]; t < Lv.int_ptr[a + 1]; ++t)
        act[(size_t)Lv.intl[t] * G.ncolors + G.color[v]] = 1;
    } else {
      act[(size_t)G.vbox[v] * G.ncolors + G.color[v]] = 1;
    }
  }
  DBuf dact;
  upload(dact, act, s);
  launch_testmat(tree->t.n, D.rowbox[level].as<int32_t>(), dact.as<uint8_t>(), G.ncolors, r,
                 level, pass, seed, D.inst_off.as<int64_t>(), tree->t.ninst(), dtype == HM_F32,
                 out, ld, (int64_t)G.ncolors * r, s);
  LAUNCH_CHECK();
  HIP_TRY(hipStreamSynchronize(s));
  return HM_OK;
  API_END
}

hm_status hm_philox4x32_10(const uint32_t *ctr, int64_t count, uint32_t key0, uint32_t key1,
                           uint32_t *out, void *stream) {
  API_BEGIN
  if (!ctr || !out || count < 0) return fail(HM_E_ARG, "bad argument");
  launch_philox_raw(ctr, count, key0, key1, out, (hipStream_t)stream);
  LAUNCH_CHECK();
  return HM_OK;
  API_END
}

hm_status hm_compress_footprint(hm_tree *tree, const hm_compress_opts *opts, int64_t *bytes) {
  API_BEGIN
  if (!tree || !opts || !bytes) return fail(HM_E_ARG, "hm_compress_footprint: null argument");
  for (const Graph &G : tree->t.graphs)
    if (!G.colored && G.nv() > 0) return fail(HM_E_STATE, "tree is not colored (hm_tree_color)");
  const int p = opts->oversample > 0 ? opts->oversample : 10;
  const int r = opts->r > 0 ? opts->r : (opts->rank > 0 ? opts->rank + p : 0);
  if (r <= 0 || r > 64) return fail(HM_E_ARG, "hm_compress_footprint: r must be in 1..64");
  if (opts->format != HM_FORMAT_H1 && opts->format != HM_FORMAT_UNIFORM_H1 &&
      opts->format != HM_FORMAT_H2)
    return fail(HM_E_ARG, "hm_compress_footprint: unknown format");
  *bytes = hm::compress_footprint(tree->t, *opts);
  return HM_OK;
  API_END
}

hm_status hm_matvec_footprint(const hm_hmatrix *H, int64_t nrhs, int dtype, int64_t *bytes) {
  if (!H || !bytes || nrhs < 0 || (dtype != HM_F64 && dtype != HM_F32))
    return fail(HM_E_ARG, "hm_matvec_footprint: bad argument");
  *bytes = hm::matvec_footprint(H, nrhs, dtype);
  return HM_OK;
}

hm_status hm_hmatrix_stats(const hm_hmatrix *H, hm_stats *out) {
  if (!H || !out) return fail(HM_E_ARG, "null argument");
  *out = H->stats;
  out->device_bytes = hm::hmatrix_device_bytes(H);
  return HM_OK;
}

hm_status hm_hmatrix_export_level(const hm_hmatrix *H, int level, int64_t *npairs,
                                  int32_t *pair_a, int32_t *pair_b, int32_t *rank_u,
                                  int32_t *rank_v, int64_t *size_u, int64_t *size_b,
                                  int64_t *size_v, double *U, double *B, double *V) {
  API_BEGIN
  if (!H) return fail(HM_E_ARG, "null H");
  const hm_hmatrix::Lv *L = nullptr;
  for (const auto &x : H->lv)
    if (x.level == level) L = &x;
  if (!L) {
    if (npairs) *npairs = 0;
    if (size_u) *size_u = 0;
    if (size_b) *size_b = 0;
    if (size_v) *size_v = 0;
    return HM_OK;
  }
  const std::vector<int64_t> &st = H->start[level];
  int64_t su = 0, sb = 0, sv = 0;
  for (int64_t q = 0; q < L->np; ++q) {
    const int ku = H->h_ranks[L->g0 + q], kv = H->h_ranks[H->np_total + L->g0 + q];
    su += (st[L->pa[q] + 1] - st[L->pa[q]]) * ku;
    sb += (int64_t)ku * kv;
    sv += (st[L->pb[q] + 1] - st[L->pb[q]]) * kv;
  }
  if (npairs) *npairs = L->np;
  if (size_u) *size_u = su;
  if (size_b) *size_b = sb;
  if (size_v) *size_v = sv;
  if (pair_a) std::memcpy(pair_a, L->pa.data(), L->np * 4);
  if (pair_b) std::memcpy(pair_b, L->pb.data(), L->np * 4);
  for (int64_t q = 0; q < L->np; ++q) {
    if (rank_u) rank_u[q] = H->h_ranks[L->g0 + q];
    if (rank_v) rank_v[q] = H->h_ranks[H->np_total + L->g0 + q];
  }
  if (U || B || V) {
    HIP_TRY(hipDeviceSynchronize());
    int64_t ou = 0, ob = 0, ov = 0;
    std::vector<double> bt((size_t)H->kmax * H->kmax);
    for (int64_t q = 0; q < L->np; ++q) {
      const int ku = H->h_ranks[L->g0 + q], kv = H->h_ranks[H->np_total + L->g0 + q];
      const int64_t ma = st[L->pa[q] + 1] - st[L->pa[q]];
      const int64_t mb = st[L->pb[q] + 1] - st[L->pb[q]];
      // H^2 keeps no pair copies: the boxes' bases (m x kmax, ld m) hold them
      const bool boxes = H->format == HM_FORMAT_H2;
      if (U && ku)
        HIP_TRY(hipMemcpy(U + ou, (boxes ? H->UB : H->U).as<double>() + L->offU[q], ma * ku * 8,
                          hipMemcpyDeviceToHost));
      if (V && kv)
        HIP_TRY(hipMemcpy(V + ov, (boxes ? H->VB : H->V).as<double>() + L->offV[q], mb * kv * 8,
                          hipMemcpyDeviceToHost));
      if (B && ku && kv) {
        HIP_TRY(hipMemcpy(bt.data(), H->B.as<double>() + L->offB[q], bt.size() * 8,
                          hipMemcpyDeviceToHost));
        for (int c = 0; c < kv; ++c)
          for (int t = 0; t < ku; ++t) B[ob + c * ku + t] = bt[(size_t)c * H->kmax + t];
      }
      ou += ma * ku;
      ob += (int64_t)ku * kv;
      ov += mb * kv;
    }
  }
  return HM_OK;
  API_END
}

hm_status hm_hmatrix_export_near(const hm_hmatrix *H, int64_t *npairs, int32_t *pair_a,
                                 int32_t *pair_b, int64_t *size, double *D) {
  API_BEGIN
  if (!H) return fail(HM_E_ARG, "null H");
  if (npairs) *npairs = (int64_t)H->na.size();
  const std::vector<int64_t> &st = H->start[H->nlev - 1];
  int64_t total = 0;
  for (size_t q = 0; q < H->na.size(); ++q)
    total += (st[H->na[q] + 1] - st[H->na[q]]) * (st[H->nb[q] + 1] - st[H->nb[q]]);
  if (size) *size = total;
  if (pair_a) std::memcpy(pair_a, H->na.data(), H->na.size() * 4);
  if (pair_b) std::memcpy(pair_b, H->nb.data(), H->nb.size() * 4);
  if (D && total) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(D, H->D.p, total * 8, hipMemcpyDeviceToHost));
  }
  return HM_OK;
  API_END
}

}  // extern "C"
