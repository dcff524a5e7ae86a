// Serving: a request loop that keeps compressed H-matrices resident on the
// GPU and runs compressions and H-matrix applies of different sizes side by
// side.
//
// Design (one GPU):
//   * nslots host workers, each with its own non-blocking HIP stream at the
//     default priority, so admitted requests overlap on the device;
//   * admission by device-memory footprint: a request starts only when its
//     bytes fit beside the resident H-matrices and the work in flight
//     (in_use + bytes <= budget); compressions reserve the footprint of
//     their own tree, computed on the host after the tree and its coloring
//     are built (no device work is needed for that);
//   * continuous batching: pending requests are scanned in arrival order and
//     every one that is ready is admitted as soon as a slot and memory free
//     up (an apply whose H-matrix is still being compressed waits; later
//     requests may pass it);
//   * at most compress_slots compressions run at once (default 1): each one
//     fills the whole GPU, so running several only stretches all of them,
//     while applies are short and slot into the gaps;
//   * scratch of a request is stream-ordered (hipMallocAsync / hipFreeAsync
//     on its stream), so finishing one request never waits for another.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hm_internal.h"

namespace hm {
namespace {

struct Req {
  int64_t id = 0;
  int kind = 0;  // 0 compress, 1 apply
  // compression
  std::vector<double> pts;
  int64_t n = 0;
  int dim = 0, leaf = 0, tree_kind = 0, adm = 0, kernel = 0;
  hm_compress_opts o{};
  // apply
  int64_t target = 0, nrhs = 0;
  int dtype = 0;
  std::vector<char> X;
  void *Y = nullptr;
  int64_t fp = 0;
  hm_completion c{};
};

struct Resident {
  hm_tree *tree = nullptr;
  hm_hmatrix *H = nullptr;
  int64_t bytes = 0, n = 0;
  int inflight = 0;
  bool ready = false, evict = false;
};

// Pinned staging of one worker, grown geometrically from 16 MiB.  A buffer
// it outgrows is kept until the worker ends: hipHostFree waits for the
// whole device, which would hold an apply behind every compression running
// on the other streams.
struct Pinned {
  void *p = nullptr;
  size_t bytes = 0;
  std::vector<void *> retired;
  void *get(size_t b) {
    if (b <= bytes) return p;
    const size_t nb = std::max({b, bytes * 2, size_t(16) << 20});
    void *q = nullptr;
    if (hipHostMalloc(&q, nb, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    if (p) retired.push_back(p);
    p = q;
    bytes = nb;
    return p;
  }
  ~Pinned() {
    for (void *r : retired) (void)hipHostFree(r);
    if (p) (void)hipHostFree(p);
  }
};

}  // namespace
}  // namespace hm

struct hm_server {
  int device = 0;
  hm_allocator al{};  // the caller's allocator (al.alloc null: the library's own)
  double slice_flops = 4e11;  // kernel-apply slice of a compression (0: whole launches)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<hm::Req *> pending;
  std::deque<hm_completion> done;
  std::map<int64_t, hm::Resident> res;
  int64_t budget = 0, in_use = 0, resident_bytes = 0;
  int64_t next_id = 1;
  int running = 0, running_compress = 0, compress_slots = 1;
  bool stop = false;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  // H-matrices and trees taken out of the map under mu, freed after it is
  // released (reap): every use of them was synchronized, so they go back
  // without waiting for the device, and no thread waits on mu meanwhile
  std::vector<std::pair<hm_hmatrix *, hm_tree *>> dead;
  void worker();
  // under mu: first pending request that may start now
  hm::Req *take_ready();
  void finish(hm::Req *q, hm_status st);
  // under mu
  void free_resident(std::map<int64_t, hm::Resident>::iterator it);
  // not under mu
  void reap();
};

hm::Req *hm_server::take_ready() {
  for (auto it = pending.begin(); it != pending.end(); ++it) {
    hm::Req *q = *it;
    if (q->kind == 0) {  // its memory is reserved once its tree is known
      if (running_compress >= compress_slots) continue;
      running_compress++;
      pending.erase(it);
      return q;
    }
    auto r = res.find(q->target);
    if (r == res.end() || !r->second.ready) continue;
    const int64_t es = q->dtype == HM_F32 ? 4 : 8;
    q->fp = hm::matvec_footprint(r->second.H, q->nrhs, q->dtype) + 2 * q->n * q->nrhs * es;
    if (in_use + q->fp > budget) continue;
    in_use += q->fp;
    r->second.inflight++;
    pending.erase(it);
    return q;
  }
  return nullptr;
}

void hm_server::free_resident(std::map<int64_t, hm::Resident>::iterator it) {
  dead.emplace_back(it->second.H, it->second.tree);
  in_use -= it->second.bytes;
  resident_bytes -= it->second.bytes;
  res.erase(it);
}

void hm_server::reap() {
  std::vector<std::pair<hm_hmatrix *, hm_tree *>> d;
  {
    std::lock_guard<std::mutex> lk(mu);
    d.swap(dead);
  }
  for (auto &x : d) {
    if (x.first) hm::free_idle(x.first);
    if (x.second) hm::free_idle(x.second);
  }
}

void hm_server::finish(hm::Req *q, hm_status st) {
  q->c.status = st;
  q->c.t_end = now();
  {
    std::lock_guard<std::mutex> lk(mu);
    done.push_back(q->c);
    running--;
    if (q->kind == 0) running_compress--;
  }
  cv_done.notify_all();
  cv_work.notify_all();
  delete q;
}

void hm_server::worker() {
  (void)hipSetDevice(device);
  // every device block of this worker's requests through the caller's
  // allocator, when the server was given one
  hm::AllocScope scope(al.alloc ? &al : nullptr);
  // compressions' kernel applies in row slices of about 4e11 flops (about
  // 8 ms of FP64 matrix-core time), so that applies on the other workers'
  // streams reach the device between slices
  hm::SliceScope slices(slice_flops);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
  hm::Pinned pin;
  // device-time markers of the applies
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (hipEventCreate(&ev0) != hipSuccess) ev0 = nullptr;
  if (hipEventCreate(&ev1) != hipSuccess) ev1 = nullptr;
  (void)hipGetLastError();
  for (;;) {
    hm::Req *q = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || (q = take_ready()) != nullptr; });
      if (!q) break;
      running++;
      q->c.t_admit = now();
    }
    if (q->kind == 0) {
      // ---- compression: host planning, then reserve its footprint
      hm_tree *T = nullptr;
      hm_status st = hm_build_tree(q->pts.data(), q->n, q->dim, q->leaf, q->tree_kind, q->adm, &T);
      if (st == HM_OK) st = hm_tree_color(T);
      int64_t fp = 0;
      bool reserved = false;
      if (st == HM_OK) {
        fp = hm::compress_footprint(T->t, q->o);
        std::unique_lock<std::mutex> lk(mu);
        if (fp > budget - resident_bytes) {
          st = hm::fail(HM_E_NOMEM, "compression needs more device memory than the budget leaves");
        } else {
          cv_work.wait(lk, [&] { return stop || in_use + fp <= budget; });
          if (stop) {
            st = hm::fail(HM_E_STATE, "server stopped");
          } else {
            in_use += fp;
            reserved = true;
          }
        }
      }
      q->c.bytes = fp;
      q->c.t_start = now();
      hm_hmatrix *H = nullptr;
      hm_blackbox bb{};
      if (st == HM_OK) st = hm_kernel_blackbox(T, q->kernel, &bb);
      if (st == HM_OK) st = hm_compress(T, &bb, &q->o, (void *)s, &H);
      {
        std::lock_guard<std::mutex> lk(mu);
        if (reserved) in_use -= fp;
        auto it = res.find(q->id);
        if (st == HM_OK) {
          it->second.tree = T;
          it->second.H = H;
          // the H-matrix and the device copy of its tree, held together
          it->second.bytes = hm::hmatrix_device_bytes(H) + hm::tree_device_bytes(T->t);
          it->second.n = q->n;
          it->second.ready = true;
          in_use += it->second.bytes;
          resident_bytes += it->second.bytes;
        } else {
          // freed below, after the lock, once the stream has drained
          dead.emplace_back(H, T);
          // applies waiting on it fail
          for (auto pit = pending.begin(); pit != pending.end();) {
            if ((*pit)->kind == 1 && (*pit)->target == q->id) {
              hm_completion c = (*pit)->c;
              c.status = HM_E_STATE;
              c.t_admit = c.t_start = c.t_end = now();
              done.push_back(c);
              delete *pit;
              pit = pending.erase(pit);
            } else {
              ++pit;
            }
          }
          res.erase(it);
        }
      }
      if (st != HM_OK) {
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
        reap();
      }
      finish(q, st);
      continue;
    }
    // ---- apply: host X -> pinned -> device, H X, device -> pinned -> host Y
    hm_status st = HM_OK;
    hm::Resident *R;
    {
      std::lock_guard<std::mutex> lk(mu);
      R = &res.at(q->target);
    }
    q->c.t_start = now();
    const size_t es = q->dtype == HM_F32 ? 4 : 8;
    const size_t bytes = (size_t)R->n * q->nrhs * es;
    void *hp = pin.get(2 * bytes);
    void *dx = nullptr, *dy = nullptr;
    if (!hp) st = hm::fail(HM_E_NOMEM, "pinned staging allocation failed");
    if (st == HM_OK) {
      try {
        dx = hm::scratch_alloc(bytes, (void *)s);
        dy = hm::scratch_alloc(bytes, (void *)s);
      } catch (const hm::Error &) {
        st = hm::fail(HM_E_NOMEM, "device staging allocation failed");
      }
    }
    if (st == HM_OK) {
      std::memcpy(hp, q->X.data(), bytes);
      if (ev0) (void)hipEventRecord(ev0, s);
      if (hipMemcpyAsync(dx, hp, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        st = hm::fail(HM_E_DEVICE, "copy of the right-hand sides failed");
    }
    if (st == HM_OK)
      st = hm_matvec(R->H, q->nrhs, q->dtype, dx, R->n, dy, R->n, HM_ORDER_ORIGINAL, (void *)s);
    if (st == HM_OK &&
        hipMemcpyAsync((char *)hp + bytes, dy, bytes, hipMemcpyDeviceToHost, s) != hipSuccess)
      st = hm::fail(HM_E_DEVICE, "copy of the result failed");
    hm::scratch_free(dx, (void *)s);
    hm::scratch_free(dy, (void *)s);
    if (ev1) (void)hipEventRecord(ev1, s);
    q->c.enqueue_ms = 1e3 * (now() - q->c.t_start);
    if (hipStreamSynchronize(s) != hipSuccess && st == HM_OK)
      st = hm::fail(HM_E_DEVICE, "apply failed on the device");
    if (st == HM_OK && ev0 && ev1) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess) q->c.device_ms = ms;
      (void)hipGetLastError();
    }
    if (st == HM_OK) std::memcpy(q->Y, (char *)hp + bytes, bytes);
    q->c.bytes = q->fp;
    {
      std::lock_guard<std::mutex> lk(mu);
      in_use -= q->fp;
      auto it = res.find(q->target);
      if (it != res.end() && --it->second.inflight == 0 && it->second.evict) free_resident(it);
    }
    reap();
    finish(q, st);
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
}

using namespace hm;

extern "C" {

hm_status hm_server_create(const hm_server_opts *opts, hm_server **out) {
  if (!opts || !out || opts->nslots < 1 || opts->nslots > 64)
    return fail(HM_E_ARG, "hm_server_create: bad argument");
  try {
    auto S = std::make_unique<hm_server>();
    if (hipGetDevice(&S->device) != hipSuccess) return fail(HM_E_DEVICE, "no device");
    S->budget = opts->hbm_budget;
    if (opts->allocator && opts->allocator->alloc && opts->allocator->free) S->al = *opts->allocator;
    S->compress_slots = opts->compress_slots > 0 ? std::min(opts->compress_slots, opts->nslots)
                                                 : 1;
    if (S->budget <= 0) {
      // idle cached blocks count as free memory here
      hm::trim_block_cache(S->device);
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(HM_E_DEVICE, "hipMemGetInfo failed");
      S->budget = (int64_t)(0.9 * (double)fr);
    }
    hm_server *raw = S.get();
    for (int i = 0; i < opts->nslots; ++i) S->workers.emplace_back([raw] { raw->worker(); });
    *out = S.release();
    return HM_OK;
  } catch (const std::exception &e) {
    return fail(HM_E_ARG, e.what());
  }
}

void hm_server_free(hm_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto &t : S->workers) t.join();
  for (hm::Req *q : S->pending) delete q;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    while (!S->res.empty()) {
      auto it = S->res.begin();
      if (it->second.H)
        S->free_resident(it);
      else
        S->res.erase(it);
    }
  }
  S->reap();
  delete S;
}

hm_status hm_server_submit_compress(hm_server *S, const double *points, int64_t n, int dim,
                                    int leaf_size, int tree_kind, int adm, int kernel,
                                    const hm_compress_opts *opts, int64_t *request_id) {
  if (!S || !points || n <= 0 || dim < 1 || dim > 3 || leaf_size < 1 || !opts || !request_id)
    return fail(HM_E_ARG, "hm_server_submit_compress: bad argument");
  if (kernel != HM_KERNEL_LOG && kernel != HM_KERNEL_INV_R) return fail(HM_E_ARG, "bad kernel");
  try {
    auto *q = new Req();
    q->kind = 0;
    q->pts.assign(points, points + n * dim);
    q->n = n;
    q->dim = dim;
    q->leaf = leaf_size;
    q->tree_kind = tree_kind;
    q->adm = adm;
    q->kernel = kernel;
    q->o = *opts;
    q->o.flags = 0;
    q->o.allocator = nullptr;  // the server's own allocator (if any) applies
    {
      std::lock_guard<std::mutex> lk(S->mu);
      q->id = S->next_id++;
      q->c.id = q->id;
      q->c.kind = 0;
      q->c.hmatrix = q->id;
      q->c.t_submit = S->now();
      Resident r;
      r.n = n;
      S->res[q->id] = r;
      S->pending.push_back(q);
    }
    *request_id = q->id;
    S->cv_work.notify_one();
    return HM_OK;
  } catch (const std::exception &e) {
    return fail(HM_E_NOMEM, e.what());
  }
}

hm_status hm_server_submit_matvec(hm_server *S, int64_t hmatrix, int64_t nrhs, int dtype,
                                  const void *X, void *Y, int64_t *request_id) {
  if (!S || !X || !Y || nrhs < 1 || !request_id || (dtype != HM_F64 && dtype != HM_F32))
    return fail(HM_E_ARG, "hm_server_submit_matvec: bad argument");
  try {
    auto *q = new Req();
    q->kind = 1;
    q->target = hmatrix;
    q->nrhs = nrhs;
    q->dtype = dtype;
    q->Y = Y;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      auto it = S->res.find(hmatrix);
      if (it == S->res.end() || it->second.evict) {
        delete q;
        return fail(HM_E_ARG, "hm_server_submit_matvec: unknown H-matrix");
      }
      q->n = it->second.n;  // known from the compression request
      q->id = S->next_id++;
      q->c.id = q->id;
      q->c.kind = 1;
      q->c.hmatrix = hmatrix;
      q->c.t_submit = S->now();
    }
    // X is copied now; the footprint is taken at admission
    const size_t es = dtype == HM_F32 ? 4 : 8;
    q->X.assign((const char *)X, (const char *)X + (size_t)q->n * nrhs * es);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->pending.push_back(q);
    }
    *request_id = q->c.id;
    S->cv_work.notify_one();
    return HM_OK;
  } catch (const std::exception &e) {
    return fail(HM_E_NOMEM, e.what());
  }
}

hm_status hm_server_poll(hm_server *S, int32_t max, int32_t wait_ms, hm_completion *out,
                         int32_t *count) {
  if (!S || !count || max < 0 || (max > 0 && !out)) return fail(HM_E_ARG, "hm_server_poll: bad argument");
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->done.empty() && wait_ms != 0) {
    auto pred = [&] { return !S->done.empty(); };
    if (wait_ms < 0)
      S->cv_done.wait(lk, pred);
    else
      S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), pred);
  }
  int32_t k = 0;
  while (k < max && !S->done.empty()) {
    out[k++] = S->done.front();
    S->done.pop_front();
  }
  *count = k;
  return HM_OK;
}

hm_status hm_server_hmatrix(hm_server *S, int64_t hmatrix, const hm_hmatrix **H) {
  if (!S || !H) return fail(HM_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->res.find(hmatrix);
  if (it == S->res.end() || !it->second.ready) return fail(HM_E_STATE, "H-matrix not resident");
  *H = it->second.H;
  return HM_OK;
}

hm_status hm_server_release(hm_server *S, int64_t hmatrix) {
  if (!S) return fail(HM_E_ARG, "null server");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->res.find(hmatrix);
    if (it == S->res.end() || !it->second.ready) return fail(HM_E_STATE, "H-matrix not resident");
    for (hm::Req *p : S->pending)
      if (p->kind == 1 && p->target == hmatrix)
        return fail(HM_E_STATE, "H-matrix has pending applies");
    if (it->second.inflight > 0)
      it->second.evict = true;
    else
      S->free_resident(it);
  }
  S->reap();
  S->cv_work.notify_all();
  return HM_OK;
}

hm_status hm_server_info(hm_server *S, double *now, int64_t *in_use, int64_t *budget,
                         int32_t *pending, int32_t *running, int32_t *residents) {
  if (!S) return fail(HM_E_ARG, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  if (now) *now = S->now();
  if (in_use) *in_use = S->in_use;
  if (budget) *budget = S->budget;
  if (pending) *pending = (int32_t)S->pending.size();
  if (running) *running = S->running;
  if (residents) {
    int32_t k = 0;
    for (auto &kv : S->res) k += kv.second.ready ? 1 : 0;
    *residents = k;
  }
  return HM_OK;
}

}  // extern "C"
