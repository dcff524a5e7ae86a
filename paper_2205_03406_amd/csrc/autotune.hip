// Autotuner for the kernel-apply column tile.
//
// The tile width (NT column fragments of 16 per workgroup) trades kernel
// evaluations (recomputed once per column tile) against accumulator
// registers (occupancy) and the dead columns of the last tile; the best
// value depends on the column count, the precision and the point count, and
// is not monotonic in any of them.  The first launch of each shape times
// every candidate on a prefix of the real work (256 row blocks or forest
// items) and keeps the fastest, then runs it on the whole; every candidate
// computes the same values bit for bit.  Decisions live for the process, and in the
// file named by HM_TUNE_FILE when it is set (one decision per line).
// HM_AUTOTUNE=0 turns tuning off (the cost rule of kapply_default_nt).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>

#include "hm_internal.h"
#include "kernels.h"

namespace hm {

namespace {

struct Entry {
  int nt;
  float ms_best, ms_default;
};

std::mutex g_mu;
std::map<std::tuple<int, int, int, int64_t, int, int>, Entry> g_table;
bool g_loaded = false;

std::tuple<int, int, int, int64_t, int, int> key_of(const KapplyShape &k) {
  const int nb = k.n > 0 ? (int)std::lround(std::log2((double)k.n)) : 0;
  return std::make_tuple((int)k.f32, k.kernel, k.dim, k.ncols, nb, (int)k.forest);
}

void load_file() {
  g_loaded = true;
  const char *path = std::getenv("HM_TUNE_FILE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  int f32, ker, dim, nb, forest, nt;
  long long nc;
  float a, b;
  while (std::fscanf(f, "%d %d %d %lld %d %d %d %f %f", &f32, &ker, &dim, &nc, &nb, &forest, &nt,
                     &a, &b) == 9)
    if (nt >= 2 && nt <= 16 && nt % 2 == 0)
      g_table[std::make_tuple(f32, ker, dim, (int64_t)nc, nb, forest)] = Entry{nt, a, b};
  std::fclose(f);
}

void append_file(const std::tuple<int, int, int, int64_t, int, int> &k, const Entry &e) {
  const char *path = std::getenv("HM_TUNE_FILE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %lld %d %d %d %.4f %.4f\n", std::get<0>(k), std::get<1>(k),
               std::get<2>(k), (long long)std::get<3>(k), std::get<4>(k), std::get<5>(k), e.nt,
               e.ms_best, e.ms_default);
  std::fclose(f);
}

}  // namespace

int autotune_kapply(const KapplyShape &shape,
                    const std::function<void(int, int64_t)> &launch, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const int def = kapply_default_nt(shape.ncols, shape.f32, shape.units);
  const char *env = std::getenv("HM_AUTOTUNE");
  if (env && std::strcmp(env, "0") == 0) {
    launch(def, 0);
    return def;
  }
  const auto key = key_of(shape);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_loaded) load_file();
    auto it = g_table.find(key);
    if (it != g_table.end()) {
      launch(it->second.nt, 0);
      return it->second.nt;
    }
  }
  // time every candidate once; an untimed launch of the default first
  // warms the caches
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) {
    launch(def, 0);
    return def;
  }
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    launch(def, 0);
    return def;
  }
  // candidates are timed on a prefix of the work (every candidate computes
  // the same values; the full launch with the winner follows)
  const int64_t sub = shape.units > 0 ? std::min<int64_t>(shape.units, 256) : 0;
  launch(def, sub);
  int best = def;
  float best_ms = 1e30f, def_ms = 1e30f;
  const int cands[] = {2, 4, 6, 8, 10, 12, 14, 16};
  for (int nt : cands) {
    if (nt > 2 && (int64_t)16 * (nt - 2) >= shape.ncols) break;  // wider than all columns
    (void)hipEventRecord(e0, s);
    launch(nt, sub);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (nt == def) def_ms = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = nt;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  launch(best, 0);
  Entry e{best, best_ms, def_ms};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_table.emplace(key, e).second) append_file(key, e);
  }
  return best;
}

std::string autotune_report() {
  std::lock_guard<std::mutex> lk(g_mu);
  std::ostringstream o;
  for (const auto &kv : g_table) {
    const auto &k = kv.first;
    o << (std::get<0>(k) ? "f32" : "f64") << " kernel=" << std::get<1>(k)
      << " dim=" << std::get<2>(k) << " ncols=" << std::get<3>(k) << " log2n=" << std::get<4>(k)
      << " forest=" << std::get<5>(k) << " -> nt=" << kv.second.nt << " (" << kv.second.ms_best
      << " ms; default " << kv.second.ms_default << " ms)\n";
  }
  return o.str();
}

}  // namespace hm
