// Tile configuration of the batched GEMM per launch: shape classes, the tuning table and the
// timed sweeps that fill it.
//
// A launch's class is its precision and the ceil(log2) of its largest m, n, k and of its entry
// count.  The table maps classes to one of the kGemmConfigs tile configurations; classes missing
// from it take configuration 0 (64 x 64 tiles).  The built-in table is the one a sweep over the
// library's own launches wrote (gemm_tune_default.json, embedded at build time); a caller can
// replace it.  A sweep forces one configuration on every launch and times each class with HIP
// events; running the same workload once per configuration gives the per-class times from which
// a table is chosen.  All configurations give bitwise equal results, so the table changes times
// only.
#include "internal.h"

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "gemm_tune_default.inc"  // kGemmTuneDefault[] = {key, cfg, ...}, kGemmTuneDefaultN entries

namespace qps {

namespace {

std::mutex g_mu;
bool g_loaded = false;
std::map<int, int> g_table;
std::atomic<int> g_force{-1};
std::atomic<bool> g_timing{false};
struct ClassTimes {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  int64_t launches = 0;
};
std::map<int, ClassTimes> g_times;

void load_default_locked() {
  g_table.clear();
  for (int i = 0; i < kGemmTuneDefaultN; ++i) {
    const int key = kGemmTuneDefault[2 * i], cfg = kGemmTuneDefault[2 * i + 1];
    if (cfg >= 0 && cfg < kGemmConfigs) g_table[key] = cfg;
  }
  g_loaded = true;
}

int ceil_log2(int64_t x) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) < x) ++b;
  return std::min(b, 63);
}

const int kWM[kGemmConfigs] = {2, 1, 2, 1};
const int kWN[kGemmConfigs] = {2, 1, 1, 2};

}  // namespace

int gemm_class_key(int prec, int64_t max_m, int64_t max_n, int64_t max_k, int64_t nd) {
  auto b = [](int64_t x) { return std::min(ceil_log2(std::max<int64_t>(1, x)), 63); };
  return (prec & 1) << 24 | b(max_m) << 18 | b(max_n) << 12 | b(max_k) << 6 | b(nd);
}

int gemm_tune_lookup(int key) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_loaded) load_default_locked();
  auto it = g_table.find(key);
  return it == g_table.end() ? -1 : it->second;
}

int gemm_config_of(int key) {
  const int f = g_force.load();
  if (f >= 0) return f;
  const int c = gemm_tune_lookup(key);
  return c >= 0 ? c : 0;
}

void gemm_tune_set(const int* keys, const int* cfgs, int n) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (n < 0) {
    load_default_locked();
    return;
  }
  g_table.clear();
  for (int i = 0; i < n; ++i)
    if (cfgs[i] >= 0 && cfgs[i] < kGemmConfigs) g_table[keys[i]] = cfgs[i];
  g_loaded = true;
}

int gemm_tune_get(int* keys, int* cfgs, int cap) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_loaded) load_default_locked();
  int i = 0;
  for (const auto& kv : g_table) {
    if (i < cap) {
      keys[i] = kv.first;
      cfgs[i] = kv.second;
    }
    ++i;
  }
  return i;
}

template <class R>
GemmPlan gemm_plan(const GemmDescT<R>* v, size_t nd) {
  int64_t mm = 0, mn = 0, mk = 0;
  for (size_t i = 0; i < nd; ++i) {
    mm = std::max<int64_t>(mm, v[i].m);
    mn = std::max<int64_t>(mn, v[i].n);
    mk = std::max<int64_t>(mk, v[i].k);
  }
  GemmPlan p;
  p.key = gemm_class_key(sizeof(R) == 8 ? 0 : 1, mm, mn, mk, (int64_t)nd);
  p.cfg = gemm_config_of(p.key);
  const int bm = 32 * kWM[p.cfg], bn = 32 * kWN[p.cfg];
  int64_t t = 0;
  for (size_t i = 0; i < nd; ++i) t = std::max<int64_t>(t, (int64_t)((v[i].m + bm - 1) / bm) * ((v[i].n + bn - 1) / bn));
  p.tiles = (int)t;
  p.xcd = nd >= 8 ? 1 : 0;
  return p;
}
template GemmPlan gemm_plan<double>(const GemmDesc*, size_t);
template GemmPlan gemm_plan<float>(const GemmDesc32*, size_t);

bool gemm_tune_begin(int cfg) {
  if (cfg < 0 || cfg >= kGemmConfigs) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_times)
    for (auto& pr : kv.second.ev) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  g_times.clear();
  g_force.store(cfg);
  g_timing.store(true);
  return true;
}

int gemm_tune_end(int* keys, double* ms, int64_t* launches, int cap, bool* ok) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_timing.store(false);
  g_force.store(-1);
  *ok = true;
  int i = 0;
  for (auto& kv : g_times) {
    double t = 0.0;
    for (auto& pr : kv.second.ev) {
      float f = 0.f;
      if (hipEventSynchronize(pr.second) != hipSuccess || hipEventElapsedTime(&f, pr.first, pr.second) != hipSuccess)
        *ok = false;
      t += f;
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    if (i < cap) {
      keys[i] = kv.first;
      ms[i] = t;
      launches[i] = kv.second.launches;
    }
    ++i;
  }
  g_times.clear();
  return i;
}

GemmTuneTimer::GemmTuneTimer(const GemmPlan& p, hipStream_t st) : key(p.key), s(st) {
  if (!g_timing.load()) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    e0 = e1 = nullptr;
    return;
  }
  (void)hipEventRecord(e0, s);
}

GemmTuneTimer::~GemmTuneTimer() {
  if (!e0) return;
  (void)hipEventRecord(e1, s);
  std::lock_guard<std::mutex> lk(g_mu);
  ClassTimes& c = g_times[key];
  c.ev.emplace_back(e0, e1);
  c.launches += 1;
}

}  // namespace qps
