// Host runtime of the library: thread-local error text, growing device buffers, kernel-family
// profiling with HIP events, and the batched inversion driver.
#include "internal.h"

#include <algorithm>
#include <cstdlib>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace qps {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }
void clear_error() { g_last_error.clear(); }

// ------------------------------------------------------------------ device memory pool
// Released buffers are kept per device and handed to later reservations of a similar size, so
// that handles built and freed in a loop (one per frequency, or per benchmark step) do not pay
// hipMalloc / hipFree each time.  Sizes are rounded to 1/8 of their power of two; a cached block
// is reused for requests down to 4/5 of its size.  At most QPS_POOL_MAX_GB (default 64) GiB stay
// cached per device, the most recently released first; a failed hipMalloc returns the cache to the
// device and retries.
// A released block may still be read or written by queued work on any stream, so it is only
// retired: it joins the free list at the next quiescent point (the end of a library call, after
// one device synchronisation when blocks are pending, or an out-of-memory retry).  Within a call
// no block is ever handed out twice, and releasing never waits for the device.
namespace {
struct Pool {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void*>> free_blocks;
  std::map<int, std::vector<std::pair<size_t, void*>>> retired;
  std::map<int, size_t> cached;
  size_t cap = 0;
};
Pool& pool() {
  static Pool* p = [] {
    Pool* q = new Pool;  // never destroyed: no HIP calls during process teardown
    const char* e = std::getenv("QPS_POOL_MAX_GB");
    double gb = e ? std::atof(e) : 64.0;
    q->cap = gb > 0 ? (size_t)(gb * 1073741824.0) : 0;
    return q;
  }();
  return *p;
}
size_t round_size(size_t b) {
  if (b <= ((size_t)1 << 20)) return (b + 255) & ~(size_t)255;
  size_t p2 = 1;
  while (p2 < b) p2 <<= 1;
  const size_t q = p2 / 8;
  return (b + q - 1) / q * q;
}
// retired blocks of device dev (the caller has synchronised it) to the free list, or back to the
// device beyond the cap.  The retired blocks served the latest call: to make room for them, blocks
// cached earlier go back to the device first, largest first.
void flush_retired(int dev) {
  Pool& P = pool();
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lk(P.mu);
    size_t incoming = 0;
    for (auto& kv : P.retired[dev])
      if (kv.first <= P.cap) incoming += kv.first;
    auto& fl = P.free_blocks[dev];
    while (!fl.empty() && P.cached[dev] + incoming > P.cap) {
      auto last = std::prev(fl.end());
      drop.push_back(last->second);
      P.cached[dev] -= last->first;
      fl.erase(last);
    }
    for (auto& kv : P.retired[dev]) {
      if (P.cached[dev] + kv.first <= P.cap) {
        fl.emplace(kv.first, kv.second);
        P.cached[dev] += kv.first;
      } else {
        drop.push_back(kv.second);
      }
    }
    P.retired[dev].clear();
  }
  for (void* b : drop) (void)hipFree(b);
}
void trim_device(int dev) {
  Pool& P = pool();
  std::vector<void*> blocks;
  {
    std::lock_guard<std::mutex> lk(P.mu);
    for (auto& kv : P.free_blocks[dev]) blocks.push_back(kv.second);
    P.free_blocks[dev].clear();
    P.cached[dev] = 0;
  }
  for (void* b : blocks) (void)hipFree(b);
}
}  // namespace

MemBudget*& current_budget() {
  static thread_local MemBudget* b = nullptr;
  return b;
}

BumpArena*& current_bump() {
  static thread_local BumpArena* b = nullptr;
  return b;
}

hipError_t DevBuf::reserve(size_t b) {
  if (b <= bytes) return hipSuccess;
  release();
  if (BumpArena* ba = current_bump()) {
    const size_t want = (b + 255) & ~(size_t)255;
    if (ba->used + want > ba->cap) {
      if (!ba->refused) ba->refused = want;
      return hipErrorOutOfMemory;
    }
    p = ba->base + ba->used;
    ba->used += want;
    bytes = want;
    borrowed = true;
    return hipSuccess;
  }
  const size_t want = round_size(b + b / 4 + 256);
  MemBudget* mb = current_budget();
  if (mb && mb->limit > 0 && mb->used + want > mb->limit) {
    mb->refused = want;
    return hipErrorOutOfMemory;
  }
  hipError_t e0 = reserve_pool(want);
  if (e0 == hipSuccess && mb) {
    budget = mb;
    charged = want;
    mb->used += want;
    mb->peak = std::max(mb->peak, mb->used);
  }
  return e0;
}

hipError_t DevBuf::reserve_pool(size_t want) {
  int d = 0;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return e;
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    auto& fl = P.free_blocks[d];
    auto it = fl.lower_bound(want);
    if (it != fl.end() && it->first <= want + want / 4) {
      p = it->second;
      bytes = it->first;
      dev = d;
      P.cached[d] -= it->first;
      fl.erase(it);
      return hipSuccess;
    }
  }
  e = hipMalloc(&p, want);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();
    flush_retired(d);
    trim_device(d);
    e = hipMalloc(&p, want);
  }
  if (e != hipSuccess) {
    p = nullptr;
    bytes = 0;
    return e;
  }
  bytes = want;
  dev = d;
  return hipSuccess;
}

void DevBuf::release() {
  if (!p) return;
  if (borrowed) {
    p = nullptr;
    bytes = 0;
    borrowed = false;
    return;
  }
  if (budget) {
    budget->used -= charged;
    budget = nullptr;
    charged = 0;
  }
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    P.retired[dev].emplace_back(bytes, p);
  }
  p = nullptr;
  bytes = 0;
}

void pool_quiesce_current() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return;
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    if (P.retired[d].empty()) return;
  }
  (void)hipDeviceSynchronize();
  flush_retired(d);
}

int pool_release_current() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return -1;
  (void)hipDeviceSynchronize();
  flush_retired(d);
  trim_device(d);
  return 0;
}

size_t pool_cached_current() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return 0;
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  return P.cached[d];
}

// ------------------------------------------------------------------ profiling
struct ProfRecord {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double flops = 0.0, bytes = 0.0;
  int64_t launches = 0;
  double ms_done = 0.0;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::map<std::string, ProfRecord> g_prof;

void profile_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& kv : g_prof)
    for (auto& pr : kv.second.ev) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  g_prof.clear();
  g_prof_on = on;
}

bool profile_read(const std::string& fam, double* ms, int64_t* launches, double* flops, double* bytes) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  auto it = g_prof.find(fam);
  if (it == g_prof.end()) {
    *ms = 0; *launches = 0; *flops = 0; *bytes = 0;
    return true;
  }
  ProfRecord& r = it->second;
  for (auto& pr : r.ev) {
    if (hipEventSynchronize(pr.second) != hipSuccess) return false;
    float t = 0.f;
    if (hipEventElapsedTime(&t, pr.first, pr.second) != hipSuccess) return false;
    r.ms_done += t;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  r.ev.clear();
  *ms = r.ms_done;
  *launches = r.launches;
  *flops = r.flops;
  *bytes = r.bytes;
  return true;
}

ProfScope::ProfScope(const char* f, hipStream_t st, double fl, double by, int nl)
    : fam(f), s(st), flops(fl), bytes(by), launches(nl) {
  if (!g_prof_on || !f) return;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    e0 = e1 = nullptr;
    return;
  }
  (void)hipEventRecord(e0, s);
}
ProfScope::~ProfScope() {
  if (!e0) return;
  (void)hipEventRecord(e1, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfRecord& r = g_prof[fam];
  r.ev.emplace_back(e0, e1);
  r.flops += flops;
  r.bytes += bytes;
  r.launches += launches;
}

// ------------------------------------------------------------------ batched inversion
// workspace of a batched inversion: panel rows (nd * 32 * maxn), pivots (nd * maxn), info (nd)
template <class R>
static void inv_layout(int nd, int maxn, size_t* tb, size_t* ib, size_t* fb) {
  *tb = ((size_t)nd * 32 * maxn * sizeof(typename cx<R>::T) + 255) / 256 * 256;
  *ib = ((size_t)nd * maxn * sizeof(int) + 255) / 256 * 256;
  *fb = (size_t)nd * sizeof(int);
}

template <class R>
void inv_batched_needs(const std::vector<InvDescT<R>>& v, size_t* arena_bytes, size_t* work_bytes) {
  int maxn = 0;
  for (const auto& d : v) maxn = std::max(maxn, d.n);
  size_t tb, ib, fb;
  inv_layout<R>((int)v.size(), maxn, &tb, &ib, &fb);
  *arena_bytes = v.size() * sizeof(InvDescT<R>);
  *work_bytes = v.empty() ? 0 : tb + ib + fb + 512;
}

// launches the inversion; the nd singularity flags go to info_dst (device) when given, else into
// work; *dinfo receives their address
template <class R>
static hipError_t inv_launch(DevBuf& arena, DevBuf& work, const std::vector<InvDescT<R>>& v, hipStream_t s, int** dinfo,
                             int* info_dst = nullptr) {
  typedef typename cx<R>::T C_t;
  int maxn = 0;
  double flops = 0.0;
  for (const auto& d : v) {
    if (d.n > maxn) maxn = d.n;
    flops += 8.0 * (double)d.n * d.n * d.n;
  }
  const int nd = (int)v.size();
  size_t tb, ib, fb;
  inv_layout<R>(nd, maxn, &tb, &ib, &fb);
  hipError_t e = work.reserve(tb + ib + fb + 512);
  if (e != hipSuccess) return e;
  char* base = work.as<char>();
  C_t* tbuf = reinterpret_cast<C_t*>(base);
  int* ipiv = reinterpret_cast<int*>(base + tb);
  int* info = info_dst ? info_dst : reinterpret_cast<int*>(base + tb + ib);
  e = upload(arena, v, s);
  if (e != hipSuccess) return e;
  {
    // launches of the elimination kernel: one per 16-column panel plus one (n <= 1024), else three
    // per 32-column panel
    const int nlaunch = maxn <= 1024 ? (maxn + 15) / 16 + 1 : 3 * ((maxn + 31) / 32);
    ProfScope ps(sizeof(R) == 8 ? "zinv" : "cinv", s, flops, 0.0, nlaunch);
    e = launch_inv<R>(arena.as<InvDescT<R>>(), nd, maxn, tbuf, ipiv, info, s);
    if (e != hipSuccess) return e;
  }
  *dinfo = info;
  return hipSuccess;
}

template <class R>
hipError_t inv_batched(DevBuf& arena, DevBuf& work, const std::vector<InvDescT<R>>& v, hipStream_t s, bool* singular) {
  *singular = false;
  if (v.empty()) return hipSuccess;
  int* info = nullptr;
  hipError_t e = inv_launch<R>(arena, work, v, s, &info);
  if (e != hipSuccess) return e;
  const int nd = (int)v.size();
  std::vector<int> hinfo(nd);
  e = hipMemcpyAsync(hinfo.data(), info, sizeof(int) * nd, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (int i = 0; i < nd; ++i)
    if (hinfo[i] != 0) *singular = true;
  return hipSuccess;
}

template <class R>
hipError_t inv_batched_async(DevBuf& arena, DevBuf& work, const std::vector<InvDescT<R>>& v, hipStream_t s, int** dinfo) {
  *dinfo = nullptr;
  if (v.empty()) return hipSuccess;
  return inv_launch<R>(arena, work, v, s, dinfo);
}

template <class R>
hipError_t inv_batched_flags(DevBuf& arena, DevBuf& work, const std::vector<InvDescT<R>>& v, hipStream_t s, int* dflags) {
  if (v.empty()) return hipSuccess;
  int* info = nullptr;
  return inv_launch<R>(arena, work, v, s, &info, dflags);
}
template void inv_batched_needs<double>(const std::vector<InvDesc>&, size_t*, size_t*);
template void inv_batched_needs<float>(const std::vector<InvDesc32>&, size_t*, size_t*);
template hipError_t inv_batched<double>(DevBuf&, DevBuf&, const std::vector<InvDesc>&, hipStream_t, bool*);
template hipError_t inv_batched<float>(DevBuf&, DevBuf&, const std::vector<InvDesc32>&, hipStream_t, bool*);
template hipError_t inv_batched_async<double>(DevBuf&, DevBuf&, const std::vector<InvDesc>&, hipStream_t, int**);
template hipError_t inv_batched_flags<double>(DevBuf&, DevBuf&, const std::vector<InvDesc>&, hipStream_t, int*);
template hipError_t inv_batched_flags<float>(DevBuf&, DevBuf&, const std::vector<InvDesc32>&, hipStream_t, int*);

}  // namespace qps
