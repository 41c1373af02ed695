// Host runtime of the library: thread-local error text, growing device buffers, kernel-family
// profiling with HIP events, and the batched inversion driver.
#include "internal.h"

#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace qps {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }
void clear_error() { g_last_error.clear(); }

hipError_t DevBuf::reserve(size_t b) {
  if (b <= bytes) return hipSuccess;
  release();
  size_t nb = b + b / 4 + 256;
  hipError_t e = hipMalloc(&p, nb);
  if (e != hipSuccess) {
    p = nullptr;
    bytes = 0;
    return e;
  }
  bytes = nb;
  return hipSuccess;
}
void DevBuf::release() {
  // the buffer may still be read by queued kernels; hipFree must not overtake them
  if (p) {
    (void)hipDeviceSynchronize();
    (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
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

ProfScope::ProfScope(const char* f, hipStream_t st, double fl, double by) : fam(f), s(st), flops(fl), bytes(by) {
  if (!g_prof_on) return;
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
  r.launches += 1;
}

// ------------------------------------------------------------------ batched inversion
template <class R>
hipError_t inv_batched(DevBuf& arena, DevBuf& work, const std::vector<InvDescT<R>>& v, hipStream_t s, bool* singular) {
  typedef typename cx<R>::T C_t;
  *singular = false;
  if (v.empty()) return hipSuccess;
  int maxn = 0;
  double flops = 0.0;
  for (const auto& d : v) {
    if (d.n > maxn) maxn = d.n;
    flops += 8.0 * (double)d.n * d.n * d.n;
  }
  const int nd = (int)v.size();
  size_t tb = (size_t)nd * 32 * maxn * sizeof(C_t);
  tb = (tb + 255) / 256 * 256;
  size_t ib = (size_t)nd * maxn * sizeof(int);
  ib = (ib + 255) / 256 * 256;
  size_t fb = (size_t)nd * sizeof(int);
  hipError_t e = work.reserve(tb + ib + fb + 512);
  if (e != hipSuccess) return e;
  char* base = work.as<char>();
  C_t* tbuf = reinterpret_cast<C_t*>(base);
  int* ipiv = reinterpret_cast<int*>(base + tb);
  int* info = reinterpret_cast<int*>(base + tb + ib);
  e = upload(arena, v, s);
  if (e != hipSuccess) return e;
  {
    ProfScope ps(sizeof(R) == 8 ? "zinv" : "cinv", s, flops, 0.0);
    e = launch_inv<R>(arena.as<InvDescT<R>>(), nd, maxn, tbuf, ipiv, info, s);
    if (e != hipSuccess) return e;
  }
  std::vector<int> hinfo(nd);
  e = hipMemcpyAsync(hinfo.data(), info, fb, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (int i = 0; i < nd; ++i)
    if (hinfo[i] != 0) *singular = true;
  return hipSuccess;
}
template hipError_t inv_batched<double>(DevBuf&, DevBuf&, const std::vector<InvDesc>&, hipStream_t, bool*);
template hipError_t inv_batched<float>(DevBuf&, DevBuf&, const std::vector<InvDesc32>&, hipStream_t, bool*);

}  // namespace qps
