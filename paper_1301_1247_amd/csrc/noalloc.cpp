// hbs_apply_noalloc: the application of the compressed inverse for callers that cannot allocate
// device memory.  Every workspace of the call is carved from `scratch`, a static device array of
// QPS_NOALLOC_SCRATCH_BYTES that each GPU holds from the call that first uses it until the process
// ends, instead of the library's pool; the call makes no hipMalloc or hipFree.
#include "hbs.h"
#include "qp_kernels.h"

#include <algorithm>
#include <mutex>
#include <string>

#define QPS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

// The host-side name of this array is only a stand-in for the symbol: host code uses the per-device
// address that hipGetSymbolAddress returns (scratch_base below), never `scratch` itself.
static __device__ __align__(256) char scratch[QPS_NOALLOC_SCRATCH_BYTES];

namespace qps {
const char* last_error();
void clear_error();

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// the current device's copy of the scratch array (looked up once per device, that device current)
int scratch_base(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error(std::string("hbs_apply_noalloc: hipGetDevice: ") + hipGetErrorString(e));
    return HBS_E_DEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("hbs_apply_noalloc: device index out of range");
    return HBS_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hbs_apply_noalloc: hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return HBS_E_DEVICE;
    }
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return HBS_OK;
}

void swap_buf(DevBuf& a, DevBuf& b) {
  std::swap(a.p, b.p);
  std::swap(a.bytes, b.bytes);
  std::swap(a.dev, b.dev);
  std::swap(a.budget, b.budget);
  std::swap(a.charged, b.charged);
  std::swap(a.borrowed, b.borrowed);
}

// The handle's apply workspaces are set aside for the call (empty stand-ins take their place, so
// that every reservation of the call comes from the scratch) and put back afterwards; the graph
// option is off for the call (capturing a graph allocates).
struct WorkspaceSwap {
  hbs_handle* h;
  DevBuf tmp[12];
  int graph;
  DevBuf* slot(int i) {
    DevBuf* s[12] = {&h->ab_up, &h->ab_x0, &h->ab_x1, &h->ab_root, &h->ab_in32, &h->ab_up32,
                     &h->ab_x32a, &h->ab_x32b, &h->arena, &h->arena32, &h->splitws, &h->work};
    return s[i];
  }
  explicit WorkspaceSwap(hbs_handle* hh) : h(hh), graph(hh->opts.graph) {
    for (int i = 0; i < 12; ++i) swap_buf(*slot(i), tmp[i]);
    h->opts.graph = 0;
  }
  ~WorkspaceSwap() {
    for (int i = 0; i < 12; ++i) swap_buf(*slot(i), tmp[i]);
    h->opts.graph = graph;
  }
};

#define CKN(expr)                                                                         \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess) {                                                               \
      set_error(std::string("hbs_apply_noalloc: ") + #expr + ": " + hipGetErrorString(_e)); \
      return _e == hipErrorOutOfMemory ? HBS_E_OOM : HBS_E_DEVICE;                        \
    }                                                                                     \
  } while (0)

// the largest workspaces of an inverse apply of r columns (level buffers, ping-pong buffers,
// root, and the two refinement buffers): a lower bound of what the call carves, checked first
size_t apply_need(const hbs_handle* h, int64_t r, int refine) {
  const int L = h->L;
  int64_t up = 0, xmax = 1;
  for (int l = 1; l <= L; ++l) up += h->lv[l].ktot;
  for (int l = 1; l < L; ++l) xmax = std::max<int64_t>(xmax, h->lv[l].ntot);
  size_t b = sizeof(cplx) * (size_t)r * (size_t)(up + 2 * xmax + h->nroot);
  if (refine > 0) b += 2 * sizeof(cplx) * (size_t)h->NU * (size_t)r;
  return b;
}

int apply_body(hbs_handle* h, const cplx* B, cplx* X, int64_t r, int refine) {
  const int64_t N = h->NU;
  hipStream_t st = h->stream;
  int rc = apply_inverse(h, B, N, X, N, r);
  if (rc != HBS_OK) return rc;
  if (refine > 0) {
    DevBuf rb, zb;
    CKN(rb.reserve(sizeof(cplx) * N * r));
    CKN(zb.reserve(sizeof(cplx) * N * r));
    for (int it = 0; it < refine; ++it) {
      rc = apply_factors(h, false, X, N, rb.as<cplx>(), N, r);
      if (rc != HBS_OK) return rc;
      CKN(launch_axpby(N, (int)r, mkc(1, 0), B, N, mkc(-1, 0), rb.as<cplx>(), N, st));
      rc = apply_inverse(h, rb.as<cplx>(), N, zb.as<cplx>(), N, r);
      if (rc != HBS_OK) return rc;
      CKN(launch_axpby(N, (int)r, mkc(1, 0), zb.as<cplx>(), N, mkc(1, 0), X, N, st));
    }
  }
  CKN(hipStreamSynchronize(st));
  return HBS_OK;
}

}  // namespace
}  // namespace qps

using namespace qps;

extern "C" int hbs_apply_noalloc(hbs_handle* h, const double* rhs, int64_t nrhs, double* out, int32_t refine) {
  clear_error();
  if (!h || nrhs < 0) { set_error("hbs_apply_noalloc: bad arguments"); return HBS_E_INVALID_ARG; }
  if (nrhs == 0) return HBS_OK;  // no columns: nothing read or written (the pointers may be NULL)
  if (!rhs || !out) { set_error("hbs_apply_noalloc: bad arguments"); return HBS_E_INVALID_ARG; }
  if (h->opts.ptr_mode != HBS_PTR_DEVICE) {
    set_error("hbs_apply_noalloc: needs a handle built with HBS_PTR_DEVICE (rhs and out in device memory)");
    return HBS_E_INVALID_ARG;
  }
  if (refine < 0 || refine > 16) { set_error("hbs_apply_noalloc: refine must lie in [0, 16]"); return HBS_E_INVALID_ARG; }
  if (rhs == out) { set_error("hbs_apply_noalloc: rhs and out may not alias"); return HBS_E_INVALID_ARG; }
  if (nrhs > (int64_t)1 << 30) { set_error("hbs_apply_noalloc: nrhs too large"); return HBS_E_INVALID_ARG; }
  const size_t need = apply_need(h, nrhs, refine);
  if (need > QPS_NOALLOC_SCRATCH_BYTES) {
    set_error("hbs_apply_noalloc: " + std::to_string(nrhs) + " columns need at least " + std::to_string(need) +
              " bytes of workspace, more than the " + std::to_string(QPS_NOALLOC_SCRATCH_BYTES) + "-byte scratch");
    return HBS_E_OOM;
  }
  char* base = nullptr;
  int rc = scratch_base(&base);
  if (rc != HBS_OK) return rc;
  BumpArena ba;
  ba.base = base;
  ba.cap = QPS_NOALLOC_SCRATCH_BYTES;
  {
    WorkspaceSwap ws(h);
    BumpScope bs(&ba);
    rc = apply_body(h, reinterpret_cast<const cplx*>(rhs), reinterpret_cast<cplx*>(out), nrhs, refine);
    // the carved pieces die with the stand-ins here; nothing of the scratch outlives the call
  }
  if (rc == HBS_E_OOM && ba.refused) {
    set_error("hbs_apply_noalloc: the workspaces of " + std::to_string(nrhs) + " columns exceed the " +
              std::to_string(QPS_NOALLOC_SCRATCH_BYTES) + "-byte scratch (" + last_error() + ")");
  }
  return rc;
}
