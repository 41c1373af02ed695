// Host-side declarations shared by the library's translation units: device-side
// descriptor structs and kernel launchers.
#pragma once
#include "qps_common.h"
#include "../../include/qpscatter.h"
#include <vector>

// Geometry of the discretized curve (structure of arrays, device pointers) and the
// quadrature data needed to evaluate entries of A = I/2 + D - i omega S.
#define QPS_ALPERT_MAXQ 16

struct Geo {
  const double *x, *y, *nx, *ny, *w;
  const double* kap;     // Kress: signed curvature
  const double* kressR;  // Kress: log weights indexed by (i - j) mod N
  int N;
  int quad;
  double omega;
  // transmission problem (Sec. 5): two unknowns per node, u = 2 i + c (c = 0: tau, c = 1: sigma;
  // row c = 0: value jump, c = 1: minus the normal-derivative jump); omega1 = n omega inside
  int two;
  double omega1;
  double kbar;  // max(omega, omega1): the single layer carries kbar, the normal-derivative row 1/kbar
  double g[6];           // Kapur-Rokhlin corrections, R_m = 1 + g_m
  // Alpert correction (quad == HBS_QUAD_ALPERT): grid nodes closer than alpa are left out; alpn
  // off-grid nodes q carry the kernel table alpT[i + q N] and Lagrange weights alpL[q alpnl + r] of
  // the grid offsets alpo[q] + r (r < alpnl)
  const cplx* alpT;
  const double* alpL;
  int alpn, alpnl, alpa;
  int alpo[QPS_ALPERT_MAXQ];
};

// A batch entry of the block evaluator: out[r + c*ld] = A(rows[r], cols[c]), or
// A(cols[c], rows[r]) when trans != 0.  Index lists hold global unknown indices (node indices, or
// 2 node + component for the transmission problem).
struct BlockDesc {
  const int* rows;
  const int* cols;
  cplx* out;
  // trans = 1: out[r, c] = A(cols[c], rows[r]); 0: A(rows[r], cols[c]); 2: both, the second block
  // pair_off rows below the first (one Hankel evaluation serves the two entries of a pair; KR6
  // quadrature or image points only)
  int nr, nc, ld, trans;
  // != 0: the `rows` points stand for their neighbour images translated by (sx, 0) (Sec. 3.2): the
  // entries are the plain kernel (no quadrature correction), with the image as source (trans = 1)
  // or as target (trans = 0)
  double sx;
  int pair_off;
};

// Proxy part of the compression matrix of one box: rows [row0, row0 + 3 np) of W^T
// (m x n, ld = m) for the n active unknowns `act` (6 np rows for the transmission problem).
struct ProxyDesc {
  const int* act;
  cplx* wt;
  int n, m, row0, np;
  double cx, cy, R;
  int nk;  // transmission problem: wavenumbers of the proxy rows (2: omega and n omega, 1: omega alone)
};

// Sketch Z (s x n, ld s) = Omega (s x m) * W^T (m x n, ld m), Omega complex Rademacher.
struct SketchDesc {
  const cplx* wt;
  cplx* z;
  int m, n, s, box;
};

// Column-pivoted QR of Z (s x n, ld s) in place: on exit perm[0:n] holds the column order,
// the leading k x k block the triangular factor and Z[0:k, k:n] the interpolation matrix
// T = R11^{-1} R12.
struct CpqrDesc {
  cplx* z;
  int* perm;
  int s, n;
};

// Batched GEMM entry: C = alpha * op(A) * B + beta * C, op(A) = A (m x k) or A^T (A is k x m).
template <class R>
struct GemmDescT {
  typedef typename cx<R>::T C_t;
  const C_t* A;
  const C_t* B;
  C_t* C;
  int m, n, k, lda, ldb, ldc, transA, pad;
  C_t alpha, beta;
};
typedef GemmDescT<double> GemmDesc;
typedef GemmDescT<float> GemmDesc32;

// Square matrix to be inverted in place.
template <class R>
struct InvDescT {
  typename cx<R>::T* a;
  int n, ld;
};
typedef InvDescT<double> InvDesc;
typedef InvDescT<float> InvDesc32;

// Interpolation matrix P (n x k, ld n) from the pivots and T = Z[0:k, k:n] (ld s).
struct PDesc {
  const cplx* z;
  const int* perm;
  cplx* P;
  int n, k, s;
};

// Sub-matrix copy dst[r + c*ldd] = src[r + c*lds] (nr x nc), or zero-fill when src == nullptr.
struct CopyDesc {
  const cplx* src;
  cplx* dst;
  int nr, nc, lds, ldd;
};

namespace qps {

// Device-memory budget of a handle (hbs_opts.mem_limit): every buffer reserved while the budget
// is current on the calling thread is charged to it until released; a reservation that would take
// the charged bytes above the limit fails with hipErrorOutOfMemory before any allocation.
struct MemBudget {
  size_t limit = 0;      // 0 = no limit
  size_t used = 0;       // bytes of the live buffers charged to the budget
  size_t peak = 0;
  size_t refused = 0;    // size of the last refused reservation (0 = none)
};
MemBudget*& current_budget();
struct BudgetScope {
  MemBudget* prev;
  explicit BudgetScope(MemBudget* b) : prev(current_budget()) { current_budget() = b; }
  ~BudgetScope() { current_budget() = prev; }
};

// A caller-provided device region that buffers are carved from instead of the pool while a
// BumpScope is active on the calling thread (the entry point that allocates nothing): a
// reservation takes the next aligned piece, release gives nothing back, and a reservation beyond
// the region fails with hipErrorOutOfMemory.
struct BumpArena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  size_t refused = 0;  // size of the first refused reservation (0 = none)
};
BumpArena*& current_bump();
struct BumpScope {
  BumpArena* prev;
  explicit BumpScope(BumpArena* b) : prev(current_bump()) { current_bump() = b; }
  ~BumpScope() { current_bump() = prev; }
};

// Device buffer drawn from the library's per-device pool (runtime.cpp); grows, never shrinks.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int dev = 0;
  MemBudget* budget = nullptr;  // the budget this buffer is charged to
  size_t charged = 0;           // bytes charged (the size asked of the pool)
  bool borrowed = false;        // carved from a BumpArena: never returned to the pool
  hipError_t reserve(size_t b);
  void release();
  ~DevBuf() { release(); }
  hipError_t reserve_pool(size_t want);  // a block of exactly `want` bytes from the pool
  template <class T> T* as() { return static_cast<T*>(p); }
};

int pool_release_current();      // return the current device's cached blocks to the device
void pool_quiesce_current();      // make retired blocks reusable (one device sync if any are pending)
// at the end of every library call that may release device buffers
struct PoolQuiesce {
  ~PoolQuiesce() { pool_quiesce_current(); }
};
size_t pool_cached_current();     // bytes cached for the current device

// upload a descriptor array into a growing device arena
template <class T>
hipError_t upload(DevBuf& buf, const std::vector<T>& v, hipStream_t s) {
  size_t b = v.size() * sizeof(T);
  if (b == 0) return hipSuccess;
  hipError_t e = buf.reserve(b);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(buf.p, v.data(), b, hipMemcpyHostToDevice, s);
}

// profiling of kernel families with HIP events
// One event pair brackets the work issued in the scope; `launches` is the number of kernel
// launches of the family it holds (the average launch duration is the summed time over them).
struct ProfScope {
  const char* fam;
  hipStream_t s;
  double flops, bytes;
  int launches;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(const char* fam, hipStream_t s, double flops, double bytes, int launches = 1);
  ~ProfScope();
};

// launchers (device code in kernels_build.hip / gemm.hip / kernels_qp.hip)
hipError_t launch_eval_blocks(const Geo& g, const BlockDesc* d, int nd, int max_elems, hipStream_t s);
// Alpert correction: T[i + q N] = wq[q] K(y_i, z_q, n_q) h |z'_q| at the interpolated off-grid node q of row i
// (D: derivative weights of the interpolants, laid out like Geo::alpL)
hipError_t launch_alpert_table(const Geo& g, const double* D, const double* wq, cplx* T, hipStream_t s);
hipError_t launch_proxy(const Geo& g, const ProxyDesc* d, int nd, int max_elems, hipStream_t s);
hipError_t launch_sketch(const SketchDesc* d, int nd, int max_s, int max_n, uint64_t seed, hipStream_t s);
// ws: workspace for the few-large-boxes path (one launch per pivot step); nullptr: one workgroup per box.
// launches (nullable): the number of kernel launches issued
hipError_t launch_cpqr(const CpqrDesc* d, int nd, int max_s, int max_n, double tol, int* k_out, hipStream_t s,
                       DevBuf* ws = nullptr, int* launches = nullptr);
hipError_t launch_buildP(const PDesc* d, int nd, int max_elems, hipStream_t s);
hipError_t launch_copy(const CopyDesc* d, int nd, int max_elems, hipStream_t s);
hipError_t launch_eye(const CopyDesc* d, int nd, int max_elems, hipStream_t s);  // dst = I (nr x nc)
// per box: centre, radius, bounding box, max and mean |curvature|, arc length (10 doubles)
hipError_t launch_box_circles(const Geo& g, const int* lo, const int* hi, int nbox, double* out, hipStream_t s);
hipError_t launch_gather_idx(const int* src, const int* idx, int* dst, int64_t n, hipStream_t s);
// Launch plan of one batched GEMM: tile configuration (cfg: 0 = 64 x 64 tiles of 2 x 2 wavefronts,
// 1 = 32 x 32 of one, 2 = 64 x 32 of 2 x 1, 3 = 32 x 64 of 1 x 2), grid width (tiles of the largest
// entry) and shape class.  Every configuration gives bitwise equal results.
constexpr int kGemmConfigs = 4;
struct GemmPlan {
  int cfg, tiles, key;
  int xcd;  // 1: XCD-aware workgroup order (a batch of >= 8 independent products, none split along K)
};
// shape class of a batch: precision (0 complex128, 1 complex64) and ceil(log2) of the largest m,
// n, k and of the entry count, packed as prec << 24 | m << 18 | n << 12 | k << 6 | count
int gemm_class_key(int prec, int64_t max_m, int64_t max_n, int64_t max_k, int64_t nd);
// the configuration of a class: the forced one while a tuning sweep runs, else the tuning table's
// entry, else 0
int gemm_config_of(int key);
template <class R>
GemmPlan gemm_plan(const GemmDescT<R>* v, size_t nd);
// tuning table and sweeps (gemm_tune.cpp)
int gemm_tune_lookup(int key);                                  // table entry or -1
void gemm_tune_set(const int* keys, const int* cfgs, int n);    // n < 0: the built-in table
int gemm_tune_get(int* keys, int* cfgs, int cap);               // entries copied (cap may be 0), returns the count
bool gemm_tune_begin(int cfg);                                  // force cfg on every launch and time each class
int gemm_tune_end(int* keys, double* ms, int64_t* launches, int cap, bool* ok);  // classes timed; ends the sweep
// times one launch per class while a sweep runs (not while the stream is being captured)
struct GemmTuneTimer {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int key = 0;
  hipStream_t s = nullptr;
  GemmTuneTimer(const GemmPlan& p, hipStream_t st);
  ~GemmTuneTimer();
};
template <class R>
hipError_t launch_gemm(const GemmDescT<R>* d, int nd, const GemmPlan& p, hipStream_t s);
inline hipError_t launch_zgemm(const GemmDesc* d, int nd, const GemmPlan& p, hipStream_t s) { return launch_gemm<double>(d, nd, p, s); }
// blocked Gauss-Jordan inversion; tbuf: nd * 32 * max_n complex; ipiv: nd * max_n ints; info: nd ints
template <class R>
hipError_t launch_inv(const InvDescT<R>* d, int nd, int max_n, typename cx<R>::T* tbuf, int* ipiv, int* info, hipStream_t s);
// precision casts of n complex values
hipError_t launch_cast_d2f(const cplx* src, cplxf* dst, int64_t n, hipStream_t s);
hipError_t launch_cast_f2d(const cplxf* src, cplx* dst, int64_t n, hipStream_t s);
hipError_t launch_hankel(const double* x, int64_t n, cplx* out, hipStream_t s);
hipError_t launch_eval_shift(const Geo& g, const int* rows, int nr, double shift, cplx* out, int ld, hipStream_t s);
hipError_t launch_entries(const Geo& g, const int* rows, const int* cols, int64_t n, cplx* out, hipStream_t s);

// gemm helper: build descriptors on the host, upload, launch
template <class R>
hipError_t gemm_batched(DevBuf& arena, const std::vector<GemmDescT<R>>& v, hipStream_t s, DevBuf* ws = nullptr);
template <class R>
hipError_t inv_batched(DevBuf& arena, DevBuf& work, const std::vector<InvDescT<R>>& v, hipStream_t s, bool* singular);
// the same without waiting: *dinfo receives the device address of the nd singularity flags (in
// work, valid once stream s has passed this point and until work is used again)
template <class R>
hipError_t inv_batched_async(DevBuf& arena, DevBuf& work, const std::vector<InvDescT<R>>& v, hipStream_t s, int** dinfo);
// the same with the nd flags written to dflags (device memory of the caller), nothing waited for
template <class R>
hipError_t inv_batched_flags(DevBuf& arena, DevBuf& work, const std::vector<InvDescT<R>>& v, hipStream_t s, int* dflags);
// bytes that gemm_batched / inv_batched reserve in their arena and workspace for a descriptor set
// (reserving them beforehand keeps those calls from touching the pool while other streams run)
template <class R>
void gemm_batched_needs(const std::vector<GemmDescT<R>>& v, size_t* arena_bytes, size_t* ws_bytes);
template <class R>
void inv_batched_needs(const std::vector<InvDescT<R>>& v, size_t* arena_bytes, size_t* work_bytes);

}  // namespace qps
