// C ABI of the library (include/qpscatter.h): validation, staging, handle lifecycle.
#include "hbs.h"
#include "qp_kernels.h"
#include "mlp.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace qps {
// built-in rank-predictor parameters (generated from the trained model file by the build)
#include "rank_mlp_default.inc"
const char* last_error();
void clear_error();
void profile_enable(bool on);
bool profile_read(const std::string& fam, double* ms, int64_t* launches, double* flops, double* bytes);

namespace {

// Kapur-Rokhlin 6th-order end corrections (Sec. 2.3).  The symmetric corrections g_m
// (R_m = 1 + g_m at index distance m = 1..6) make the punctured trapezoid rule exact for the
// terms of its error expansion for phi(s) ln|s| + psi(s) up to h^5:
//   sum g_m m^{2p} = 1/2 [p = 0],  sum g_m ln m = -ln(2 pi)/2,  sum g_m m^{2p} ln m = zeta'(-2p) (p = 1, 2),
// with zeta'(-2) = -zeta(3) / (4 pi^2), zeta'(-4) = 3 zeta(5) / (4 pi^4).  Solved in long double.
long double zeta_ld(int s) {
  // direct sum to K-1 plus the Euler-Maclaurin tail at K
  const int K = 64;
  long double acc = 0.0L;
  for (int n = K - 1; n >= 1; --n) acc += std::pow((long double)n, (long double)-s);
  const long double k = K;
  const long double ks = std::pow(k, (long double)-s);
  acc += k * ks / (s - 1) + ks / 2 + s * ks / (12 * k) - (long double)s * (s + 1) * (s + 2) * ks / (720 * k * k * k) +
         (long double)s * (s + 1) * (s + 2) * (s + 3) * (s + 4) * ks / (30240 * k * k * k * k * k);
  return acc;
}

void kr6_corrections(double out[6]) {
  const long double pi = std::acos(-1.0L);
  long double a[6][7];
  for (int m = 1; m <= 6; ++m) {
    const long double lm = std::log((long double)m);
    const long double m2 = (long double)m * m;
    a[0][m - 1] = 1.0L;
    a[1][m - 1] = m2;
    a[2][m - 1] = m2 * m2;
    a[3][m - 1] = lm;
    a[4][m - 1] = m2 * lm;
    a[5][m - 1] = m2 * m2 * lm;
  }
  a[0][6] = 0.5L;
  a[1][6] = 0.0L;
  a[2][6] = 0.0L;
  a[3][6] = -0.5L * std::log(2.0L * pi);
  a[4][6] = -zeta_ld(3) / (4.0L * pi * pi);
  a[5][6] = 3.0L * zeta_ld(5) / (4.0L * pi * pi * pi * pi);
  for (int c = 0; c < 6; ++c) {
    int p = c;
    for (int r = c + 1; r < 6; ++r)
      if (std::fabs(a[r][c]) > std::fabs(a[p][c])) p = r;
    for (int j = 0; j < 7; ++j) std::swap(a[c][j], a[p][j]);
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const long double f = a[r][c] / a[c][c];
      for (int j = c; j < 7; ++j) a[r][j] -= f * a[c][j];
    }
  }
  for (int c = 0; c < 6; ++c) out[c] = (double)(a[c][6] / a[c][c]);
}

// Alpert's hybrid Gauss-trapezoidal correction (Sec. 2.3 names it as the alternative to
// Kapur-Rokhlin): the grid nodes closer than a to the target are left out and m nodes t_i +- x_j h
// (weights h w_j) are added on each side.  Exactness for phi(s) ln|s| + psi(s) with phi, psi of degree
// < 2m follows from the error h^{p+1} [2 zeta(-p) ln h - 2 zeta'(-p)] of the punctured trapezoid rule
// on |s|^p ln|s|: for even p < 2m,
//   sum_j w_j x_j^p = sum_{k<a} k^p - zeta(-p),   sum_j w_j x_j^p ln x_j = sum_{k<a} k^p ln k + zeta'(-p),
// zeta(0) = -1/2, zeta(-p) = 0 (p > 0), zeta'(0) = -ln(2 pi)/2, zeta'(-2q) = (-1)^q (2q)! zeta(2q+1) / (2 (2 pi)^{2q}).
// Newton's method in long double from x_j = a (j + 1/2) / m, w_j = (a - 1/2) / m, each step halved until
// the nodes stay positive; returns the nodes ascending.
// the rule the library uses: 5 off-grid nodes per side, 6 grid nodes left out, 12-point interpolation
constexpr int kAlpM = 5, kAlpA = 6, kAlpNL = 12;

bool alpert_rule(int m, int a, long double* xo, long double* wo) {
  const long double pi = std::acos(-1.0L);
  const int n2 = 2 * m;
  std::vector<long double> A(m), B(m), x(m), w(m);
  for (int q = 0; q < m; ++q) {
    const int p = 2 * q;
    long double sa = 0, sb = 0;
    for (int k = 1; k < a; ++k) {
      const long double kp = std::pow((long double)k, (long double)p);
      sa += kp;
      sb += kp * std::log((long double)k);
    }
    long double zp;  // zeta'(-p)
    if (q == 0) {
      zp = -0.5L * std::log(2.0L * pi);
    } else {
      long double fact = 1;
      for (int t = 2; t <= 2 * q; ++t) fact *= t;
      zp = ((q & 1) ? -1.0L : 1.0L) * fact * zeta_ld(2 * q + 1) / (2.0L * std::pow(2.0L * pi, (long double)(2 * q)));
    }
    A[q] = sa + (q == 0 ? 0.5L : 0.0L);
    B[q] = sb + zp;
  }
  for (int j = 0; j < m; ++j) {
    x[j] = (long double)a * (j + 0.5L) / m;
    w[j] = ((long double)a - 0.5L) / m;
  }
  bool done = false;
  int conv = 0;  // steps taken since the step size fell to rounding level (a few more polish the root)
  for (int it = 0; it < 200 && !done; ++it) {
    std::vector<long double> J((size_t)n2 * n2), F(n2);
    for (int q = 0; q < m; ++q) {
      const int p = 2 * q;
      long double f1 = -A[q], f2 = -B[q];
      for (int j = 0; j < m; ++j) {
        const long double xp = std::pow(x[j], (long double)p), lx = std::log(x[j]);
        const long double xp1 = p ? std::pow(x[j], (long double)(p - 1)) : 0.0L;
        f1 += w[j] * xp;
        f2 += w[j] * xp * lx;
        J[q * n2 + j] = xp;
        J[q * n2 + m + j] = w[j] * p * xp1;
        J[(m + q) * n2 + j] = xp * lx;
        J[(m + q) * n2 + m + j] = w[j] * std::pow(x[j], (long double)(p - 1)) * (p * lx + 1.0L);
      }
      F[q] = f1;
      F[m + q] = f2;
    }
    // Gaussian elimination with partial pivoting: d = J^{-1} F
    for (int c = 0; c < n2; ++c) {
      int pr = c;
      for (int r = c + 1; r < n2; ++r)
        if (std::fabs(J[r * n2 + c]) > std::fabs(J[pr * n2 + c])) pr = r;
      if (J[pr * n2 + c] == 0.0L) return false;
      for (int k = 0; k < n2; ++k) std::swap(J[c * n2 + k], J[pr * n2 + k]);
      std::swap(F[c], F[pr]);
      for (int r = c + 1; r < n2; ++r) {
        const long double f = J[r * n2 + c] / J[c * n2 + c];
        for (int k = c; k < n2; ++k) J[r * n2 + k] -= f * J[c * n2 + k];
        F[r] -= f * F[c];
      }
    }
    std::vector<long double> d(n2);
    for (int r = n2 - 1; r >= 0; --r) {
      long double t = F[r];
      for (int k = r + 1; k < n2; ++k) t -= J[r * n2 + k] * d[k];
      d[r] = t / J[r * n2 + r];
    }
    long double lam = 1.0L;
    std::vector<long double> xn(m);
    for (int h = 0; h < 60; ++h) {
      bool pos = true;
      for (int j = 0; j < m; ++j) {
        xn[j] = x[j] - lam * d[m + j];
        pos = pos && xn[j] > 0;
      }
      if (pos) break;
      lam *= 0.5L;
    }
    long double step = 0, size = 0;
    for (int j = 0; j < m; ++j) {
      step = std::max(step, std::fabs(lam * d[j]) + std::fabs(lam * d[m + j]));
      size = std::max(size, std::fabs(w[j]) + std::fabs(x[j]));
      w[j] -= lam * d[j];
      x[j] = xn[j];
    }
    if (lam == 1.0L && step <= 1e-14L * size) ++conv;
    done = conv >= 4;
  }
  if (!done) return false;
  std::vector<int> ord(m);
  for (int j = 0; j < m; ++j) ord[j] = j;
  std::sort(ord.begin(), ord.end(), [&](int p, int q) { return x[p] < x[q]; });
  for (int j = 0; j < m; ++j) {
    xo[j] = x[ord[j]];
    wo[j] = w[ord[j]];
  }
  return true;
}

// Kress weights R(t_m) = -(2 pi / n) sum_{k=1}^{n-1} cos(k t_m) / k - (pi / n^2) cos(n t_m), t_m = 2 pi m / N
std::vector<double> kress_weights(int64_t N) {
  const int64_t n = N / 2;
  const long double pi = std::acos(-1.0L);
  std::vector<double> R(N);
  for (int64_t m = 0; m < N; ++m) {
    long double acc = 0.0L;
    for (int64_t k = 1; k < n; ++k) {
      const int64_t ph = (k * m) % N;
      acc += std::cos(2.0L * pi * (long double)ph / (long double)N) / (long double)k;
    }
    const int64_t ph = (n * m) % N;
    R[m] = (double)(-(2.0L * pi / n) * acc - (pi / ((long double)n * n)) * std::cos(2.0L * pi * ph / (long double)N));
  }
  return R;
}

bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

hipStream_t stream_of(const hbs_opts* o) { return o ? (hipStream_t)o->stream : nullptr; }

#define CKD(expr)                                                                          \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess) {                                                                \
      set_error(std::string(#expr) + ": " + hipGetErrorString(_e));                        \
      return _e == hipErrorOutOfMemory ? HBS_E_OOM : HBS_E_DEVICE;                         \
    }                                                                                      \
  } while (0)

// copy n doubles from caller memory (host or device) to a host vector
int fetch(const double* p, int64_t n, int mode, std::vector<double>& out) {
  out.resize(n);
  if (n == 0) return HBS_OK;
  if (mode == HBS_PTR_DEVICE) {
    CKD(hipMemcpy(out.data(), p, sizeof(double) * n, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(out.data(), p, sizeof(double) * n);
  }
  return HBS_OK;
}

}  // namespace
}  // namespace qps

using namespace qps;

// A call that failed for want of memory because the handle's mem_limit refused a reservation
// says so (the HIP error text alone would suggest the device ran out).
static int budget_status(hbs_handle* h, int code) {
  if (code == HBS_E_OOM && h && h->budget.refused > 0) {
    set_error("mem_limit of " + std::to_string(h->budget.limit) + " device bytes exceeded: " +
              std::to_string(h->budget.used) + " held, " + std::to_string(h->budget.refused) + " more requested (" +
              last_error() + ")");
  }
  if (h) h->budget.refused = 0;
  return code;
}

extern "C" {

void hbs_opts_init(hbs_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(hbs_opts);
  o->quad = HBS_QUAD_KR6;
  o->compress = HBS_COMPRESS_PROXY;
  o->leaf_size = 64;
  o->proxy_ratio = 2.0;
  o->proxy_min = 64;
  o->ptr_mode = HBS_PTR_HOST;
  o->seed = 0x5EED1301ull;
}

void qp_opts_init(qp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(qp_opts);
  o->h = 0.1;
  o->ca = 1.0;
  o->cb = 1.0;
  o->wood_min_kn = 0.75;
  o->refine_max_iter = 2;
  o->refine_tol = 1e-13;
}

const char* hbs_last_error(void) { return qps::last_error(); }

int hbs_build(const double* nodes, const double* weights, const double* normals, int64_t N, double omega, double tol,
              const hbs_opts* opts, hbs_handle** out) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  clear_error();
  if (!out) { set_error("hbs_build: out is NULL"); return HBS_E_INVALID_ARG; }
  *out = nullptr;
  hbs_opts o;
  hbs_opts_init(&o);
  if (opts) {
    if (opts->struct_size != (int32_t)sizeof(hbs_opts)) { set_error("hbs_build: opts->struct_size mismatch"); return HBS_E_INVALID_ARG; }
    o = *opts;
    if (o.leaf_size <= 0) o.leaf_size = 64;
    if (!(o.proxy_ratio > 0)) o.proxy_ratio = 2.0;
    if (o.proxy_min <= 0) o.proxy_min = 64;
  }
  if (!nodes || !weights || !normals) { set_error("hbs_build: NULL geometry pointer"); return HBS_E_INVALID_ARG; }
  if (!(omega > 0) || !std::isfinite(omega)) { set_error("hbs_build: omega must be positive and finite"); return HBS_E_INVALID_ARG; }
  if (!(tol >= 1e-15 && tol <= 1e-2)) { set_error("hbs_build: tol must lie in [1e-15, 1e-2]"); return HBS_E_INVALID_ARG; }
  if (o.quad != HBS_QUAD_KR6 && o.quad != HBS_QUAD_KRESS && o.quad != HBS_QUAD_ALPERT) {
    set_error("hbs_build: unknown quadrature");
    return HBS_E_INVALID_ARG;
  }
  if (o.compress != HBS_COMPRESS_PROXY && o.compress != HBS_COMPRESS_EXACT) { set_error("hbs_build: unknown compression"); return HBS_E_INVALID_ARG; }
  if (o.ptr_mode != HBS_PTR_HOST && o.ptr_mode != HBS_PTR_DEVICE) { set_error("hbs_build: unknown ptr_mode"); return HBS_E_INVALID_ARG; }
  if (o.precision != HBS_FP64 && o.precision != HBS_FP32_PRECOND) { set_error("hbs_build: unknown precision"); return HBS_E_INVALID_ARG; }
  if (o.rank_predictor != 0 && o.rank_predictor != 1) { set_error("hbs_build: rank_predictor must be 0 or 1"); return HBS_E_INVALID_ARG; }
  if (o.graph != 0 && o.graph != 1) { set_error("hbs_build: graph must be 0 or 1"); return HBS_E_INVALID_ARG; }
  if (o.root_level < 0 || o.root_level > 2) { set_error("hbs_build: root_level must be 0, 1 or 2"); return HBS_E_INVALID_ARG; }
  if (o.rank_scale < 0 || !std::isfinite(o.rank_scale)) { set_error("hbs_build: rank_scale must be >= 0"); return HBS_E_INVALID_ARG; }
  if (o.defer_root != 0 && o.defer_root != 1) { set_error("hbs_build: defer_root must be 0 or 1"); return HBS_E_INVALID_ARG; }
  if (!(o.image_period >= 0) || !std::isfinite(o.image_period)) {
    set_error("hbs_build: image_period must be finite and >= 0");
    return HBS_E_INVALID_ARG;
  }
  if (o.image_period > 0 && !(o.far_radius > 0)) {
    set_error("hbs_build: image_period needs far_radius > 0 (the far-field circle represents the images beyond it)");
    return HBS_E_INVALID_ARG;
  }
  if (!(o.index >= 0) || !std::isfinite(o.index)) { set_error("hbs_build: index must be finite and >= 0"); return HBS_E_INVALID_ARG; }
  if (o.index > 0) {
    // the transmission problem (Sec. 5) is built on the Kapur-Rokhlin operator; the Dirichlet-trained
    // rank model is not carried over to it
    if (o.quad != HBS_QUAD_KR6) { set_error("hbs_build: the transmission problem (index > 0) needs HBS_QUAD_KR6"); return HBS_E_INVALID_ARG; }
    if (o.rank_predictor) { set_error("hbs_build: the transmission problem (index > 0) takes rank_predictor = 0"); return HBS_E_INVALID_ARG; }
    if (N > ((int64_t)1 << 29)) { set_error("hbs_build: N too large for the transmission problem"); return HBS_E_INVALID_ARG; }
  }
  if (o.rank_predictor && !o.rank_model && kRankModelDefaultN != MLP_NPARAM) {
    set_error("hbs_build: the library has no built-in rank model; pass hbs_opts.rank_model");
    return HBS_E_INVALID_ARG;
  }
  if (o.quad == HBS_QUAD_KR6 && N < 13) { set_error("hbs_build: KR6 needs N >= 13"); return HBS_E_INVALID_ARG; }
  if (o.quad == HBS_QUAD_ALPERT) {
    // the corrected band reaches kAlpA + kAlpNL / 2 - 1 = 11 nodes from the target: it must stay inside
    // the target's box and its index neighbours, and away from its own periodic image
    if (N < 2 * (kAlpA + kAlpNL / 2) + 1) { set_error("hbs_build: Alpert quadrature needs N >= 25"); return HBS_E_INVALID_ARG; }
    if (o.leaf_size < kAlpA + kAlpNL / 2) { set_error("hbs_build: Alpert quadrature needs leaf_size >= 12"); return HBS_E_INVALID_ARG; }
  }
  if (o.quad == HBS_QUAD_KRESS) {
    if (N % 2) { set_error("hbs_build: Kress quadrature needs even N"); return HBS_E_INVALID_ARG; }
    if (!o.curvature) { set_error("hbs_build: Kress quadrature needs opts->curvature"); return HBS_E_INVALID_ARG; }
    if (o.compress != HBS_COMPRESS_EXACT) {
      set_error("hbs_build: Kress quadrature is a global correction; use HBS_COMPRESS_EXACT");
      return HBS_E_INVALID_ARG;
    }
  }
  if ((o.index > 0 ? 2 : 1) * N < 2 * (int64_t)o.leaf_size) {
    set_error("hbs_build: the number of unknowns must be at least 2 * leaf_size");
    return HBS_E_INVALID_ARG;
  }
  if (N > (int64_t)1 << 30) { set_error("hbs_build: N too large"); return HBS_E_INVALID_ARG; }
  std::vector<double> xy, w, nrm, kap;
  int r;
  if ((r = fetch(nodes, 2 * N, o.ptr_mode, xy)) != HBS_OK) return r;
  if ((r = fetch(weights, N, o.ptr_mode, w)) != HBS_OK) return r;
  if ((r = fetch(normals, 2 * N, o.ptr_mode, nrm)) != HBS_OK) return r;
  if (o.quad == HBS_QUAD_KRESS && (r = fetch(o.curvature, N, o.ptr_mode, kap)) != HBS_OK) return r;
  if (!finite_all(xy.data(), 2 * N) || !finite_all(w.data(), N) || !finite_all(nrm.data(), 2 * N) ||
      !finite_all(kap.data(), (int64_t)kap.size())) {
    set_error("hbs_build: non-finite value in the geometry");
    return HBS_E_NONFINITE;
  }
  for (int64_t i = 0; i < N; ++i) {
    if (!(w[i] > 0)) { set_error("hbs_build: weights must be positive"); return HBS_E_INVALID_ARG; }
    const double nn = std::hypot(nrm[2 * i], nrm[2 * i + 1]);
    if (std::fabs(nn - 1.0) > 1e-8) { set_error("hbs_build: normals must have unit length"); return HBS_E_INVALID_ARG; }
  }
  hbs_handle* h = new hbs_handle();
  h->budget.limit = (size_t)o.mem_limit;
  BudgetScope bscope(&h->budget);
  h->N = N;
  h->nc = o.index > 0 ? 2 : 1;
  h->NU = h->nc * N;
  h->omega = omega;
  h->tol = tol;
  h->opts = o;
  h->stream = stream_of(&o);
  h->hx.resize(N); h->hy.resize(N); h->hnx.resize(N); h->hny.resize(N);
  for (int64_t i = 0; i < N; ++i) {
    h->hx[i] = xy[2 * i];
    h->hy[i] = xy[2 * i + 1];
    h->hnx[i] = nrm[2 * i];
    h->hny[i] = nrm[2 * i + 1];
  }
  h->hw = w;
  h->hkap = kap;
  auto fail = [&](int code) {
    code = budget_status(h, code);
    delete h;
    return code;
  };
  const int nf = (o.quad == HBS_QUAD_KRESS) ? 6 : 5;
  if (h->dgeo.reserve(sizeof(double) * N * nf) != hipSuccess) { set_error("hbs_build: out of device memory"); return fail(HBS_E_OOM); }
  double* g = h->dgeo.as<double>();
  const double* src[6] = {h->hx.data(), h->hy.data(), h->hnx.data(), h->hny.data(), h->hw.data(), h->hkap.data()};
  for (int f = 0; f < nf; ++f)
    if (hipMemcpy(g + f * N, src[f], sizeof(double) * N, hipMemcpyHostToDevice) != hipSuccess) {
      set_error("hbs_build: geometry upload failed");
      return fail(HBS_E_DEVICE);
    }
  Geo& G = h->geo;
  G.x = g; G.y = g + N; G.nx = g + 2 * N; G.ny = g + 3 * N; G.w = g + 4 * N;
  G.kap = (nf == 6) ? g + 5 * N : nullptr;
  G.kressR = nullptr;
  G.N = (int)N;
  G.quad = o.quad;
  G.omega = omega;
  G.two = o.index > 0;
  G.omega1 = o.index > 0 ? o.index * omega : 0.0;
  G.kbar = o.index > 0 ? std::max(omega, o.index * omega) : 1.0;
  kr6_corrections(G.g);
  if (o.quad == HBS_QUAD_KRESS) {
    std::vector<double> R = kress_weights(N);
    if (h->dkressR.reserve(sizeof(double) * N) != hipSuccess ||
        hipMemcpy(h->dkressR.p, R.data(), sizeof(double) * N, hipMemcpyHostToDevice) != hipSuccess) {
      set_error("hbs_build: Kress table upload failed");
      return fail(HBS_E_DEVICE);
    }
    G.kressR = h->dkressR.as<double>();
  }
  G.alpT = nullptr;
  G.alpL = nullptr;
  G.alpn = G.alpnl = G.alpa = 0;
  if (o.quad == HBS_QUAD_ALPERT) {
    long double xl[kAlpM], wl[kAlpM];
    if (!alpert_rule(kAlpM, kAlpA, xl, wl)) {
      set_error("hbs_build: the Alpert rule's Newton iteration did not converge");
      return fail(HBS_E_NOT_CONVERGED);
    }
    // off-grid node q: u = +x_q (q < m) or -x_{q-m}; 12-point Lagrange stencil at offsets floor(u) - 5 ..
    const int nq = 2 * kAlpM;
    std::vector<double> L((size_t)nq * kAlpNL), D((size_t)nq * kAlpNL), wq(nq);
    for (int q = 0; q < nq; ++q) {
      const long double u = q < kAlpM ? xl[q] : -xl[q - kAlpM];
      const int o0 = (int)std::floor((double)u) - kAlpNL / 2 + 1;
      G.alpo[q] = o0;
      wq[q] = (double)wl[q % kAlpM];
      for (int r = 0; r < kAlpNL; ++r) {
        // L_r(u) and its derivative L_r(u) sum_{t != r} 1 / (u - o_t) (u is never a grid offset)
        long double v = 1.0L, dsum = 0.0L;
        for (int t = 0; t < kAlpNL; ++t)
          if (t != r) {
            v *= (u - (long double)(o0 + t)) / (long double)(r - t);
            dsum += 1.0L / (u - (long double)(o0 + t));
          }
        L[(size_t)q * kAlpNL + r] = (double)v;
        D[(size_t)q * kAlpNL + r] = (double)(v * dsum);
      }
    }
    G.alpn = nq;
    G.alpnl = kAlpNL;
    G.alpa = kAlpA;
    if (h->dalp.reserve(sizeof(double) * (2 * L.size() + wq.size())) != hipSuccess ||
        h->dalpT.reserve(sizeof(cplx) * (size_t)N * nq) != hipSuccess) {
      set_error("hbs_build: out of device memory (Alpert tables)");
      return fail(HBS_E_OOM);
    }
    double* dl = h->dalp.as<double>();
    if (hipMemcpy(dl, L.data(), sizeof(double) * L.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dl + L.size(), D.data(), sizeof(double) * D.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dl + 2 * L.size(), wq.data(), sizeof(double) * wq.size(), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("hbs_build: Alpert table upload failed");
      return fail(HBS_E_DEVICE);
    }
    G.alpL = dl;
    if (launch_alpert_table(G, dl + L.size(), dl + 2 * L.size(), h->dalpT.as<cplx>(), h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
      set_error("hbs_build: Alpert kernel table failed");
      return fail(HBS_E_DEVICE);
    }
    G.alpT = h->dalpT.as<cplx>();
  }
  if (o.rank_predictor) {
    const float* src = o.rank_model ? o.rank_model : kRankModelDefault;
    h->rank_model.assign(src, src + MLP_NPARAM);
    for (float v : h->rank_model)
      if (!std::isfinite(v)) { set_error("hbs_build: non-finite rank model parameter"); return fail(HBS_E_NONFINITE); }
  }
  int rc = qps::build(h);
  if (rc != HBS_OK) return fail(rc);
  *out = h;
  return HBS_OK;
}

static int apply_common_(hbs_handle* h, const double* in, int64_t nrhs, double* outp, bool inverse, int refine);
static int apply_common(hbs_handle* h, const double* in, int64_t nrhs, double* outp, bool inverse, int refine) {
  clear_error();
  if (!h || nrhs < 0) { set_error("hbs_apply: bad arguments"); return HBS_E_INVALID_ARG; }
  if (nrhs == 0) return HBS_OK;  // no columns: nothing read or written (the pointers may be NULL)
  if (!in || !outp) { set_error("hbs_apply: bad arguments"); return HBS_E_INVALID_ARG; }
  BudgetScope bscope(&h->budget);
  return budget_status(h, apply_common_(h, in, nrhs, outp, inverse, refine));
}
static int apply_common_(hbs_handle* h, const double* in, int64_t nrhs, double* outp, bool inverse, int refine) {
  if (nrhs == 0) return HBS_OK;
  if (in == outp) { set_error("hbs_apply: rhs and out may not alias"); return HBS_E_INVALID_ARG; }
  hipStream_t st = h->stream;
  const int64_t N = h->NU;
  const size_t bytes = sizeof(cplx) * N * nrhs;
  const cplx* B;
  cplx* X;
  DevBuf sb, sx;
  if (h->opts.ptr_mode == HBS_PTR_HOST) {
    if (!finite_all(in, 2 * N * nrhs)) { set_error("hbs_apply: non-finite right-hand side"); return HBS_E_NONFINITE; }
    CKD(sb.reserve(bytes));
    CKD(sx.reserve(bytes));
    CKD(hipMemcpyAsync(sb.p, in, bytes, hipMemcpyHostToDevice, st));
    B = sb.as<cplx>();
    X = sx.as<cplx>();
  } else {
    B = reinterpret_cast<const cplx*>(in);
    X = reinterpret_cast<cplx*>(outp);
  }
  int rc = inverse ? qps::apply_inverse(h, B, N, X, N, nrhs) : qps::apply_factors(h, false, B, N, X, N, nrhs);
  if (rc != HBS_OK) return rc;
  if (inverse && refine > 0) {
    // x <- x + A^{-1}(b - A x) with the compressed forward operator
    DevBuf rb, zb;
    CKD(rb.reserve(bytes));
    CKD(zb.reserve(bytes));
    for (int it = 0; it < refine; ++it) {
      rc = qps::apply_factors(h, false, X, N, rb.as<cplx>(), N, nrhs);
      if (rc != HBS_OK) return rc;
      CKD(launch_axpby(N, (int)nrhs, mkc(1, 0), B, N, mkc(-1, 0), rb.as<cplx>(), N, st));
      rc = qps::apply_inverse(h, rb.as<cplx>(), N, zb.as<cplx>(), N, nrhs);
      if (rc != HBS_OK) return rc;
      CKD(launch_axpby(N, (int)nrhs, mkc(1, 0), zb.as<cplx>(), N, mkc(1, 0), X, N, st));
    }
  }
  if (h->opts.ptr_mode == HBS_PTR_HOST) {
    CKD(hipMemcpyAsync(outp, X, bytes, hipMemcpyDeviceToHost, st));
  }
  CKD(hipStreamSynchronize(st));
  return HBS_OK;
}

int hbs_apply(hbs_handle* h, const double* rhs, int64_t nrhs, double* out, int32_t refine) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  return apply_common(h, rhs, nrhs, out, true, refine);
}

int hbs_forward(hbs_handle* h, const double* x, int64_t nrhs, double* out) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  return apply_common(h, x, nrhs, out, false, 0);
}

static int qp_common_(hbs_handle* h, double period, const double* thetas, int64_t n, const qp_opts* opts, bool check,
                      double are, double aim, double* eta, double* xi, double* bragg, int32_t* nlo, int32_t* nm, double* flux);
static int qp_common(hbs_handle* h, double period, const double* thetas, int64_t n, const qp_opts* opts, bool check,
                     double are, double aim, double* eta, double* xi, double* bragg, int32_t* nlo, int32_t* nm, double* flux) {
  clear_error();
  if (!h || n < 0) { set_error("qp_solve: bad arguments"); return HBS_E_INVALID_ARG; }
  if (n == 0) return HBS_OK;  // no angles: nothing to solve, nothing written
  if (!thetas || !eta) { set_error("qp_solve: bad arguments"); return HBS_E_INVALID_ARG; }
  BudgetScope bscope(&h->budget);
  return budget_status(h, qp_common_(h, period, thetas, n, opts, check, are, aim, eta, xi, bragg, nlo, nm, flux));
}
static int qp_common_(hbs_handle* h, double period, const double* thetas, int64_t n, const qp_opts* opts, bool check,
                      double are, double aim, double* eta, double* xi, double* bragg, int32_t* nlo, int32_t* nm, double* flux) {
  qp_opts o;
  qp_opts_init(&o);
  if (opts) {
    if (opts->struct_size != (int32_t)sizeof(qp_opts)) { set_error("qp_solve: opts->struct_size mismatch"); return HBS_E_INVALID_ARG; }
    o = *opts;
  }
  if (!(period > 0) || !std::isfinite(period)) { set_error("qp_solve: period must be positive"); return HBS_E_INVALID_ARG; }
  if (o.wood != 0 && o.wood != -1) { set_error("qp_solve: wood must be 0 or -1"); return HBS_E_INVALID_ARG; }
  if (!(o.wood_shift >= 0) || !(o.wood_shift < h->omega)) {
    set_error("qp_solve: wood_shift must lie in [0, omega)");
    return HBS_E_INVALID_ARG;
  }
  if (o.wood_samples < 0 || o.wood_samples > 8192) { set_error("qp_solve: wood_samples must lie in [0, 8192]"); return HBS_E_INVALID_ARG; }
  std::vector<double> th;
  int r = fetch(thetas, n, h->opts.ptr_mode, th);
  if (r != HBS_OK) return r;
  for (double t : th) {
    if (!std::isfinite(t)) { set_error("qp_solve: non-finite angle"); return HBS_E_NONFINITE; }
    if (!(t > -M_PI && t < 0)) { set_error("qp_solve: angles must lie in (-pi, 0)"); return HBS_E_INVALID_ARG; }
  }
  if (check) {
    for (double t : th) {
      const double ph = h->omega * period * std::cos(t);
      if (std::hypot(std::cos(ph) - are, std::sin(ph) - aim) > 1e-12) {
        set_error("qp_solve: alpha does not match exp(i omega d cos theta)");
        return HBS_E_ALPHA_MISMATCH;
      }
    }
  }
  const int M = qps::qp_contour_M(h, period, &o);
  if (M <= 0) return HBS_E_INVALID_ARG;
  const int maxm = qps::qp_max_modes_impl(h->omega, period);
  hipStream_t st = h->stream;
  const int64_t N = h->NU;
  DevBuf de, dx, db;
  cplx *pe, *px = nullptr, *pb = nullptr;
  const bool host = h->opts.ptr_mode == HBS_PTR_HOST;
  if (host) {
    CKD(de.reserve(sizeof(cplx) * N * n));
    pe = de.as<cplx>();
    if (xi) { CKD(dx.reserve(sizeof(cplx) * 2 * M * n)); px = dx.as<cplx>(); }
    if (bragg) { CKD(db.reserve(sizeof(cplx) * 2 * maxm * n)); pb = db.as<cplx>(); }
  } else {
    pe = reinterpret_cast<cplx*>(eta);
    px = reinterpret_cast<cplx*>(xi);
    pb = reinterpret_cast<cplx*>(bragg);
  }
  r = qps::qp_solve_impl(h, period, th, &o, pe, px, pb, nlo, nm, flux);
  if (r != HBS_OK) return r;
  if (host) {
    CKD(hipMemcpyAsync(eta, pe, sizeof(cplx) * N * n, hipMemcpyDeviceToHost, st));
    if (xi) CKD(hipMemcpyAsync(xi, px, sizeof(cplx) * 2 * M * n, hipMemcpyDeviceToHost, st));
    if (bragg) CKD(hipMemcpyAsync(bragg, pb, sizeof(cplx) * 2 * maxm * n, hipMemcpyDeviceToHost, st));
  }
  CKD(hipStreamSynchronize(st));
  return HBS_OK;
}

int qp_solve(hbs_handle* h, double period, double alpha_re, double alpha_im, const double* thetas, int64_t q,
             const qp_opts* opts, double* eta, double* xi, double* bragg, int32_t* nlo_out, int32_t* n_modes_out,
             double* flux_err) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  return qp_common(h, period, thetas, q, opts, true, alpha_re, alpha_im, eta, xi, bragg, nlo_out, n_modes_out, flux_err);
}

int qp_solve_many(hbs_handle* h, double period, const double* thetas, int64_t n, const qp_opts* opts, double* eta,
                  double* xi, double* bragg, int32_t* nlo_out, int32_t* n_modes_out, double* flux_err) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  return qp_common(h, period, thetas, n, opts, false, 0, 0, eta, xi, bragg, nlo_out, n_modes_out, flux_err);
}

int32_t qp_contour_size(const hbs_handle* h, double period, const qp_opts* opts) {
  if (!h) return -1;
  qp_opts o;
  qp_opts_init(&o);
  if (opts) o = *opts;
  return qps::qp_contour_M(h, period, &o);
}

int32_t qp_max_modes(double omega, double period) { return qps::qp_max_modes_impl(omega, period); }

int hbs_stats(const hbs_handle* h, hbs_stats_t* s) {
  if (!h || !s) { set_error("hbs_stats: NULL"); return HBS_E_INVALID_ARG; }
  *s = h->stats;
  s->struct_size = sizeof(hbs_stats_t);
  s->levels = h->L;
  s->N = h->N;
  s->unknowns = h->NU;
  s->root_size = h->nroot;
  int mr = 0;
  for (int l = 1; l <= h->L; ++l)
    for (int k : h->lv[l].k) mr = std::max(mr, k);
  s->max_rank = mr;
  s->factor_bytes = h->factor_bytes;
  s->build_seconds = h->build_seconds;
  s->root_level = h->top_identity ? 2 : 1;
  s->graph_captures = h->graph_captures;
  s->graph_replays = h->graph_replays;
  s->device_bytes_peak = (int64_t)h->budget.peak;
  return HBS_OK;
}

void hbs_free(hbs_handle* h) {
  PoolQuiesce pq_;
  delete h;
}

int qps_hankel01(const double* x, int64_t n, double* out, int32_t ptr_mode) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  clear_error();
  if (!x || !out || n < 0) { set_error("qps_hankel01: bad arguments"); return HBS_E_INVALID_ARG; }
  if (n == 0) return HBS_OK;
  if (ptr_mode == HBS_PTR_HOST) {
    for (int64_t i = 0; i < n; ++i)
      if (!(x[i] > 0) || !std::isfinite(x[i])) { set_error("qps_hankel01: x must be positive and finite"); return HBS_E_INVALID_ARG; }
    DevBuf dx, dout;
    CKD(dx.reserve(sizeof(double) * n));
    CKD(dout.reserve(sizeof(cplx) * 2 * n));
    CKD(hipMemcpy(dx.p, x, sizeof(double) * n, hipMemcpyHostToDevice));
    CKD(launch_hankel(dx.as<double>(), n, dout.as<cplx>(), nullptr));
    CKD(hipMemcpy(out, dout.p, sizeof(cplx) * 2 * n, hipMemcpyDeviceToHost));
  } else {
    CKD(launch_hankel(x, n, reinterpret_cast<cplx*>(out), nullptr));
    CKD(hipDeviceSynchronize());
  }
  return HBS_OK;
}

int qps_alpert_rule(int32_t m, int32_t a, double* x, double* w) {
  clear_error();
  if (!x || !w || m < 1 || m > 8 || a < 1 || a > 12) { set_error("qps_alpert_rule: bad arguments"); return HBS_E_INVALID_ARG; }
  long double xl[8], wl[8];
  if (!alpert_rule(m, a, xl, wl)) { set_error("qps_alpert_rule: Newton did not converge"); return HBS_E_NOT_CONVERGED; }
  for (int j = 0; j < m; ++j) {
    x[j] = (double)xl[j];
    w[j] = (double)wl[j];
  }
  return HBS_OK;
}

int qps_kr6_corrections(double out[6]) {
  if (!out) return HBS_E_INVALID_ARG;
  kr6_corrections(out);
  return HBS_OK;
}

int qps_matrix_entries(hbs_handle* h, const int32_t* rows, const int32_t* cols, int64_t n, double* out) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  clear_error();
  if (!h || !rows || !cols || !out || n < 0) { set_error("qps_matrix_entries: bad arguments"); return HBS_E_INVALID_ARG; }
  if (n == 0) return HBS_OK;
  for (int64_t i = 0; i < n; ++i)
    if (rows[i] < 0 || rows[i] >= h->NU || cols[i] < 0 || cols[i] >= h->NU) {
      set_error("qps_matrix_entries: index out of range");
      return HBS_E_INVALID_ARG;
    }
  DevBuf dr, dc, dout;
  CKD(dr.reserve(sizeof(int) * n));
  CKD(dc.reserve(sizeof(int) * n));
  CKD(dout.reserve(sizeof(cplx) * n));
  CKD(hipMemcpy(dr.p, rows, sizeof(int) * n, hipMemcpyHostToDevice));
  CKD(hipMemcpy(dc.p, cols, sizeof(int) * n, hipMemcpyHostToDevice));
  CKD(launch_entries(h->geo, dr.as<int>(), dc.as<int>(), n, dout.as<cplx>(), h->stream));
  CKD(hipStreamSynchronize(h->stream));
  CKD(hipMemcpy(out, dout.p, sizeof(cplx) * n, hipMemcpyDeviceToHost));
  return HBS_OK;
}

}  // extern "C"

namespace {
// shared body of the complex128 / complex64 GEMM diagnostics
template <class R>
int gemm_diag(const char* name, const R* A, const R* B, R* C, int32_t m, int32_t n, int32_t k, int32_t nbatch,
              int32_t transA, int32_t accumulate, int32_t ptr_mode) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  typedef typename cx<R>::T T;
  clear_error();
  if (!A || !B || !C || m <= 0 || n <= 0 || k < 0 || nbatch <= 0) { set_error(std::string(name) + ": bad arguments"); return HBS_E_INVALID_ARG; }
  const size_t sa = (size_t)m * k, sb = (size_t)k * n, sc = (size_t)m * n;
  DevBuf da, dbb, dc, arena, ws;
  const T *pa, *pb;
  T* pc;
  if (ptr_mode == HBS_PTR_HOST) {
    CKD(da.reserve(sizeof(T) * sa * nbatch + 16));
    CKD(dbb.reserve(sizeof(T) * sb * nbatch + 16));
    CKD(dc.reserve(sizeof(T) * sc * nbatch));
    if (sa) CKD(hipMemcpy(da.p, A, sizeof(T) * sa * nbatch, hipMemcpyHostToDevice));
    if (sb) CKD(hipMemcpy(dbb.p, B, sizeof(T) * sb * nbatch, hipMemcpyHostToDevice));
    CKD(hipMemcpy(dc.p, C, sizeof(T) * sc * nbatch, hipMemcpyHostToDevice));
    pa = da.as<T>(); pb = dbb.as<T>(); pc = dc.as<T>();
  } else {
    pa = reinterpret_cast<const T*>(A); pb = reinterpret_cast<const T*>(B); pc = reinterpret_cast<T*>(C);
  }
  std::vector<GemmDescT<R>> v;
  for (int b = 0; b < nbatch; ++b) {
    GemmDescT<R> g;
    g.A = pa + sa * b; g.B = pb + sb * b; g.C = pc + sc * b;
    g.m = m; g.n = n; g.k = k;
    g.lda = transA ? k : m; g.ldb = k; g.ldc = m;
    g.transA = transA; g.pad = 0;
    g.alpha = cx<R>::make(1, 0);
    g.beta = accumulate ? cx<R>::make(1, 0) : cx<R>::make(0, 0);
    v.push_back(g);
  }
  CKD(gemm_batched<R>(arena, v, nullptr, &ws));
  CKD(hipDeviceSynchronize());
  if (ptr_mode == HBS_PTR_HOST) CKD(hipMemcpy(C, pc, sizeof(T) * sc * nbatch, hipMemcpyDeviceToHost));
  return HBS_OK;
}

template <class R>
int inv_diag(const char* name, R* A, int32_t n, int32_t nbatch, int32_t ptr_mode) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  typedef typename cx<R>::T T;
  clear_error();
  if (!A || n <= 0 || nbatch <= 0) { set_error(std::string(name) + ": bad arguments"); return HBS_E_INVALID_ARG; }
  const size_t sz = (size_t)n * n;
  DevBuf da, arena, work;
  T* pa;
  if (ptr_mode == HBS_PTR_HOST) {
    CKD(da.reserve(sizeof(T) * sz * nbatch));
    CKD(hipMemcpy(da.p, A, sizeof(T) * sz * nbatch, hipMemcpyHostToDevice));
    pa = da.as<T>();
  } else {
    pa = reinterpret_cast<T*>(A);
  }
  std::vector<InvDescT<R>> v;
  for (int b = 0; b < nbatch; ++b) v.push_back({pa + sz * b, n, n});
  bool sing = false;
  CKD(inv_batched<R>(arena, work, v, nullptr, &sing));
  CKD(hipDeviceSynchronize());
  if (ptr_mode == HBS_PTR_HOST) CKD(hipMemcpy(A, pa, sizeof(T) * sz * nbatch, hipMemcpyDeviceToHost));
  if (sing) { set_error(std::string(name) + ": singular matrix"); return HBS_E_SINGULAR; }
  return HBS_OK;
}
}  // namespace

extern "C" {

int qps_zgemm(const double* A, const double* B, double* C, int32_t m, int32_t n, int32_t k, int32_t nbatch, int32_t transA,
              int32_t accumulate, int32_t ptr_mode) {
  return gemm_diag<double>("qps_zgemm", A, B, C, m, n, k, nbatch, transA, accumulate, ptr_mode);
}
int qps_cgemm(const float* A, const float* B, float* C, int32_t m, int32_t n, int32_t k, int32_t nbatch, int32_t transA,
              int32_t accumulate, int32_t ptr_mode) {
  return gemm_diag<float>("qps_cgemm", A, B, C, m, n, k, nbatch, transA, accumulate, ptr_mode);
}
int qps_zinv(double* A, int32_t n, int32_t nbatch, int32_t ptr_mode) { return inv_diag<double>("qps_zinv", A, n, nbatch, ptr_mode); }
int qps_cinv(float* A, int32_t n, int32_t nbatch, int32_t ptr_mode) { return inv_diag<float>("qps_cinv", A, n, nbatch, ptr_mode); }

int32_t qps_rank_model_size(void) { return MLP_NPARAM; }

int qps_rank_model_default(float* out) {
  clear_error();
  if (!out) { set_error("qps_rank_model_default: NULL"); return HBS_E_INVALID_ARG; }
  if (kRankModelDefaultN != MLP_NPARAM) { set_error("qps_rank_model_default: no built-in model"); return HBS_E_INVALID_ARG; }
  std::memcpy(out, kRankModelDefault, sizeof(float) * MLP_NPARAM);
  return HBS_OK;
}

int qps_rank_features(const hbs_handle* h, float* feats, int32_t* ranks, int32_t* levels, float* predicted, int64_t cap,
                      int64_t* count) {
  clear_error();
  if (!h || !count) { set_error("qps_rank_features: NULL"); return HBS_E_INVALID_ARG; }
  const int64_t nbox = (int64_t)h->feat_rank.size();
  *count = nbox;
  if (!feats && !ranks && !levels && !predicted) return HBS_OK;
  if (cap < nbox) { set_error("qps_rank_features: capacity too small"); return HBS_E_INVALID_ARG; }
  if (feats) std::memcpy(feats, h->feat.data(), sizeof(float) * MLP_IN * nbox);
  for (int64_t b = 0; b < nbox; ++b) {
    if (ranks) ranks[b] = h->feat_rank[b];
    if (levels) levels[b] = h->feat_level[b];
    if (predicted) predicted[b] = h->feat_pred[b];
  }
  return HBS_OK;
}

namespace {
// stage n floats of caller memory on the device (host mode) or borrow them (device mode)
struct FStage {
  DevBuf buf;
  float* p = nullptr;
  hipError_t in(const float* src, size_t n, int mode) {
    if (mode == HBS_PTR_DEVICE) { p = const_cast<float*>(src); return hipSuccess; }
    hipError_t e = buf.reserve(sizeof(float) * std::max<size_t>(1, n));
    if (e != hipSuccess) return e;
    p = buf.as<float>();
    return src && n ? hipMemcpy(p, src, sizeof(float) * n, hipMemcpyHostToDevice) : hipSuccess;
  }
  hipError_t out(float* dst, size_t n, int mode) {
    if (mode == HBS_PTR_DEVICE || !dst || !n) return hipSuccess;
    return hipMemcpy(dst, p, sizeof(float) * n, hipMemcpyDeviceToHost);
  }
};
bool mlp_args_ok(const char* name, const void* params, const void* x, int64_t n, int32_t ptr_mode) {
  if (!params || !x || n <= 0 || (ptr_mode != HBS_PTR_HOST && ptr_mode != HBS_PTR_DEVICE)) {
    set_error(std::string(name) + ": bad arguments");
    return false;
  }
  return true;
}
}  // namespace

int qps_mlp_forward(const float* params, const float* x, int64_t n, float* y, int32_t ptr_mode) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  clear_error();
  if (!mlp_args_ok("qps_mlp_forward", params, x, n, ptr_mode) || !y) return HBS_E_INVALID_ARG;
  FStage P, X, Y;
  CKD(P.in(params, MLP_NPARAM, ptr_mode));
  CKD(X.in(x, (size_t)n * MLP_IN, ptr_mode));
  if (ptr_mode == HBS_PTR_DEVICE) Y.p = y; else CKD(Y.in(nullptr, n, HBS_PTR_HOST));
  CKD(mlp_forward(P.p, X.p, n, Y.p, nullptr));
  CKD(hipDeviceSynchronize());
  CKD(Y.out(y, n, ptr_mode));
  return HBS_OK;
}

int qps_mlp_grad(const float* params, const float* x, const float* t, int64_t n, float tau, float* grad, float* loss,
                 int32_t ptr_mode) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  clear_error();
  if (!mlp_args_ok("qps_mlp_grad", params, x, n, ptr_mode) || !t || !grad || !loss) return HBS_E_INVALID_ARG;
  if (!(tau > 0.f && tau < 1.f)) { set_error("qps_mlp_grad: tau must lie in (0, 1)"); return HBS_E_INVALID_ARG; }
  FStage P, X, T, G, Lo;
  DevBuf work;
  CKD(P.in(params, MLP_NPARAM, ptr_mode));
  CKD(X.in(x, (size_t)n * MLP_IN, ptr_mode));
  CKD(T.in(t, n, ptr_mode));
  if (ptr_mode == HBS_PTR_DEVICE) { G.p = grad; Lo.p = loss; }
  else { CKD(G.in(nullptr, MLP_NPARAM, HBS_PTR_HOST)); CKD(Lo.in(nullptr, 1, HBS_PTR_HOST)); }
  CKD(mlp_grad(work, P.p, X.p, T.p, n, tau, G.p, Lo.p, nullptr));
  CKD(hipDeviceSynchronize());
  CKD(G.out(grad, MLP_NPARAM, ptr_mode));
  CKD(Lo.out(loss, 1, ptr_mode));
  return HBS_OK;
}

int qps_mlp_train(float* params, const float* x, const float* t, int64_t n, float tau, int32_t steps, float lr, float* loss_hist,
                  int32_t ptr_mode) {
  PoolQuiesce pq_;  // retired device buffers become reusable once the call is done
  clear_error();
  if (!mlp_args_ok("qps_mlp_train", params, x, n, ptr_mode) || !t || steps < 0 || !(lr > 0.f)) return HBS_E_INVALID_ARG;
  if (!(tau > 0.f && tau < 1.f)) { set_error("qps_mlp_train: tau must lie in (0, 1)"); return HBS_E_INVALID_ARG; }
  FStage P, X, T, Hh;
  DevBuf work;
  CKD(P.in(params, MLP_NPARAM, ptr_mode));
  CKD(X.in(x, (size_t)n * MLP_IN, ptr_mode));
  CKD(T.in(t, n, ptr_mode));
  float* hist = nullptr;
  if (loss_hist) {
    if (ptr_mode == HBS_PTR_DEVICE) hist = loss_hist;
    else { CKD(Hh.in(nullptr, std::max(1, steps), HBS_PTR_HOST)); hist = Hh.p; }
  }
  CKD(mlp_train(work, P.p, X.p, T.p, n, tau, steps, lr, hist, nullptr));
  CKD(hipDeviceSynchronize());
  CKD(P.out(params, MLP_NPARAM, ptr_mode));
  if (loss_hist) CKD(Hh.out(loss_hist, steps, ptr_mode));
  return HBS_OK;
}

int qps_pool_release(void) {
  clear_error();
  if (pool_release_current() != 0) { set_error("qps_pool_release: no current device"); return HBS_E_DEVICE; }
  return HBS_OK;
}

int64_t qps_pool_cached_bytes(void) { return (int64_t)pool_cached_current(); }

int qps_profile_enable(int32_t on) {
  profile_enable(on != 0);
  return HBS_OK;
}

int qps_profile_read(const char* family, double* ms, int64_t* launches, double* flops, double* bytes) {
  if (!family || !ms || !launches || !flops || !bytes) return HBS_E_INVALID_ARG;
  if (!profile_read(family, ms, launches, flops, bytes)) { set_error("qps_profile_read: event query failed"); return HBS_E_DEVICE; }
  return HBS_OK;
}

int qps_gemm_class(int32_t complex64, int64_t max_m, int64_t max_n, int64_t max_k, int64_t count, int32_t* key) {
  clear_error();
  if (!key || max_m < 0 || max_n < 0 || max_k < 0 || count < 0) {
    set_error("qps_gemm_class: sizes must be >= 0 and key non-null");
    return HBS_E_INVALID_ARG;
  }
  *key = gemm_class_key(complex64 ? 1 : 0, max_m, max_n, max_k, count);
  return HBS_OK;
}

int qps_gemm_tune_lookup(int32_t key, int32_t* cfg) {
  clear_error();
  if (!cfg) { set_error("qps_gemm_tune_lookup: cfg is null"); return HBS_E_INVALID_ARG; }
  *cfg = gemm_tune_lookup(key);
  return HBS_OK;
}

int qps_gemm_tune_set(const int32_t* keys, const int32_t* cfgs, int32_t n) {
  clear_error();
  if (n > 0 && (!keys || !cfgs)) { set_error("qps_gemm_tune_set: null table"); return HBS_E_INVALID_ARG; }
  for (int32_t i = 0; i < n; ++i)
    if (cfgs[i] < 0 || cfgs[i] >= kGemmConfigs) {
      set_error("qps_gemm_tune_set: configuration out of range");
      return HBS_E_INVALID_ARG;
    }
  gemm_tune_set(keys, cfgs, n);
  return HBS_OK;
}

int qps_gemm_tune_get(int32_t* keys, int32_t* cfgs, int32_t cap, int32_t* n) {
  clear_error();
  if (!n || cap < 0 || (cap > 0 && (!keys || !cfgs))) { set_error("qps_gemm_tune_get: bad arguments"); return HBS_E_INVALID_ARG; }
  *n = gemm_tune_get(keys, cfgs, cap);
  return HBS_OK;
}

int qps_gemm_tune_begin(int32_t cfg) {
  clear_error();
  if (!gemm_tune_begin(cfg)) { set_error("qps_gemm_tune_begin: configuration out of range"); return HBS_E_INVALID_ARG; }
  return HBS_OK;
}

int qps_gemm_tune_end(int32_t* keys, double* ms, int64_t* launches, int32_t cap, int32_t* n) {
  clear_error();
  if (!n || cap < 0 || (cap > 0 && (!keys || !ms || !launches))) {
    set_error("qps_gemm_tune_end: bad arguments");
    return HBS_E_INVALID_ARG;
  }
  bool ok = true;
  *n = gemm_tune_end(keys, ms, launches, cap, &ok);
  if (!ok) { set_error("qps_gemm_tune_end: event query failed"); return HBS_E_DEVICE; }
  return HBS_OK;
}

}  // extern "C"
