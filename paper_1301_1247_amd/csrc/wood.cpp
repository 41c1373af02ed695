// Angles at and near Wood's anomalies (Sec. 2.4, second improvement).
//
// The wall densities of Eq. 2.14 have poles at k = +-k_n (k_n = sqrt(omega^2 - kappa_n^2)); when an
// angle brings some k_n near 0 they close in on the Sommerfeld contour where it crosses the origin.
// Such angles are solved on the contour k(t) = t - i a tanh((t - delta)/b), whose real-axis crossing is
// moved to delta > 0.  The contour then passes above the poles +k_n with k_n < delta (and +i|k_n|
// with |k_n| < a tanh(delta/b)), which belong below it; for each such order n the deformation leaves
// out one quasi-periodic plane wave, phi_n = exp(i (kappa_n x + k_n y)) (the residues of the two
// walls' densities lie in the null space of Q(k_n) and combine into that one wave).  So the
// representation gains one unknown a_n per crossed order and the system one row stating that no
// radiation of order n comes in from below: i k_n U_n(-y0) + U_n'(-y0) = 0, with U_n the Fourier
// coefficient of order n of the field sampled on y = -y0 (Remark 2.3).
//
// By linearity the extended system needs nothing new of the block solve: with (eta_b, xi_b) the
// solution for the incident data b and (eta_n, xi_n) the one for -phi_n on the displaced contour,
//   eta = eta_b + sum_n a_n eta_n,  xi = xi_b + sum_n a_n xi_n,
//   sum_n [L_m(eta_n, xi_n) + delta_mn 2 i k_m e^{-i k_m y0}] a_n = -L_m(eta_b, xi_b)   (one c x c system per angle),
// L_m the radiation row of order m (L_m(phi_n) = 2 i k_m e^{-i k_m y0} delta_mn).  The waves are
// extra right-hand-side columns of one block solve per Bloch phase, the rows one GPU kernel and two
// GEMMs, the c x c systems are solved on the host.
#include "hbs.h"
#include "qp_kernels.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

namespace qps {

typedef std::complex<double> zc;

namespace {

#define CK(expr)                                                                                  \
  do {                                                                                            \
    hipError_t _e = (expr);                                                                       \
    if (_e != hipSuccess) {                                                                       \
      set_error(std::string("qp_solve (Wood): ") + #expr + ": " + hipGetErrorString(_e));         \
      return _e == hipErrorOutOfMemory ? HBS_E_OOM : HBS_E_DEVICE;                                \
    }                                                                                             \
  } while (0)

#define CR(expr)                      \
  do {                                \
    int _r = (expr);                  \
    if (_r != HBS_OK) return _r;      \
  } while (0)

inline cplx toc(zc z) { return mkc(z.real(), z.imag()); }

struct Order {
  int n;
  double kap;
  zc kn;
};

// Orders around the propagating range (three evanescent ones on each side), k_n with Im >= 0.
std::vector<Order> orders_of(double om, double period, double kap) {
  const int nlo = (int)std::ceil((-om - kap) * period / (2 * M_PI)) - 3;
  const int nhi = (int)std::floor((om - kap) * period / (2 * M_PI)) + 3;
  std::vector<Order> out;
  for (int n = nlo; n <= nhi; ++n) {
    const double kx = kap + 2 * M_PI * n / period;
    out.push_back({n, kx, std::sqrt(zc(om * om - kx * kx, 0.0))});
  }
  return out;
}

double min_kn(double om, double period, double kap) {
  double mn = 1e300;
  for (const Order& o : orders_of(om, period, kap)) mn = std::min(mn, std::abs(o.kn));
  return mn;
}

// distance of a pole p from the real axis of the contour parameter: |Im t*| with t* - i a tanh((t* - delta)/b) = p
double pole_tdist(zc p, double delta, double a, double b) {
  zc t(p.real(), 0.0);
  for (int it = 0; it < 60; ++it) {
    const zc th = std::tanh((t - delta) / b);
    const zc f = t - zc(0.0, a) * th - p;
    const zc fp = 1.0 - zc(0.0, a / b) * (1.0 - th * th);
    const zc dt = f / fp;
    t -= dt;
    if (std::abs(dt) < 1e-15) break;
  }
  return std::fabs(t.imag());
}

double pole_distance(const std::vector<Order>& ords, double delta, double K, double a, double b) {
  double best = 1e300;
  for (const Order& o : ords)
    for (int sg = -1; sg <= 1; sg += 2) {
      const zc p = (double)sg * o.kn;
      if (std::fabs(p.real()) <= K) best = std::min(best, pole_tdist(p, delta, a, b));
    }
  return best;
}

// the shift in [0.25, 3] (step 0.05) with the poles farthest from the parameter's real axis
double choose_delta(const std::vector<Order>& ords, double K, double a, double b) {
  double best = 0.25, bd = -1.0;
  for (int i = 0; i <= 55; ++i) {
    const double dl = 0.25 + 0.05 * i;
    const double d = pole_distance(ords, dl, K, a, b);
    if (d > bd + 1e-12) {
      best = dl;
      bd = d;
    }
  }
  return best;
}

double contour_im(double re, double a, double b, double delta) { return -a * std::tanh((re - delta) / b); }

// orders whose pole +k_n the displaced contour passes above (it belongs below the contour's path)
int crossed_orders(const std::vector<Order>& ords, double delta, double a, double b, std::vector<Order>* out) {
  out->clear();
  for (const Order& o : ords) {
    const zc p = o.kn;
    if (p.imag() < contour_im(p.real(), a, b, delta) && p.imag() >= contour_im(p.real(), a, b, 0.0) - 1e-15)
      out->push_back(o);
    const zc q = -p;
    if (q.imag() > contour_im(q.real(), a, b, delta) + 1e-15) {
      set_error("qp_solve: the displaced contour crossed a pole -k_n (wood_shift must be positive)");
      return HBS_E_INVALID_ARG;
    }
  }
  return HBS_OK;
}

// x = A^{-1} b for a small dense complex system (partial pivoting); false when singular
bool small_solve(std::vector<zc> A, int n, std::vector<zc>& b) {
  for (int p = 0; p < n; ++p) {
    int piv = p;
    for (int i = p + 1; i < n; ++i)
      if (std::abs(A[i + p * n]) > std::abs(A[piv + p * n])) piv = i;
    if (std::abs(A[piv + p * n]) == 0.0) return false;
    if (piv != p) {
      for (int j = 0; j < n; ++j) std::swap(A[p + j * n], A[piv + j * n]);
      std::swap(b[p], b[piv]);
    }
    for (int i = p + 1; i < n; ++i) {
      const zc f = A[i + p * n] / A[p + p * n];
      for (int j = p; j < n; ++j) A[i + j * n] -= f * A[p + j * n];
      b[i] -= f * b[p];
    }
  }
  for (int p = n - 1; p >= 0; --p) {
    zc s = b[p];
    for (int j = p + 1; j < n; ++j) s -= A[p + j * n] * b[j];
    b[p] = s / A[p + p * n];
  }
  return true;
}

GemmDesc gdw(const cplx* A, int64_t lda, const cplx* B, int64_t ldb, cplx* C, int64_t ldc, int m, int n, int k, cplx beta) {
  GemmDesc g;
  g.A = A; g.B = B; g.C = C;
  g.m = m; g.n = n; g.k = k;
  g.lda = (int)lda; g.ldb = (int)ldb; g.ldc = (int)ldc;
  g.transA = 0; g.pad = 0;
  g.alpha = mkc(1, 0); g.beta = beta;
  return g;
}

}  // namespace

int qp_plan_y0(const hbs_handle* h, double period, const qp_opts* o, double* K, double* y0, int* M);

// One Bloch phase's near-Wood angles idx (caller positions) on the displaced contour.
static int solve_wood_group(hbs_handle* h, double period, const std::vector<double>& th, const std::vector<int>& idx,
                            const qp_opts* o, cplx* eta_out, cplx* xi_out, cplx* bragg_out, int32_t* nlo_out,
                            int32_t* nm_out, double* flux_out) {
  hipStream_t st = h->stream;
  const double om = h->omega;
  const int N = (int)h->N;
  const int q = (int)idx.size();
  const int P = o->P;
  double K = 0, y0 = 0;
  int M = 0;
  CR(qp_plan_y0(h, period, o, &K, &y0, &M));
  const double ca = o->ca > 0 ? o->ca : 1.0, cb = o->cb > 0 ? o->cb : 1.0;
  // samples: the alias kappa_n +- 2 pi ns / d of every propagating order must decay by e^-37 over the
  // gap g between y = -y0 and the obstacle: 2 pi ns / d - omega >= sqrt(omega^2 + (37 / g)^2)
  double maxy = 0;
  for (int64_t i = 0; i < h->N; ++i) maxy = std::max(maxy, std::fabs(h->hy[i]));
  const double gy = std::max(y0 - maxy, 1e-3);
  const int ns = o->wood_samples > 0 ? o->wood_samples
                                     : std::max(64, (int)std::ceil((om + std::sqrt(om * om + std::pow(37.0 / gy, 2))) *
                                                                   period / (2 * M_PI)));
  const double kap0 = om * std::cos(th[idx[0]]);
  const zc alpha = std::exp(zc(0.0, kap0 * period));
  const std::vector<Order> ords = orders_of(om, period, kap0);
  const double delta = o->wood_shift > 0 ? o->wood_shift : choose_delta(ords, K, ca, cb);
  std::vector<Order> cr;
  CR(crossed_orders(ords, delta, ca, cb, &cr));
  const int c = (int)cr.size();
  // the block solve for [b_1 .. b_q | -phi_1 .. -phi_c]
  QPCols cols;
  cols.delta = delta;
  cols.alpha = alpha;
  for (int a : idx) {
    cols.kx.push_back(om * std::cos(th[a]));
    cols.ky.push_back(zc(om * std::sin(th[a]), 0.0));
  }
  for (const Order& r : cr) {
    cols.kx.push_back(r.kap);
    cols.ky.push_back(r.kn);
  }
  const int nc = q + c;
  const int M2 = 2 * M;
  const int maxm = qp_max_modes_impl(om, period);
  DevBuf wb;
  size_t need = sizeof(cplx) * ((size_t)N * nc + (size_t)M2 * nc + (size_t)c * (N + M2) + (size_t)c * nc + (size_t)c * q +
                                (size_t)2 * maxm * q) +
                sizeof(RadOrder) * std::max(c, 1) + sizeof(double) * q + sizeof(int) * 3 * q + 2048;
  CK(wb.reserve(need));
  char* p = wb.as<char>();
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
  };
  cplx* etaG = (cplx*)take(sizeof(cplx) * (size_t)N * nc);
  cplx* xiG = (cplx*)take(sizeof(cplx) * (size_t)M2 * nc);
  cplx* Reta = (cplx*)take(sizeof(cplx) * (size_t)c * N);
  cplx* Rxi = (cplx*)take(sizeof(cplx) * (size_t)c * M2);
  cplx* L = (cplx*)take(sizeof(cplx) * (size_t)c * nc);
  cplx* Acoef = (cplx*)take(sizeof(cplx) * (size_t)c * q);
  cplx* brg = (cplx*)take(sizeof(cplx) * (size_t)2 * maxm * q);
  RadOrder* dord = (RadOrder*)take(sizeof(RadOrder) * std::max(c, 1));
  double* dkap = (double*)take(sizeof(double) * q);
  int* dpos = (int*)take(sizeof(int) * q);
  int* dnlo = (int*)take(sizeof(int) * q);
  int* dnm = (int*)take(sizeof(int) * q);
  std::vector<int32_t> nlo_c(nc), nm_c(nc);
  CR(qp_solve_core(h, period, th, o, &cols, etaG, xiG, nullptr, nlo_c.data(), nm_c.data(), nullptr));
  const int refine_iters = h->stats.refine_iters;
  const double refine_res = h->stats.refine_residual;
  if (c > 0) {
    // radiation rows of the crossed orders, applied to every column
    std::vector<RadOrder> ho(c);
    for (int m = 0; m < c; ++m) ho[m] = {cr[m].kap, 0.0, toc(cr[m].kn)};
    CK(hipMemcpyAsync(dord, ho.data(), sizeof(RadOrder) * c, hipMemcpyHostToDevice, st));
    std::vector<cplx> cont(3 * M);
    for (int m = 0; m < M; ++m) {
      const double h_ = 2.0 * K / M;
      const double t = -K + (m + 0.5) * h_;
      const zc k(t, -ca * std::tanh((t - delta) / cb));
      const double sech = 1.0 / std::cosh((t - delta) / cb);
      cont[m] = toc(k);
      cont[M + m] = toc(std::sqrt(om * om - k * k));
      cont[2 * M + m] = toc(h_ * zc(1.0, -(ca / cb) * sech * sech));
    }
    DevBuf dcont;
    CK(dcont.reserve(sizeof(cplx) * 3 * M));
    CK(hipMemcpyAsync(dcont.p, cont.data(), sizeof(cplx) * 3 * M, hipMemcpyHostToDevice, st));
    QPGeo Q{};
    Q.x = h->geo.x; Q.y = h->geo.y; Q.nx = h->geo.nx; Q.ny = h->geo.ny; Q.w = h->geo.w;
    Q.k = dcont.as<cplx>(); Q.s = Q.k + M; Q.wk = Q.k + 2 * M;
    Q.N = N; Q.M = M; Q.omega = om; Q.period = period; Q.shift = 0.0; Q.idx = nullptr;
    CK(launch_rad_rows(Q, dord, c, ns, P, toc(alpha), y0, Reta, Rxi, st));
    CK(gemm_batched(h->arena, std::vector<GemmDesc>{gdw(Reta, c, etaG, N, L, c, c, nc, N, mkc(0, 0))}, st, &h->splitws));
    CK(gemm_batched(h->arena, std::vector<GemmDesc>{gdw(Rxi, c, xiG, M2, L, c, c, nc, M2, mkc(1, 0))}, st, &h->splitws));
    std::vector<cplx> hL((size_t)c * nc);
    CK(hipMemcpyAsync(hL.data(), L, sizeof(cplx) * hL.size(), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    std::vector<zc> G((size_t)c * c);
    for (int m = 0; m < c; ++m)
      for (int n = 0; n < c; ++n) {
        const cplx v = hL[m + (size_t)(q + n) * c];
        G[m + (size_t)n * c] = zc(v.x, v.y);
        if (m == n) G[m + (size_t)n * c] += zc(0.0, 2.0) * cr[m].kn * std::exp(zc(0.0, -1.0) * cr[m].kn * y0);
      }
    std::vector<cplx> ha((size_t)c * q);
    for (int j = 0; j < q; ++j) {
      std::vector<zc> rhs(c);
      for (int m = 0; m < c; ++m) rhs[m] = -zc(hL[m + (size_t)j * c].x, hL[m + (size_t)j * c].y);
      if (!small_solve(G, c, rhs)) {
        set_error("qp_solve: singular radiation-condition system at a Wood's anomaly");
        return HBS_E_SINGULAR;
      }
      for (int m = 0; m < c; ++m) ha[m + (size_t)j * c] = toc(rhs[m]);
    }
    CK(hipMemcpyAsync(Acoef, ha.data(), sizeof(cplx) * ha.size(), hipMemcpyHostToDevice, st));
    // eta_b += [eta_1 .. eta_c] a,  xi_b += [xi_1 .. xi_c] a
    CK(gemm_batched(h->arena,
                    std::vector<GemmDesc>{gdw(etaG + (size_t)q * N, N, Acoef, c, etaG, N, N, q, c, mkc(1, 0)),
                                          gdw(xiG + (size_t)q * M2, M2, Acoef, c, xiG, M2, M2, q, c, mkc(1, 0))},
                    st, &h->splitws));
  }
  // Bragg amplitudes of the final densities (lattice sums; a grazing order is reported as NaN)
  std::vector<double> hk(q);
  std::vector<int> hpos(q), hnlo(q), hnm(q);
  for (int j = 0; j < q; ++j) {
    hk[j] = cols.kx[j];
    hpos[j] = idx[j];
    hnlo[j] = nlo_c[j];
    hnm[j] = nm_c[j];
  }
  CK(hipMemcpyAsync(dkap, hk.data(), sizeof(double) * q, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dpos, hpos.data(), sizeof(int) * q, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dnlo, hnlo.data(), sizeof(int) * q, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dnm, hnm.data(), sizeof(int) * q, hipMemcpyHostToDevice, st));
  {
    QPGeo Q{};
    Q.x = h->geo.x; Q.y = h->geo.y; Q.nx = h->geo.nx; Q.ny = h->geo.ny; Q.w = h->geo.w;
    Q.k = nullptr; Q.s = nullptr; Q.wk = nullptr;
    Q.N = N; Q.M = M; Q.omega = om; Q.period = period; Q.shift = 0.0; Q.idx = nullptr;
    CK(launch_bragg(Q, dkap, dnlo, dnm, maxm, q, etaG, N, y0, brg, st));
  }
  std::vector<cplx> hb((size_t)2 * maxm * q);
  CK(hipMemcpyAsync(hb.data(), brg, sizeof(cplx) * hb.size(), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  const double kzero = 1e-9 * std::max(1.0, om);
  const double nan = std::nan("");
  for (int j = 0; j < q; ++j) {
    const double kap = hk[j];
    const double k0 = std::sqrt(std::max(om * om - kap * kap, 0.0));
    double fl = 0;
    cplx* col = hb.data() + (size_t)j * 2 * maxm;
    for (int s = 0; s < hnm[j]; ++s) {
      const int nn = hnlo[j] + s;
      const double kxn = kap + 2 * M_PI * nn / period;
      const double kn = std::sqrt(std::max(om * om - kxn * kxn, 0.0));
      if (kn <= kzero) {
        col[s] = mkc(nan, nan);
        col[maxm + s] = mkc(nan, nan);
        continue;
      }
      zc cc(col[s].x, col[s].y), dd(col[maxm + s].x, col[maxm + s].y);
      if (nn == 0) dd += std::exp(zc(0.0, k0 * y0));
      fl += kn * (std::norm(cc) + std::norm(dd));
    }
    if (flux_out) flux_out[idx[j]] = std::fabs(fl - k0) / k0;
    if (nlo_out) nlo_out[idx[j]] = hnlo[j];
    if (nm_out) nm_out[idx[j]] = hnm[j];
  }
  CK(hipMemcpyAsync(brg, hb.data(), sizeof(cplx) * hb.size(), hipMemcpyHostToDevice, st));
  // into the caller's columns
  CK(launch_permute_cols(N, q, dpos, etaG, N, eta_out, N, st));
  if (xi_out) CK(launch_permute_cols(M2, q, dpos, xiG, M2, xi_out, M2, st));
  if (bragg_out) CK(launch_permute_cols(2 * maxm, q, dpos, brg, 2 * maxm, bragg_out, 2 * maxm, st));
  CK(hipStreamSynchronize(st));
  h->stats.refine_iters = refine_iters;
  h->stats.refine_residual = refine_res;
  h->stats.wood_angles += q;
  h->stats.wood_orders += c;
  h->stats.wood_shift = delta;
  return HBS_OK;
}

// Angles away from every anomaly go through the block solve on the undisplaced contour in one
// pass; the others by Bloch phase as above (or are refused with qp_opts.wood = -1).
int qp_solve_impl(hbs_handle* h, double period, const std::vector<double>& th, const qp_opts* o, cplx* eta_out,
                  cplx* xi_out, cplx* bragg_out, int32_t* nlo_out, int32_t* nm_out, double* flux_out) {
  const double om = h->omega;
  const double wood = o->wood_min_kn > 0 ? o->wood_min_kn : 0.75;
  const int n = (int)th.size();
  h->stats.wood_angles = 0;
  h->stats.wood_orders = 0;
  h->stats.wood_shift = 0.0;
  std::vector<int> normal, near;
  for (int a = 0; a < n; ++a) (min_kn(om, period, om * std::cos(th[a])) < wood ? near : normal).push_back(a);
  if (near.empty()) return qp_solve_core(h, period, th, o, nullptr, eta_out, xi_out, bragg_out, nlo_out, nm_out, flux_out);
  if (o->wood < 0 || h->nc != 1) {
    // the displaced-contour scheme is built for the Dirichlet problem only
    set_error("qp_solve: angle " + std::to_string(th[near[0]]) + " is within wood_min_kn of a Wood's anomaly" +
              (h->nc != 1 ? " (the transmission problem has no displaced-contour solve)" : ""));
    return HBS_E_WOOD;
  }
  hipStream_t st = h->stream;
  const int N = (int)h->N;
  double K = 0, y0 = 0;
  int M = 0;
  CR(qp_plan_y0(h, period, o, &K, &y0, &M));
  const int maxm = qp_max_modes_impl(om, period);
  int worst_iters = 0;
  double worst_res = 0;
  if (!normal.empty()) {
    const int q = (int)normal.size();
    std::vector<double> ths(q);
    for (int j = 0; j < q; ++j) ths[j] = th[normal[j]];
    DevBuf tb;
    CK(tb.reserve(sizeof(cplx) * ((size_t)N * q + (size_t)2 * M * q + (size_t)2 * maxm * q) + sizeof(int) * q + 1024));
    cplx* e = tb.as<cplx>();
    cplx* x = e + (size_t)N * q;
    cplx* b = x + (size_t)2 * M * q;
    int* dpos = (int*)(b + (size_t)2 * maxm * q);
    std::vector<int32_t> nl(q), nmv(q);
    std::vector<double> fl(q);
    CR(qp_solve_core(h, period, ths, o, nullptr, e, x, b, nl.data(), nmv.data(), fl.data()));
    worst_iters = h->stats.refine_iters;
    worst_res = h->stats.refine_residual;
    CK(hipMemcpyAsync(dpos, normal.data(), sizeof(int) * q, hipMemcpyHostToDevice, st));
    CK(launch_permute_cols(N, q, dpos, e, N, eta_out, N, st));
    if (xi_out) CK(launch_permute_cols(2 * M, q, dpos, x, 2 * M, xi_out, 2 * M, st));
    if (bragg_out) CK(launch_permute_cols(2 * maxm, q, dpos, b, 2 * maxm, bragg_out, 2 * maxm, st));
    CK(hipStreamSynchronize(st));
    for (int j = 0; j < q; ++j) {
      if (nlo_out) nlo_out[normal[j]] = nl[j];
      if (nm_out) nm_out[normal[j]] = nmv[j];
      if (flux_out) flux_out[normal[j]] = fl[j];
    }
  }
  // near-Wood angles by Bloch phase (phases equal to the rounding of omega d cos(theta))
  const double gtol = 32.0 * 2.220446049250313e-16 * std::max(1.0, om * period);
  std::vector<char> done(near.size(), 0);
  for (size_t i = 0; i < near.size(); ++i) {
    if (done[i]) continue;
    const zc ai = std::exp(zc(0.0, om * std::cos(th[near[i]]) * period));
    std::vector<int> grp;
    for (size_t j = i; j < near.size(); ++j) {
      if (done[j]) continue;
      const zc aj = std::exp(zc(0.0, om * std::cos(th[near[j]]) * period));
      if (std::abs(aj - ai) <= gtol) {
        grp.push_back(near[j]);
        done[j] = 1;
      }
    }
    CR(solve_wood_group(h, period, th, grp, o, eta_out, xi_out, bragg_out, nlo_out, nm_out, flux_out));
    worst_iters = std::max(worst_iters, h->stats.refine_iters);
    worst_res = std::max(worst_res, h->stats.refine_residual);
  }
  h->stats.refine_iters = worst_iters;
  h->stats.refine_residual = worst_res;
  return HBS_OK;
}

}  // namespace qps
