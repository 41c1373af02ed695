// Quasi-periodic block solve (Sec. 3.1) on top of the compressed inverse.
//
// With B(alpha) = B_L + alpha B_R and C(alpha) = C_L - alpha^{-1} C_R (Eqs. 2.16-2.17), one
// application of A^{-1} to [B_L | B_R | b_1 .. b_n] serves every Bloch phase (Remark 3.1), and
// the Schur complements follow from four alpha-free products:
//   S(alpha) = Q(alpha) - [C_L X_L + alpha C_L X_R - alpha^{-1} C_R X_L - C_R X_R].
// Per angle (Eq. 3.1 with the sign of the printed first line corrected):
//   xi = -S^{-1} C(alpha) A^{-1} b,  eta = A^{-1} b - A^{-1} B(alpha) xi.
// The bordered system [[A, B], [C, Q]] is then refined: the residual is formed with the
// compressed forward operator and corrected with the same block solve.
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
      set_error(std::string("qp_solve: ") + #expr + ": " + hipGetErrorString(_e));                \
      return _e == hipErrorOutOfMemory ? HBS_E_OOM : HBS_E_DEVICE;                                \
    }                                                                                             \
  } while (0)

#define CR(expr)                      \
  do {                                \
    int _r = (expr);                  \
    if (_r != HBS_OK) return _r;      \
  } while (0)

GemmDesc gd(const cplx* A, int64_t lda, int transA, const cplx* B, int64_t ldb, cplx* C, int64_t ldc, int m, int n, int k,
            cplx alpha, cplx beta) {
  GemmDesc g;
  g.A = A; g.B = B; g.C = C;
  g.m = m; g.n = n; g.k = k;
  g.lda = (int)lda; g.ldb = (int)ldb; g.ldc = (int)ldc;
  g.transA = transA; g.pad = 0;
  g.alpha = alpha; g.beta = beta;
  return g;
}

inline cplx toc(zc z) { return mkc(z.real(), z.imag()); }

}  // namespace

int qp_max_modes_impl(double om, double period) { return (int)std::floor(2.0 * om * period / (2.0 * M_PI)) + 2; }

struct QPPlan {
  int M = 0;
  double K = 0, h = 0, ca = 1, cb = 1, y0 = 0, gap = 0;
};

int qp_plan(const hbs_handle* h, double period, const qp_opts* o, QPPlan* p) {
  double maxx = 0, maxy = 0;
  for (int64_t i = 0; i < h->N; ++i) {
    maxx = std::max(maxx, std::fabs(h->hx[i]));
    maxy = std::max(maxy, std::fabs(h->hy[i]));
  }
  const int P = o->P;
  p->gap = (P + 0.5) * period - maxx;
  if (!(p->gap > 0)) {
    set_error("qp_solve: the obstacle reaches the unit-cell walls (period too small)");
    return HBS_E_INVALID_ARG;
  }
  p->h = o->h > 0 ? o->h : 0.1;
  p->K = o->K > 0 ? o->K : std::sqrt(h->omega * h->omega + std::pow(37.0 / p->gap, 2));
  p->M = o->M > 0 ? o->M : (int)std::ceil(2.0 * p->K / p->h);
  p->h = 2.0 * p->K / p->M;
  p->ca = o->ca > 0 ? o->ca : 1.0;
  p->cb = o->cb > 0 ? o->cb : 1.0;
  p->y0 = o->y0 > 0 ? o->y0 : maxy + 0.5;
  return HBS_OK;
}

int qp_contour_M(const hbs_handle* h, double period, const qp_opts* o) {
  QPPlan p;
  if (qp_plan(h, period, o, &p) != HBS_OK) return -1;
  return p.M;
}

// All outputs in "caller order"; eta/xi/bragg are device pointers here (the C ABI stages host copies).
int qp_solve_impl(hbs_handle* h, double period, const std::vector<double>& th, const qp_opts* o, cplx* eta_out,
                  cplx* xi_out, cplx* bragg_out, int32_t* nlo_out, int32_t* nm_out, double* flux_out) {
  hipStream_t st = h->stream;
  const int N = (int)h->N;
  const int nang = (int)th.size();
  const double om = h->omega;
  if (o->P != 0) {
    set_error("qp_solve: only P = 0 is supported by this build");
    return HBS_E_INVALID_ARG;
  }
  QPPlan pl;
  CR(qp_plan(h, period, o, &pl));
  const int M = pl.M, M2 = 2 * M, M4 = 4 * M;
  const double wood = o->wood_min_kn > 0 ? o->wood_min_kn : 0.75;
  // Bloch phases, Wood's check, grouping
  std::vector<zc> al(nang);
  for (int a = 0; a < nang; ++a) {
    const double kap = om * std::cos(th[a]);
    al[a] = std::exp(zc(0.0, kap * period));
    double mn = 1e300;
    const int n0 = (int)std::floor((-om - kap) * period / (2 * M_PI)) - 1;
    const int n1 = (int)std::ceil((om - kap) * period / (2 * M_PI)) + 1;
    for (int nn = n0; nn <= n1; ++nn) {
      const double kx = kap + 2 * M_PI * nn / period;
      mn = std::min(mn, std::sqrt(std::fabs(om * om - kx * kx)));
    }
    if (mn < wood) {
      set_error("qp_solve: angle " + std::to_string(th[a]) + " is within wood_min_kn of a Wood's anomaly");
      return HBS_E_WOOD;
    }
  }
  std::vector<int> grp(nang, -1);
  std::vector<zc> galpha;
  for (int a = 0; a < nang; ++a) {
    for (size_t g = 0; g < galpha.size(); ++g)
      if (std::abs(al[a] - galpha[g]) <= 1e-10) { grp[a] = (int)g; break; }
    if (grp[a] < 0) {
      grp[a] = (int)galpha.size();
      galpha.push_back(al[a]);
    }
  }
  const int ng = (int)galpha.size();
  std::vector<int> order;  // grouped position -> caller index
  std::vector<int> goff(ng + 1, 0), gcnt(ng, 0);
  for (int g = 0; g < ng; ++g) {
    for (int a = 0; a < nang; ++a)
      if (grp[a] == g) order.push_back(a);
    goff[g + 1] = (int)order.size();
    gcnt[g] = goff[g + 1] - goff[g];
  }
  // contour (Sec. 2.3): k(t) = t - i ca tanh(t/cb), trapezoid in t
  std::vector<cplx> cont(3 * M);
  for (int m = 0; m < M; ++m) {
    const double t = -pl.K + (m + 0.5) * pl.h;
    const zc k(t, -pl.ca * std::tanh(t / pl.cb));
    const double sech = 1.0 / std::cosh(t / pl.cb);
    const zc wk = pl.h * zc(1.0, -(pl.ca / pl.cb) * sech * sech);
    const zc s = std::sqrt(om * om - k * k);
    cont[m] = toc(k);
    cont[M + m] = toc(s);
    cont[2 * M + m] = toc(wk);
  }
  // per-angle data in grouped order
  std::vector<double> kx(nang), ky(nang), kapv(nang);
  std::vector<cplx> alcol(nang), galc(ng);
  std::vector<int> perm(nang), nlo(nang), nm(nang);
  const int maxm = qp_max_modes_impl(om, period);
  for (int q = 0; q < nang; ++q) {
    const int a = order[q];
    kx[q] = om * std::cos(th[a]);
    ky[q] = om * std::sin(th[a]);
    kapv[q] = kx[q];
    alcol[q] = toc(galpha[grp[a]]);
    perm[q] = a;
    const double kap = kx[q];
    nlo[q] = (int)std::ceil((-om - kap) * period / (2 * M_PI));
    int nhi = (int)std::floor((om - kap) * period / (2 * M_PI));
    nm[q] = std::min(maxm, nhi - nlo[q] + 1);
  }
  for (int g = 0; g < ng; ++g) galc[g] = toc(galpha[g]);

  // device workspace
  const int64_t W = (int64_t)M4 + nang;
  std::vector<size_t> sizes = {
      sizeof(cplx) * 3 * M,                 // 0 contour
      sizeof(double) * nang * 3,            // 1 kx, ky, kappa
      sizeof(cplx) * (nang + ng),           // 2 alpha per column, per group
      sizeof(int) * nang * 3,               // 3 perm, nlo, nmodes
      sizeof(cplx) * N * W,                 // 4 Y
      sizeof(cplx) * N * W,                 // 5 X
      sizeof(cplx) * (size_t)M2 * N * 2,    // 6 C_L, C_R
      sizeof(cplx) * (size_t)M2 * W * 2,    // 7 G1, G2
      sizeof(cplx) * (size_t)M2 * M2 * ng,  // 8 S
      sizeof(cplx) * (size_t)M2 * nang * 8, // 9 xi, W, T1, T2, R2, U1, U2, dxi
      sizeof(cplx) * (size_t)M4 * nang,     // 10 stack
      sizeof(cplx) * (size_t)N * nang * 4,  // 11 eta, F/R1, Z1, perm staging
      sizeof(cplx) * 2 * maxm * nang * 2,   // 12 bragg (grouped, caller order)
      sizeof(double) * nang * 3};           // 13 norms
  std::vector<size_t> off(sizes.size() + 1, 0);
  for (size_t i = 0; i < sizes.size(); ++i) off[i + 1] = off[i] + ((sizes[i] + 255) / 256) * 256;
  CK(h->scratch.reserve(off.back()));
  char* base = h->scratch.as<char>();
  cplx* dcont = (cplx*)(base + off[0]);
  double* dkx = (double*)(base + off[1]);
  double* dky = dkx + nang;
  double* dkap = dky + nang;
  cplx* dalcol = (cplx*)(base + off[2]);
  cplx* dgal = dalcol + nang;
  int* dperm = (int*)(base + off[3]);
  int* dnlo = dperm + nang;
  int* dnm = dnlo + nang;
  cplx* Y = (cplx*)(base + off[4]);
  cplx* X = (cplx*)(base + off[5]);
  cplx* CL = (cplx*)(base + off[6]);
  cplx* CRm = CL + (size_t)M2 * N;
  cplx* G1 = (cplx*)(base + off[7]);
  cplx* G2 = G1 + (size_t)M2 * W;
  cplx* S = (cplx*)(base + off[8]);
  cplx* xi = (cplx*)(base + off[9]);
  cplx* Wv = xi + (size_t)M2 * nang;
  cplx* T1 = Wv + (size_t)M2 * nang;
  cplx* T2 = T1 + (size_t)M2 * nang;
  cplx* R2 = T2 + (size_t)M2 * nang;
  cplx* U1 = R2 + (size_t)M2 * nang;
  cplx* U2 = U1 + (size_t)M2 * nang;
  cplx* dxi = U2 + (size_t)M2 * nang;
  cplx* stk = (cplx*)(base + off[10]);
  cplx* eta = (cplx*)(base + off[11]);
  cplx* R1 = eta + (size_t)N * nang;
  cplx* Z1 = R1 + (size_t)N * nang;
  cplx* F = Z1 + (size_t)N * nang;
  cplx* brg = (cplx*)(base + off[12]);
  cplx* brg2 = brg + (size_t)2 * maxm * nang;
  double* nrm = (double*)(base + off[13]);

  CK(hipMemcpyAsync(dcont, cont.data(), sizeof(cplx) * 3 * M, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dkx, kx.data(), sizeof(double) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dky, ky.data(), sizeof(double) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dkap, kapv.data(), sizeof(double) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dalcol, alcol.data(), sizeof(cplx) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dgal, galc.data(), sizeof(cplx) * ng, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dperm, perm.data(), sizeof(int) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dnlo, nlo.data(), sizeof(int) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dnm, nm.data(), sizeof(int) * nang, hipMemcpyHostToDevice, st));

  QPGeo Q;
  Q.x = h->geo.x; Q.y = h->geo.y; Q.nx = h->geo.nx; Q.ny = h->geo.ny; Q.w = h->geo.w;
  Q.k = dcont; Q.s = dcont + M; Q.wk = dcont + 2 * M;
  Q.N = N; Q.M = M; Q.omega = om; Q.period = period; Q.shift = 0.0;
  const cplx one = mkc(1, 0), zero = mkc(0, 0), mone = mkc(-1, 0);
  {
    ProfScope ps("assemble", st, 0.0, 0.0);
    CK(launch_gen_B(Q, Y, N, st));
    CK(launch_gen_inc(Q, dkx, dky, nang, Y + (size_t)M4 * N, N, st));
    CK(launch_gen_C(Q, 0, 0.0, CL, st));
    CK(launch_gen_C(Q, 1, 0.0, CRm, st));
  }
  // one application of A^{-1} for every alpha
  CR(apply_factors(h, true, Y, N, X, N, W));
  // alpha-free products C_L X, C_R X
  {
    std::vector<GemmDesc> g = {gd(CL, M2, 0, X, N, G1, M2, M2, (int)W, N, one, zero),
                               gd(CRm, M2, 0, X, N, G2, M2, M2, (int)W, N, one, zero)};
    CK(gemm_batched(h->arena, g, st, &h->splitws));
    CK(hipStreamSynchronize(st));
  }
  CK(launch_form_S(Q, dgal, ng, G1, G2, S, st));
  {
    std::vector<InvDesc> iv;
    for (int g = 0; g < ng; ++g) iv.push_back({S + (size_t)g * M2 * M2, M2, M2});
    bool sing = false;
    CK(inv_batched(h->arena, h->work, iv, st, &sing));
    if (sing) {
      set_error("qp_solve: singular Schur complement");
      return HBS_E_SINGULAR;
    }
  }
  // xi = -S^{-1} C(alpha) X_b
  CK(launch_combine_c(M2, nang, dalcol, G1 + (size_t)M4 * M2, M2, G2 + (size_t)M4 * M2, M2, nullptr, Wv, st));
  auto solve_S = [&](const cplx* rhs, cplx* out, cplx alpha) -> int {
    std::vector<GemmDesc> g;
    for (int gg = 0; gg < ng; ++gg)
      g.push_back(gd(S + (size_t)gg * M2 * M2, M2, 0, rhs + (size_t)goff[gg] * M2, M2, out + (size_t)goff[gg] * M2, M2, M2,
                     gcnt[gg], M2, alpha, zero));
    CK(gemm_batched(h->arena, g, st, &h->splitws));
    CK(hipStreamSynchronize(st));
    return HBS_OK;
  };
  CR(solve_S(Wv, xi, mone));
  // eta = X_b - [X_L | X_R] [xi; alpha xi]
  CK(launch_stack(M2, nang, dalcol, xi, stk, st));
  CK(launch_axpby(N, nang, one, X + (size_t)M4 * N, N, zero, eta, N, st));
  {
    std::vector<GemmDesc> g = {gd(X, N, 0, stk, M4, eta, N, N, nang, M4, mone, one)};
    CK(gemm_batched(h->arena, g, st, &h->splitws));
    CK(hipStreamSynchronize(st));
  }
  // iterative refinement of the bordered system
  int maxit = o->refine_max_iter < 0 ? 0 : (o->refine_max_iter == 0 ? 2 : o->refine_max_iter);
  const double rtol = o->refine_tol > 0 ? o->refine_tol : 1e-13;
  std::vector<double> hn(3 * nang);
  CK(launch_colnorm2(N, nang, Y + (size_t)M4 * N, N, nrm + 2 * nang, st));
  double relres = -1;
  int iters = 0;
  for (int it = 0; it <= maxit; ++it) {
    // R1 = b - A eta - B(alpha) xi ;  R2 = -C(alpha) eta - Q(alpha) xi
    CR(apply_factors(h, false, eta, N, F, N, nang));
    CK(launch_axpby(N, nang, one, Y + (size_t)M4 * N, N, zero, R1, N, st));
    CK(launch_axpby(N, nang, mone, F, N, one, R1, N, st));
    {
      std::vector<GemmDesc> g = {gd(Y, N, 0, stk, M4, R1, N, N, nang, M4, mone, one),
                                 gd(CL, M2, 0, eta, N, T1, M2, M2, nang, N, one, zero),
                                 gd(CRm, M2, 0, eta, N, T2, M2, M2, nang, N, one, zero)};
      CK(gemm_batched(h->arena, g, st, &h->splitws));
      CK(hipStreamSynchronize(st));
    }
    CK(launch_resid2(Q, nang, dalcol, T1, T2, xi, R2, st));
    CK(launch_colnorm2(N, nang, R1, N, nrm, st));
    CK(launch_colnorm2(M2, nang, R2, M2, nrm + nang, st));
    CK(hipMemcpyAsync(hn.data(), nrm, sizeof(double) * 3 * nang, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    relres = 0;
    for (int q = 0; q < nang; ++q) relres = std::max(relres, std::sqrt((hn[q] + hn[nang + q]) / hn[2 * nang + q]));
    if (relres < rtol || it == maxit) break;
    ++iters;
    // correction by the block solve: Z1 = A^{-1} R1; dxi = S^{-1}(R2 - C(alpha) Z1); deta = Z1 - X(alpha) dxi
    CR(apply_factors(h, true, R1, N, Z1, N, nang));
    {
      std::vector<GemmDesc> g = {gd(CL, M2, 0, Z1, N, U1, M2, M2, nang, N, one, zero),
                                 gd(CRm, M2, 0, Z1, N, U2, M2, M2, nang, N, one, zero)};
      CK(gemm_batched(h->arena, g, st, &h->splitws));
      CK(hipStreamSynchronize(st));
    }
    CK(launch_combine_c(M2, nang, dalcol, U1, M2, U2, M2, R2, Wv, st));
    CR(solve_S(Wv, dxi, one));
    CK(launch_stack(M2, nang, dalcol, dxi, stk, st));
    CK(launch_axpby(N, nang, one, Z1, N, one, eta, N, st));
    {
      std::vector<GemmDesc> g = {gd(X, N, 0, stk, M4, eta, N, N, nang, M4, mone, one)};
      CK(gemm_batched(h->arena, g, st, &h->splitws));
      CK(hipStreamSynchronize(st));
    }
    CK(launch_axpby(M2, nang, one, dxi, M2, one, xi, M2, st));
    CK(launch_stack(M2, nang, dalcol, xi, stk, st));
  }
  h->stats.refine_iters = iters;
  h->stats.refine_residual = relres;
  h->stats.contour_M = M;
  if (maxit > 0 && relres >= rtol && relres > 1e-8) {
    set_error("qp_solve: refinement stalled at relative residual " + std::to_string(relres));
    return HBS_E_NOT_CONVERGED;
  }
  // Bragg amplitudes
  {
    ProfScope ps("bragg", st, 0.0, 0.0);
    CK(launch_bragg(Q, dkap, dnlo, dnm, maxm, nang, eta, N, pl.y0, brg, st));
  }
  // outputs in caller order
  CK(launch_permute_cols(N, nang, dperm, eta, N, eta_out, N, st));
  if (xi_out) CK(launch_permute_cols(M2, nang, dperm, xi, M2, xi_out, M2, st));
  CK(launch_permute_cols(2 * maxm, nang, dperm, brg, 2 * maxm, brg2, 2 * maxm, st));
  if (bragg_out) CK(hipMemcpyAsync(bragg_out, brg2, sizeof(cplx) * 2 * maxm * nang, hipMemcpyDeviceToDevice, st));
  std::vector<cplx> hb((size_t)2 * maxm * nang);
  CK(hipMemcpyAsync(hb.data(), brg2, sizeof(cplx) * hb.size(), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  // flux error (Remark 6.1): |sum_prop k_n (|c_n|^2 + |d_n|^2) with d_0 -> d_0 + e^{i k_0 y0}, minus k_0| / k_0
  for (int q = 0; q < nang; ++q) {
    const int a = order[q];
    if (nlo_out) nlo_out[a] = nlo[q];
    if (nm_out) nm_out[a] = nm[q];
    if (!flux_out) continue;
    const double kap = kx[q];
    const double k0 = std::sqrt(std::max(om * om - kap * kap, 0.0));
    double fl = 0;
    const cplx* col = hb.data() + (size_t)a * 2 * maxm;
    for (int j = 0; j < nm[q]; ++j) {
      const int nn = nlo[q] + j;
      const double kxn = kap + 2 * M_PI * nn / period;
      const double kn = std::sqrt(std::max(om * om - kxn * kxn, 0.0));
      zc c(col[j].x, col[j].y), d(col[maxm + j].x, col[maxm + j].y);
      if (nn == 0) d += std::exp(zc(0.0, k0 * pl.y0));
      fl += kn * (std::norm(c) + std::norm(d));
    }
    flux_out[a] = std::fabs(fl - k0) / k0;
  }
  return HBS_OK;
}

}  // namespace qps
