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

int qp_plan_y0(const hbs_handle* h, double period, const qp_opts* o, double* K, double* y0, int* M) {
  QPPlan p;
  const int rc = qp_plan(h, period, o, &p);
  if (rc != HBS_OK) return rc;
  *K = p.K;
  *y0 = p.y0;
  *M = p.M;
  return HBS_OK;
}

int qp_contour_M(const hbs_handle* h, double period, const qp_opts* o) {
  QPPlan p;
  if (qp_plan(h, period, o, &p) != HBS_OK) return -1;
  return p.M;
}

// All outputs in "caller order"; eta/xi/bragg are device pointers here (the C ABI stages host copies).
//
// With P neighbour images (Sec. 2.4) the obstacle block is A~(alpha) = A + sum_{j=+-1} alpha^j A_j.  The
// skeletons of a handle built with far_radius represent the interaction of every box with sources
// beyond that radius, and with image_period also with the images' near points (Sec. 3.2), so the rows
// of A_j factor through the nested interpolation U of the tree:
// A_j = U A_j(J, :) with J the root's active set.  Then A~ = A + U R(alpha), R = alpha R_1 + alpha^{-1} R_{-1},
// and (Eq. 3.2 with the sign of its second term corrected)
//   A~^{-1} = A^{-1} - V K R A^{-1},  V = A^{-1} U,  K(alpha) = (I + R V)^{-1}  (root-size),
// where V joins the single application of A^{-1}.  C~(alpha) = alpha^P C_L[dOmega + P d] - alpha^{-(P+1)} C_R[dOmega - P d].
//
// cols (nullable): the columns are not incident angles but the given plane waves
// -exp(i (kx x + ky y)) (ky complex), all with the Bloch phase cols->alpha, solved on the contour
// whose real-axis crossing is displaced to cols->delta (the Wood's-anomaly scheme); th is ignored.
int qp_solve_core(hbs_handle* h, double period, const std::vector<double>& th, const qp_opts* o, const QPCols* cols,
                  cplx* eta_out, cplx* xi_out, cplx* bragg_out, int32_t* nlo_out, int32_t* nm_out, double* flux_out) {
  hipStream_t st = h->stream;
  const int N = (int)h->NU;  // length of the obstacle's vectors (two unknowns per node: transmission)
  const int nang = cols ? (int)cols->kx.size() : (int)th.size();
  const double om = h->omega;
  const int P = o->P;
  if (P != 0 && P != 1) {
    set_error("qp_solve: P must be 0 or 1");
    return HBS_E_INVALID_ARG;
  }
  if (h->nc != 1 && cols) {
    set_error("qp_solve: the transmission problem has no displaced-contour solve");
    return HBS_E_INVALID_ARG;
  }
  if (P == 1) {
    if (!(h->opts.far_radius > 0)) {
      set_error("qp_solve: P = 1 needs a handle built with hbs_opts.far_radius > 0");
      return HBS_E_INVALID_ARG;
    }
    // images inside far_radius are represented only by a handle built with their explicit columns
    const bool imgs = h->opts.image_period > 0 && std::fabs(h->opts.image_period - period) <= 1e-12 * period;
    if (!imgs && !(period - h->robs > h->opts.far_radius)) {
      set_error("qp_solve: the neighbour images come closer than far_radius to the obstacle's centre "
                "(build the handle with hbs_opts.image_period = period)");
      return HBS_E_INVALID_ARG;
    }
  }
  // wall blocks through the root skeletons: needs every wall outside the far-field circle
  const bool far_ok = h->opts.far_radius > 0 && 0.5 * period - std::fabs(h->c0x) >= h->opts.far_radius;
  if (o->compress_walls > 0 && !far_ok) {
    set_error("qp_solve: compress_walls needs a handle whose far_radius circle excludes the walls");
    return HBS_E_INVALID_ARG;
  }
  // the transmission operator takes its wall blocks through the skeletons only on request: there they
  // carry the decompositions' error about 3e3 times over (against about 10 for the Dirichlet operator)
  const bool cw = (h->nc == 1 ? o->compress_walls >= 0 : o->compress_walls > 0) && far_ok;
  // compress_walls = 2: the solve as with 1, the refinement's residual with the uncompressed wall
  // blocks (formed in full), so that the corrections remove the error the skeletons give B and C
  // (the displaced-contour columns take 1)
  const bool xw = cw && o->compress_walls == 2 && !cols && o->refine_max_iter >= 0;
  QPPlan pl;
  CR(qp_plan(h, period, o, &pl));
  const int M = pl.M, M2 = 2 * M, M4 = 4 * M;
  const int nr = P ? h->nroot : 0;       // Woodbury size
  const int nu = (P || cw) ? h->nroot : 0;  // columns of the nested interpolation U
  const double wood = o->wood_min_kn > 0 ? o->wood_min_kn : 0.75;
  // Bloch phases, Wood's check, grouping
  std::vector<zc> al(nang);
  for (int a = 0; a < nang && cols; ++a) al[a] = cols->alpha;
  for (int a = 0; a < nang && !cols; ++a) {
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
  // Angles share a group (and its alpha in the alpha-dependent blocks) only when their Bloch phases
  // agree to the rounding of omega d cos(theta): a few ulps of a phase of size omega d.
  const double gtol = 32.0 * 2.220446049250313e-16 * std::max(1.0, om * period);
  std::vector<int> grp(nang, -1);
  std::vector<zc> galpha;
  for (int a = 0; a < nang; ++a) {
    for (size_t g = 0; g < galpha.size(); ++g)
      if (std::abs(al[a] - galpha[g]) <= gtol) { grp[a] = (int)g; break; }
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
  // (displaced: k(t) = t - i ca tanh((t - delta)/cb), crossing the real axis at delta)
  const double cdel = cols ? cols->delta : 0.0;
  for (int m = 0; m < M; ++m) {
    const double t = -pl.K + (m + 0.5) * pl.h;
    const zc k(t, -pl.ca * std::tanh((t - cdel) / pl.cb));
    const double sech = 1.0 / std::cosh((t - cdel) / pl.cb);
    const zc wk = pl.h * zc(1.0, -(pl.ca / pl.cb) * sech * sech);
    const zc s = std::sqrt(om * om - k * k);
    cont[m] = toc(k);
    cont[M + m] = toc(s);
    cont[2 * M + m] = toc(wk);
  }
  // per-angle data in grouped order; C~(alpha) = c1 C1 + c2 C2 with c1 = alpha^P, c2 = -alpha^{-(P+1)}
  std::vector<double> kx(nang), ky(nang), kyi(nang, 0.0);
  std::vector<cplx> colc(5 * nang), gcoef(3 * ng + 4 * ng);
  std::vector<int> perm(nang), nlo(nang), nm(nang);
  const int maxm = qp_max_modes_impl(om, period);
  auto c1_of = [&](zc a) { return P ? a : zc(1.0, 0.0); };
  auto c2_of = [&](zc a) { return -std::pow(a, -(P + 1)); };
  for (int q = 0; q < nang; ++q) {
    const int a = order[q];
    const zc ag = galpha[grp[a]];
    kx[q] = cols ? cols->kx[a] : om * std::cos(th[a]);
    ky[q] = cols ? cols->ky[a].real() : om * std::sin(th[a]);
    kyi[q] = cols ? cols->ky[a].imag() : 0.0;
    colc[q] = toc(ag);                        // alpha
    colc[nang + q] = toc(c1_of(ag));          // c1
    colc[2 * nang + q] = toc(c2_of(ag));      // c2
    colc[3 * nang + q] = toc(1.0 / ag);       // alpha^{-1}
    colc[4 * nang + q] = toc(-ag);            // -alpha (for in-place subtractions)
    perm[q] = a;
    const double kap = kx[q];
    nlo[q] = (int)std::ceil((-om - kap) * period / (2 * M_PI));
    int nhi = (int)std::floor((om - kap) * period / (2 * M_PI));
    nm[q] = std::min(maxm, nhi - nlo[q] + 1);
  }
  for (int g = 0; g < ng; ++g) {
    const zc ag = galpha[g];
    gcoef[3 * g] = toc(ag);
    gcoef[3 * g + 1] = toc(c1_of(ag));
    gcoef[3 * g + 2] = toc(c2_of(ag));
    // per-group scalars for the neighbour terms: alpha, alpha^{-1}, alpha^2, -alpha
    gcoef[3 * ng + 4 * g] = toc(ag);
    gcoef[3 * ng + 4 * g + 1] = toc(1.0 / ag);
    gcoef[3 * ng + 4 * g + 2] = toc(ag * ag);
    gcoef[3 * ng + 4 * g + 3] = toc(-ag);
  }
  const cplx onec = mkc(1, 0), minus1c = mkc(-1, 0);

  // device workspace.  G1, G2 and R_{+-1} X use the column layout [L | R | b | U] of width W; Y and X
  // hold [B_L | B_R | b | U] (uncompressed walls) or [U | b] (compressed walls).
  const int64_t W = (int64_t)M4 + nang + nr;
  const int colB = M4, colU = M4 + nang;
  const int64_t Wy = cw ? (int64_t)nu + nang : W;
  const int ycolB = cw ? nu : M4, ycolU = cw ? 0 : M4 + nang;
  const int64_t NC = cw ? nu : N;  // columns of C1, C2
  const int nrr = std::max(nr, 1);
  const int nuu = std::max(nu, 1);
  std::vector<size_t> sizes = {
      sizeof(cplx) * 3 * M,                          // 0 contour
      sizeof(double) * nang * 4,                     // 1 kx, ky, kappa, Im ky
      sizeof(cplx) * (5 * nang + 7 * ng + 2),        // 2 column and group coefficients, constants
      sizeof(int) * nang * 3,                        // 3 perm, nlo, nmodes
      sizeof(cplx) * N * Wy,                         // 4 Y
      sizeof(cplx) * N * Wy,                         // 5 X
      sizeof(cplx) * (size_t)M2 * NC * 2,            // 6 C1, C2
      sizeof(cplx) * (size_t)M2 * W * 2,             // 7 G1, G2
      cw ? 0 : sizeof(cplx) * (size_t)M2 * M2 * ng, // 8 S (uncompressed walls)
      sizeof(cplx) * (size_t)M2 * nang * 8,          // 9 xi, W, T1, T2, R2, U1, U2, dxi
      sizeof(cplx) * (size_t)M4 * nang,              // 10 stack
      sizeof(cplx) * (size_t)N * nang * 4,           // 11 eta, R1, Z1, F
      sizeof(cplx) * 2 * maxm * nang * 2,            // 12 bragg (grouped, caller order)
      sizeof(double) * nang * 3,                     // 13 norms
      sizeof(cplx) * (size_t)nr * N * 2,             // 14 R_{+1}, R_{-1}
      sizeof(cplx) * (size_t)nr * W * 2,             // 15 R_{+1} X, R_{-1} X
      sizeof(cplx) * (size_t)nrr * nrr * ng * 2,     // 16 K(alpha) (and I + R V)
      sizeof(cplx) * (size_t)nrr * M2 * ng * 2,      // 17 R(alpha) X(alpha), K R X scratch
      sizeof(cplx) * (size_t)M2 * nrr * ng,          // 18 C~ V
      sizeof(cplx) * (size_t)nrr * nang * 4,         // 19 R b, u, y, misc (nr x nang)
      cw ? sizeof(cplx) * ((size_t)nuu * (M4 + W + Wy + 2 * nang) + (size_t)nr * Wy * 2 + (size_t)N * nang) : 0,
                                                     // 20 B_J, X_c, U^T X, t1, t2, R_{+-1} X, U t
      cw ? sizeof(cplx) * ((size_t)ng * (2 * (size_t)nuu * M2 + 3 * (size_t)nuu * nuu) + 3 * (size_t)M2 * nuu +
                           (size_t)M2 * nang + 2 * (size_t)nuu * nang) : 0,
                                                     // 21 Woodbury form of S^{-1}: B_J(alpha), Q^{-1} C~ H~, K2, H~,
                                                     //    scratch; C~_J H~; Q^{-1} r; two nu x nang
      xw ? sizeof(cplx) * ((size_t)N * M4 + (size_t)M2 * N * 2) : 0};
                                                     // 22 the uncompressed [B_L | B_R], C1, C2 of the residual
  std::vector<size_t> off(sizes.size() + 1, 0);
  for (size_t i = 0; i < sizes.size(); ++i) off[i + 1] = off[i] + ((sizes[i] + 255) / 256) * 256;
  CK(h->scratch.reserve(off.back()));
  char* base = h->scratch.as<char>();
  cplx* dcont = (cplx*)(base + off[0]);
  double* dkx = (double*)(base + off[1]);
  double* dky = dkx + nang;
  double* dkap = dky + nang;
  double* dkyi = cols ? dkap + nang : nullptr;
  cplx* dcol = (cplx*)(base + off[2]);
  cplx* d_al = dcol;
  cplx* d_c1 = dcol + nang;
  cplx* d_c2 = dcol + 2 * nang;
  cplx* d_ainv = dcol + 3 * nang;
  cplx* d_gco = dcol + 5 * nang;         // 3 ng: (alpha, c1, c2)
  cplx* d_gsc = d_gco + 3 * ng;           // 4 ng: (alpha, 1/alpha, alpha^2, -alpha)
  cplx* d_one = d_gsc + 4 * ng;           // constants 1, -1
  int* dperm = (int*)(base + off[3]);
  int* dnlo = dperm + nang;
  int* dnm = dnlo + nang;
  cplx* Y = (cplx*)(base + off[4]);
  cplx* X = (cplx*)(base + off[5]);
  cplx* C1 = (cplx*)(base + off[6]);
  cplx* C2 = C1 + (size_t)M2 * NC;
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
  cplx* Rp = (cplx*)(base + off[14]);
  cplx* Rm = Rp + (size_t)nr * N;
  cplx* RXp = (cplx*)(base + off[15]);
  cplx* RXm = RXp + (size_t)nr * W;
  cplx* Kg = (cplx*)(base + off[16]);
  cplx* KVg = Kg + (size_t)nrr * nrr * ng;
  cplx* RAX = (cplx*)(base + off[17]);
  cplx* KRAX = RAX + (size_t)nrr * M2 * ng;
  cplx* CV = (cplx*)(base + off[18]);
  cplx* Rb = (cplx*)(base + off[19]);
  cplx* uu = Rb + (size_t)nrr * nang;
  cplx* yy = uu + (size_t)nrr * nang;
  cplx* vv = yy + (size_t)nrr * nang;
  cplx* BJ = (cplx*)(base + off[20]);       // nu x 4M: [B_L | B_R](J, :)
  cplx* Xc = BJ + (size_t)nuu * M4;         // nu x W: U^T [X_L | X_R | X_b | V]
  cplx* Zt = Xc + (size_t)nuu * W;          // nu x Wy: U^T X
  cplx* t1 = Zt + (size_t)nuu * Wy;         // nu x nang
  cplx* t2 = t1 + (size_t)nuu * nang;       // nu x nang
  cplx* RZp = t2 + (size_t)nuu * nang;      // nr x Wy
  cplx* RZm = RZp + (size_t)nr * Wy;        // nr x Wy
  cplx* tN = RZm + (size_t)nr * Wy;         // N x nang
  cplx* BJa = (cplx*)(base + off[21]);      // per group nu x 2M: B_J,L + alpha B_J,R
  cplx* Cq = BJa + (size_t)ng * nuu * M2;   // per group 2M x nu: Q^{-1} C~_J H~
  cplx* K2 = Cq + (size_t)ng * nuu * M2;    // per group nu x nu: (I - B_J(alpha) Cq)^{-1}
  cplx* Ht = K2 + (size_t)ng * nuu * nuu;   // per group nu x nu: U^T A~^{-1} U
  cplx* Hs = Ht + (size_t)ng * nuu * nuu;   // per group nu x nu scratch
  cplx* CH = Hs + (size_t)ng * nuu * nuu;   // 2M x nu
  cplx* C1H = CH + (size_t)M2 * nuu;        // 2M x nu: C1_J H (shared by the phases when P = 0)
  cplx* C2H = C1H + (size_t)M2 * nuu;       // 2M x nu: C2_J H
  cplx* yq = C2H + (size_t)M2 * nuu;        // 2M x nang
  cplx* zq = yq + (size_t)M2 * nang;        // nu x nang
  cplx* zq2 = zq + (size_t)nuu * nang;      // nu x nang
  cplx* Yx = xw ? (cplx*)(base + off[22]) : nullptr;  // N x 4M: [B_L | B_R]
  cplx* C1x = xw ? Yx + (size_t)N * M4 : nullptr;      // 2M x N
  cplx* C2x = xw ? C1x + (size_t)M2 * N : nullptr;     // 2M x N

  std::vector<cplx> consts = {onec, minus1c};
  CK(hipMemcpyAsync(dcont, cont.data(), sizeof(cplx) * 3 * M, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dkx, kx.data(), sizeof(double) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dky, ky.data(), sizeof(double) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dkap, kx.data(), sizeof(double) * nang, hipMemcpyHostToDevice, st));
  if (dkyi) CK(hipMemcpyAsync(dkyi, kyi.data(), sizeof(double) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dcol, colc.data(), sizeof(cplx) * 5 * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(d_gco, gcoef.data(), sizeof(cplx) * 7 * ng, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(d_one, consts.data(), sizeof(cplx) * 2, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dperm, perm.data(), sizeof(int) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dnlo, nlo.data(), sizeof(int) * nang, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dnm, nm.data(), sizeof(int) * nang, hipMemcpyHostToDevice, st));

  QPGeo Q{};
  Q.two = h->nc == 2;
  Q.kb = h->geo.kbar;
  Q.x = h->geo.x; Q.y = h->geo.y; Q.nx = h->geo.nx; Q.ny = h->geo.ny; Q.w = h->geo.w;
  Q.k = dcont; Q.s = dcont + M; Q.wk = dcont + 2 * M;
  Q.N = (int)h->N; Q.M = M; Q.omega = om; Q.period = period; Q.shift = 0.0;
  Q.idx = nullptr;
  const int* J = h->lv[1].skel.as<int>();  // the root's active set (nroot nodes)
  QPGeo QJ = Q;
  QJ.idx = J;
  QJ.N = nu;
  const cplx zero = mkc(0, 0);
  // batched GEMMs are stream-ordered with the surrounding kernels; the host waits only where it
  // reads results back
  auto gemm = [&](const std::vector<GemmDesc>& g) -> int {
    CK(gemm_batched(h->arena, g, st, &h->splitws));
    return HBS_OK;
  };
  // the side stream (when used) is joined before returning, also on error paths
  struct SideJoin {
    hipStream_t s = nullptr;
    ~SideJoin() {
      if (s) (void)hipStreamSynchronize(s);
    }
  } side_join;
  // an early return after the side stream took the deferred root inversion: read its flag (after the
  // side stream is joined) so that later calls see the root's state
  struct RootSettle {
    hbs_handle* h;
    ~RootSettle() {
      if (h->root_state != 2) return;
      int f = 1;
      if (hipStreamSynchronize(h->side_stream) == hipSuccess &&
          hipMemcpy(&f, h->root_flag, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess)
        h->root_state = f ? 3 : 0;
      else
        h->root_state = 3;
    }
  } root_settle{h};
  // S(alpha) = Q - C~_J(alpha) H~(alpha) B_J(alpha) with H~ = U^T A~^{-1} U = H - H K(alpha) R(alpha) V (P = 1) or H;
  // Woodbury around the 2 x 2-block-diagonal Q: S^{-1} = [I + Cq K2 B_J(alpha)] Q^{-1},
  // Cq = Q^{-1} C~_J H~, K2 = (I - B_J(alpha) Cq)^{-1}  (root-size inversions only).
  // Issued on stream s with its own descriptor arena and workspaces.
  // dinfo: leave the singularity check to the caller (device flags in wk) instead of waiting
  // With the root inverse still to be formed (hbs_opts.defer_root), P = 0: H = R^{-1} and
  //   Cq K2 = Q^{-1} C~_J H (I - B_J Q^{-1} C~_J H)^{-1} = Q^{-1} C~_J (R - B_J Q^{-1} C~_J)^{-1},
  // so Cq = Q^{-1} C~_J and K2 = (R - B_J Cq)^{-1} give the same S^{-1} without R^{-1}, and R itself
  // joins the capacitance matrices in one batched inversion.
  auto woodbury = [&](hipStream_t s, DevBuf& ar, DevBuf& ws, DevBuf& wk, int** dinfo, bool defer) -> int {
    const cplx* H = Zt;  // U^T V (nu x nu)
    // every descriptor set first, so that the arena and workspaces are reserved before any launch
    std::vector<GemmDesc> gp1, gp2, gch, gbc;
    std::vector<std::vector<GemmDesc>> gcq(P ? ng : 0);
    std::vector<InvDesc> iv;
    for (int g = 0; g < ng; ++g) {
      if (P) {
        gp1.push_back(gd(Kg + (size_t)g * nr * nr, nr, 0, KVg + (size_t)g * nr * nr, nr, Hs + (size_t)g * nu * nu, nu, nu, nu,
                         nr, onec, zero));
        gp2.push_back(gd(H, nu, 0, Hs + (size_t)g * nu * nu, nu, Ht + (size_t)g * nu * nu, nu, nu, nu, nu, minus1c, onec));
        gcq[g] = {gd(Cq + (size_t)g * M2 * nu, M2, 0, Ht + (size_t)g * nu * nu, nu, CH, M2, M2, nu, nu, onec, zero)};
      }
      gbc.push_back(gd(BJa + (size_t)g * nu * M2, nu, 0, Cq + (size_t)g * M2 * nu, M2, Hs + (size_t)g * nu * nu, nu, nu, nu, M2,
                       minus1c, zero));
      iv.push_back({K2 + (size_t)g * nu * nu, nu, nu});
    }
    if (!P && !defer)
      gch = {gd(C1, M2, 0, H, nu, C1H, M2, M2, nu, nu, onec, zero), gd(C2, M2, 0, H, nu, C2H, M2, M2, nu, nu, onec, zero)};
    if (defer) iv.push_back({h->Rinv.as<cplx>(), nu, nu});
    {
      size_t amax = 0, wmax = 0, a, w;
      auto need = [&](const std::vector<GemmDesc>& v) {
        gemm_batched_needs(v, &a, &w);
        amax = std::max(amax, a);
        wmax = std::max(wmax, w);
      };
      need(gp1);
      need(gp2);
      need(gch);
      need(gbc);
      for (const auto& v : gcq) need(v);
      size_t wi;
      inv_batched_needs(iv, &a, &wi);
      CK(ar.reserve(std::max(amax, a)));
      if (wmax) CK(ws.reserve(wmax));
      CK(wk.reserve(wi));
    }
    auto gemm_s = [&](const std::vector<GemmDesc>& g) -> int {
      CK(gemm_batched(ar, g, s, &ws));
      return HBS_OK;
    };
    for (int g = 0; g < ng; ++g) {
      CK(launch_lincomb(nu, M2, d_one, d_gco + 3 * g, 0, BJ, nu, BJ + (size_t)M2 * nu, nu, nullptr, 0,
                        BJa + (size_t)g * nu * M2, nu, s));
    }
    if (P) {
      CR(gemm_s(gp1));
      for (int g = 0; g < ng; ++g)
        CK(hipMemcpyAsync(Ht + (size_t)g * nu * nu, H, sizeof(cplx) * (size_t)nu * nu, hipMemcpyDeviceToDevice, s));
      CR(gemm_s(gp2));
      for (int g = 0; g < ng; ++g) {
        // C~_J(alpha) = c1 C1_J + c2 C2_J (staged in Cq), then Cq = Q^{-1} C~_J H~
        cplx* cq = Cq + (size_t)g * M2 * nu;
        CK(launch_lincomb(M2, nu, d_gco + 3 * g + 1, d_gco + 3 * g + 2, 0, C1, M2, C2, M2, nullptr, 0, cq, M2, s));
        CR(gemm_s(gcq[g]));
        CK(launch_qsolve(Q, d_gco + 3 * g, 0, nu, CH, M2, cq, M2, s));
      }
    } else if (defer) {
      // Cq = Q^{-1} (c1 C1_J + c2 C2_J)
      for (int g = 0; g < ng; ++g) {
        cplx* cq = Cq + (size_t)g * M2 * nu;
        CK(launch_lincomb(M2, nu, d_gco + 3 * g + 1, d_gco + 3 * g + 2, 0, C1, M2, C2, M2, nullptr, 0, CH, M2, s));
        CK(launch_qsolve(Q, d_gco + 3 * g, 0, nu, CH, M2, cq, M2, s));
      }
    } else {
      // H~ = H for every phase: C~_J H = c1 (C1_J H) + c2 (C2_J H)
      CR(gemm_s(gch));
      for (int g = 0; g < ng; ++g) {
        cplx* cq = Cq + (size_t)g * M2 * nu;
        CK(launch_lincomb(M2, nu, d_gco + 3 * g + 1, d_gco + 3 * g + 2, 0, C1H, M2, C2H, M2, nullptr, 0, CH, M2, s));
        CK(launch_qsolve(Q, d_gco + 3 * g, 0, nu, CH, M2, cq, M2, s));
      }
    }
    CR(gemm_s(gbc));
    if (defer) {
      // K2 = R + Hs = R - B_J Cq, the root matrix still in Rinv
      for (int g = 0; g < ng; ++g)
        CK(launch_lincomb(nu, nu, d_one, d_one, 0, h->Rinv.as<cplx>(), nu, Hs + (size_t)g * nu * nu, nu, nullptr, 0,
                          K2 + (size_t)g * nu * nu, nu, s));
    } else {
      CK(launch_eye_plus(nu, ng, Hs, nu, (int64_t)nu * nu, K2, s));
    }
    if (dinfo) {
      CK(inv_batched_async(ar, wk, iv, s, dinfo));
      if (defer) {
        h->root_flag = *dinfo + ng;
        h->root_state = 2;
      }
      return HBS_OK;
    }
    bool sing = false;
    CK(inv_batched(ar, wk, iv, s, &sing));
    if (sing) {
      set_error("qp_solve: singular Schur complement");
      return HBS_E_SINGULAR;
    }
    return HBS_OK;
  };
  {
    ProfScope ps("assemble", st, 0.0, 0.0);
    if (cw) {
      // only the skeleton rows of B and the skeleton columns of C are needed
      CK(launch_gen_B(QJ, BJ, nu, st));
      CK(launch_gen_C(QJ, 0, P * period, C1, st));
      CK(launch_gen_C(QJ, 1, -P * period, C2, st));
      if (xw) {
        CK(launch_gen_B(Q, Yx, N, st));
        CK(launch_gen_C(Q, 0, P * period, C1x, st));
        CK(launch_gen_C(Q, 1, -P * period, C2x, st));
      }
    } else {
      CK(launch_gen_B(Q, Y, N, st));
      CK(launch_gen_C(Q, 0, P * period, C1, st));
      CK(launch_gen_C(Q, 1, -P * period, C2, st));
    }
    CK(launch_gen_inc(Q, dkx, dky, dkyi, nang, Y + (size_t)ycolB * N, N, st));
  }
  // compressed walls on complex128 factors: V = A^{-1} U and U^T A^{-1} [U | b] come from the
  // root inverse and the E-only downward pass, without forming U (F^T P = I, G P = 0, P^T E = I)
  const bool fastU = cw && h->fp64_top >= h->L;
  // without neighbour images the Woodbury factors need only R^{-1}, B_J and C_J: they are formed on
  // the side stream while the main stream applies A^{-1} to the incident fields
  const bool overlap = fastU && !P;
  // a deferred root inversion joins the side stream's capacitance inversions (graph capture cannot
  // take the cross-stream wait of the root product)
  const bool defer = overlap && h->root_state == 1 && !h->opts.graph;
  if (!defer) CR(ensure_root(h));
  int* side_dinfo = nullptr;  // the side stream's singularity flags (device)
  if (nu && !fastU) {
    // U (N x nroot) = nested interpolation of the identity
    CK(h->ab_root.reserve(sizeof(cplx) * (size_t)nu * nu));
    std::vector<cplx> eye((size_t)nu * nu, zero);
    for (int i = 0; i < nu; ++i) eye[(size_t)i * nu + i] = onec;
    CK(hipMemcpyAsync(h->ab_root.p, eye.data(), sizeof(cplx) * eye.size(), hipMemcpyHostToDevice, st));
    CR(apply_interp(h, h->ab_root.as<cplx>(), nu, Y + (size_t)ycolU * N, N, nu));
  }
  if (P) {
    // R_{+-1} = A_{+-1}(J, :)
    CK(launch_eval_shift(h->geo, J, nr, period, Rp, nr, st));
    CK(launch_eval_shift(h->geo, J, nr, -period, Rm, nr, st));
  }
  const bool fp32 = h->opts.precision == HBS_FP32_PRECOND;
  if (cw) {
    // one application of A^{-1} to [U | b]: X = [V | X_b]; then with H = U^T V,
    //   U^T [X_L | X_R | X_b | V] = [H B_J,L | H B_J,R | U^T X_b | H]  and  G = C_J (that)
    if (fastU) {
      if (!defer) CK(hipMemcpyAsync(Zt, h->Rinv.p, sizeof(cplx) * (size_t)nu * nu, hipMemcpyDeviceToDevice, st));
      if (overlap) {
        // the side stream waits for R^{-1} and the wall blocks and forms the Woodbury factors while
        // the main stream applies A^{-1}; the main stream waits for them before the first solve with S
        CR(side_stream_init(h));
        CK(hipEventRecord(h->side_ev[0], st));
        side_join.s = h->side_stream;
        CK(hipStreamWaitEvent(h->side_stream, h->side_ev[0], 0));
        CR(woodbury(h->side_stream, h->arena_s, h->splitws_s, h->work_s, &side_dinfo, defer));
        CK(hipEventRecord(h->side_ev[1], h->side_stream));
      }
      if (overlap) {
        // only the upward pass and the root now: eta comes from one downward pass once xi is known
        // (a deferred root inverse: the root product waits for the side stream's batched inversion)
        CR(apply_inverse_up(h, Y + (size_t)ycolB * N, N, nang, Zt + (size_t)nu * nu, nu, defer ? h->side_ev[1] : nullptr));
        if (defer) CK(hipMemcpyAsync(Zt, h->Rinv.p, sizeof(cplx) * (size_t)nu * nu, hipMemcpyDeviceToDevice, st));
      } else {
        CR(apply_inverse_root(h, Y + (size_t)ycolB * N, N, X + (size_t)ycolB * N, N, nang, Zt + (size_t)nu * nu, nu));
      }
      // V itself is needed only with neighbour images; without them X(alpha) xi = V (B_J v) is
      // applied as E_L ... E_1 (R^{-1} B_J v) where needed
      if (P) CR(apply_down_E(h, Zt, nu, X + (size_t)ycolU * N, N, nu));
    } else {
      CR(apply_factors(h, true, Y, N, X, N, Wy));
      CR(apply_interp_t(h, X, N, Zt, nu, Wy));
    }
    // the Woodbury form of S^{-1} uses only the b (and U) columns of C [X_L | X_R | X_b | V]:
    // G[:, b | U] = C_J [U^T X_b | H]
    CK(hipMemcpyAsync(Xc + (size_t)colB * nu, Zt + (size_t)nu * nu, sizeof(cplx) * (size_t)nu * nang,
                      hipMemcpyDeviceToDevice, st));
    if (P) CK(hipMemcpyAsync(Xc + (size_t)colU * nu, Zt, sizeof(cplx) * (size_t)nu * nu, hipMemcpyDeviceToDevice, st));
    const int wbu = nang + nr;
    std::vector<GemmDesc> g = {gd(C1, M2, 0, Xc + (size_t)colB * nu, nu, G1 + (size_t)colB * M2, M2, M2, wbu, nu, onec, zero),
                               gd(C2, M2, 0, Xc + (size_t)colB * nu, nu, G2 + (size_t)colB * M2, M2, M2, wbu, nu, onec, zero)};
    if (P) {
      g.push_back(gd(Rp, nr, 0, X, N, RZp, nr, nr, (int)Wy, N, onec, zero));
      g.push_back(gd(Rm, nr, 0, X, N, RZm, nr, nr, (int)Wy, N, onec, zero));
    }
    CR(gemm(g));
    if (P) {
      // R_{+-1} [X_L | X_R | X_b | V] = [(R V) B_J | R X_b | R V]
      CR(gemm({gd(RZp, nr, 0, BJ, nu, RXp, nr, nr, M4, nu, onec, zero), gd(RZm, nr, 0, BJ, nu, RXm, nr, nr, M4, nu, onec, zero)}));
      for (int s2 = 0; s2 < 2; ++s2) {
        const cplx* src = s2 ? RZm : RZp;
        cplx* dst = s2 ? RXm : RXp;
        CK(hipMemcpyAsync(dst + (size_t)colB * nr, src + (size_t)nu * nr, sizeof(cplx) * (size_t)nr * nang,
                          hipMemcpyDeviceToDevice, st));
        CK(hipMemcpyAsync(dst + (size_t)colU * nr, src, sizeof(cplx) * (size_t)nr * nu, hipMemcpyDeviceToDevice, st));
      }
      CK(hipStreamSynchronize(st));
    }
  } else if (!fp32) {
    // one application of A^{-1} for every alpha (and V = A^{-1} U)
    CR(apply_factors(h, true, Y, N, X, N, W));
    // alpha-free products
    std::vector<GemmDesc> g = {gd(C1, M2, 0, X, N, G1, M2, M2, (int)W, N, onec, zero),
                               gd(C2, M2, 0, X, N, G2, M2, M2, (int)W, N, onec, zero)};
    if (P) {
      g.push_back(gd(Rp, nr, 0, X, N, RXp, nr, nr, (int)W, N, onec, zero));
      g.push_back(gd(Rm, nr, 0, X, N, RXm, nr, nr, (int)W, N, onec, zero));
    }
    CR(gemm(g));
  } else {
    // complex64 preconditioner: the big apply and the Schur products on FP32 matrix cores
    CR(apply_inverse(h, Y, N, X, N, W));
    CK(h->qp32.reserve(sizeof(cplxf) * ((size_t)N * W + (size_t)M2 * N * 2 + (size_t)M2 * W * 2)));
    cplxf* X32 = h->qp32.as<cplxf>();
    cplxf* C132 = X32 + (size_t)N * W;
    cplxf* C232 = C132 + (size_t)M2 * N;
    cplxf* G132 = C232 + (size_t)M2 * N;
    cplxf* G232 = G132 + (size_t)M2 * W;
    CK(launch_cast_d2f(X, X32, (int64_t)N * W, st));
    CK(launch_cast_d2f(C1, C132, (int64_t)M2 * N, st));
    CK(launch_cast_d2f(C2, C232, (int64_t)M2 * N, st));
    auto g32 = [&](const cplxf* A, int lda, const cplxf* B, int ldb, cplxf* C, int ldc, int m, int n, int k) {
      GemmDesc32 g;
      g.A = A; g.B = B; g.C = C; g.m = m; g.n = n; g.k = k; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
      g.transA = 0; g.pad = 0; g.alpha = mkcf(1, 0); g.beta = mkcf(0, 0);
      return g;
    };
    std::vector<GemmDesc32> g = {g32(C132, M2, X32, N, G132, M2, M2, (int)W, N), g32(C232, M2, X32, N, G232, M2, M2, (int)W, N)};
    CK(gemm_batched<float>(h->arena, g, st, &h->splitws));
    CK(launch_cast_f2d(G132, G1, (int64_t)M2 * W, st));
    CK(launch_cast_f2d(G232, G2, (int64_t)M2 * W, st));
    CK(hipStreamSynchronize(st));
    if (P) CR(gemm({gd(Rp, nr, 0, X, N, RXp, nr, nr, (int)W, N, onec, zero), gd(Rm, nr, 0, X, N, RXm, nr, nr, (int)W, N, onec, zero)}));
  }
  if (!cw) CK(launch_form_S(Q, d_gco, ng, G1, G2, S, st));
  if (P) {
    // per alpha: K = (I + R V)^{-1}, R X(alpha), C~ V;  S += C~V K R X(alpha)
    for (int g = 0; g < ng; ++g) {
      const cplx* sc = d_gsc + 4 * g;  // alpha, 1/alpha, alpha^2, -alpha
      cplx* kv = KVg + (size_t)g * nr * nr;
      CK(launch_lincomb(nr, nr, sc, sc + 1, 0, RXp + (size_t)colU * nr, nr, RXm + (size_t)colU * nr, nr, nullptr, 0, kv, nr, st));
      cplx* rax = RAX + (size_t)g * nr * M2;
      // R X(alpha) = alpha^2 R1 X_R + R-1 X_R + alpha R1 X_L + alpha^{-1} R-1 X_L
      CK(launch_lincomb(nr, M2, sc + 2, d_one, 0, RXp + (size_t)M2 * nr, nr, RXm + (size_t)M2 * nr, nr, nullptr, 0, rax, nr, st));
      std::vector<cplx> negs = {mkc(-galpha[g].real(), -galpha[g].imag()), toc(-1.0 / galpha[g])};
      CK(hipMemcpyAsync(vv, negs.data(), sizeof(cplx) * 2, hipMemcpyHostToDevice, st));
      CK(launch_lincomb(nr, M2, vv, vv + 1, 0, RXp, nr, RXm, nr, rax, nr, rax, nr, st));
      CK(launch_lincomb(M2, nr, d_gco + 3 * g + 1, d_gco + 3 * g + 2, 0, G1 + (size_t)colU * M2, M2, G2 + (size_t)colU * M2,
                        M2, nullptr, 0, CV + (size_t)g * M2 * nr, M2, st));
      CK(hipStreamSynchronize(st));
    }
    CK(launch_eye_plus(nr, ng, KVg, nr, (int64_t)nr * nr, Kg, st));
    {
      std::vector<InvDesc> iv;
      for (int g = 0; g < ng; ++g) iv.push_back({Kg + (size_t)g * nr * nr, nr, nr});
      bool sing = false;
      CK(inv_batched(h->arena, h->work, iv, st, &sing));
      if (sing) { set_error("qp_solve: singular Woodbury capacitance matrix"); return HBS_E_SINGULAR; }
    }
    if (!cw) {
      std::vector<GemmDesc> g1, g2;
      for (int g = 0; g < ng; ++g)
        g1.push_back(gd(Kg + (size_t)g * nr * nr, nr, 0, RAX + (size_t)g * nr * M2, nr, KRAX + (size_t)g * nr * M2, nr, nr, M2,
                        nr, onec, zero));
      CR(gemm(g1));
      for (int g = 0; g < ng; ++g)
        g2.push_back(gd(CV + (size_t)g * M2 * nr, M2, 0, KRAX + (size_t)g * nr * M2, nr, S + (size_t)g * M2 * M2, M2, M2, M2,
                        nr, onec, onec));
      CR(gemm(g2));
    }
  }
  if (cw) {
    if (!overlap) CR(woodbury(st, h->arena, h->splitws, h->work, nullptr, false));
  } else {
    std::vector<InvDesc> iv;
    for (int g = 0; g < ng; ++g) iv.push_back({S + (size_t)g * M2 * M2, M2, M2});
    bool sing = false;
    CK(inv_batched(h->arena, h->work, iv, st, &sing));
    if (sing) {
      set_error("qp_solve: singular Schur complement");
      return HBS_E_SINGULAR;
    }
  }
  // y = K R(alpha) Z for the columns of Z (nr x nang rows-by-angle), per group
  auto neighbour_K = [&](const cplx* RZp, const cplx* RZm, cplx* out) -> int {
    CK(launch_lincomb(nr, nang, d_al, d_ainv, 1, RZp, nr, RZm, nr, nullptr, 0, uu, nr, st));
    std::vector<GemmDesc> g;
    for (int gg = 0; gg < ng; ++gg)
      g.push_back(gd(Kg + (size_t)gg * nr * nr, nr, 0, uu + (size_t)goff[gg] * nr, nr, out + (size_t)goff[gg] * nr, nr, nr,
                     gcnt[gg], nr, onec, zero));
    return gemm(g);
  };
  auto solve_S = [&](const cplx* rhs, cplx* out, cplx alpha) -> int {
    if (cw) {
      // out = alpha [y + Cq K2 B_J(alpha) y],  y = Q^{-1} rhs  (per group of angles)
      CK(launch_qsolve(Q, d_al, 1, nang, rhs, M2, yq, M2, st));
      std::vector<GemmDesc> g1, g2, g3;
      for (int gg = 0; gg < ng; ++gg)
        g1.push_back(gd(BJa + (size_t)gg * nu * M2, nu, 0, yq + (size_t)goff[gg] * M2, M2, zq + (size_t)goff[gg] * nu, nu, nu,
                        gcnt[gg], M2, onec, zero));
      CR(gemm(g1));
      for (int gg = 0; gg < ng; ++gg)
        g2.push_back(gd(K2 + (size_t)gg * nu * nu, nu, 0, zq + (size_t)goff[gg] * nu, nu, zq2 + (size_t)goff[gg] * nu, nu, nu,
                        gcnt[gg], nu, onec, zero));
      CR(gemm(g2));
      CK(launch_axpby(M2, nang, alpha, yq, M2, zero, out, M2, st));
      for (int gg = 0; gg < ng; ++gg)
        g3.push_back(gd(Cq + (size_t)gg * M2 * nu, M2, 0, zq2 + (size_t)goff[gg] * nu, nu, out + (size_t)goff[gg] * M2, M2, M2,
                        gcnt[gg], nu, alpha, onec));
      return gemm(g3);
    }
    std::vector<GemmDesc> g;
    for (int gg = 0; gg < ng; ++gg)
      g.push_back(gd(S + (size_t)gg * M2 * M2, M2, 0, rhs + (size_t)goff[gg] * M2, M2, out + (size_t)goff[gg] * M2, M2, M2,
                     gcnt[gg], M2, alpha, zero));
    return gemm(g);
  };
  const cplx* Vc = X + (size_t)ycolU * N;
  // out -= X(alpha) v for v = [xi; alpha xi] stacked (4M x nang): X_LR v, or V (B_J v) with compressed walls
  auto sub_Xv = [&](const cplx* v, cplx* out) -> int {
    if (!cw) return gemm({gd(X, N, 0, v, M4, out, N, N, nang, M4, minus1c, onec)});
    CR(gemm({gd(BJ, nu, 0, v, M4, t1, nu, nu, nang, M4, onec, zero)}));
    if (fastU && !P) {
      // V t1 = E_L ... E_1 (R^{-1} t1)
      CR(gemm({gd(Zt, nu, 0, t1, nu, t2, nu, nu, nang, nu, onec, zero)}));
      CR(apply_down_E(h, t2, nu, tN, N, nang));
      CK(launch_axpby(N, nang, minus1c, tN, N, onec, out, N, st));
      return HBS_OK;
    }
    return gemm({gd(Vc, N, 0, t1, nu, out, N, N, nang, nu, minus1c, onec)});
  };
  // out -= B(alpha) xi = [B_L | B_R] v, or U (B_J v)
  auto sub_Bv = [&](const cplx* v, cplx* out) -> int {
    if (!cw) return gemm({gd(Y, N, 0, v, M4, out, N, N, nang, M4, minus1c, onec)});
    CR(gemm({gd(BJ, nu, 0, v, M4, t1, nu, nu, nang, M4, onec, zero)}));
    CR(apply_interp(h, t1, nu, tN, N, nang));
    CK(launch_axpby(N, nang, minus1c, tN, N, onec, out, N, st));
    return HBS_OK;
  };
  // T1 = C1 v, T2 = C2 v for v (N x nang); C v = C_J (U^T v) with compressed walls
  auto C_v = [&](const cplx* v, cplx* T1o, cplx* T2o) -> int {
    if (!cw) return gemm({gd(C1, M2, 0, v, N, T1o, M2, M2, nang, N, onec, zero), gd(C2, M2, 0, v, N, T2o, M2, M2, nang, N, onec, zero)});
    CR(apply_interp_t(h, v, N, t2, nu, nang));
    return gemm({gd(C1, M2, 0, t2, nu, T1o, M2, M2, nang, nu, onec, zero), gd(C2, M2, 0, t2, nu, T2o, M2, M2, nang, nu, onec, zero)});
  };
  // right-hand sides: C~ A~^{-1} b = C~ X_b - C~V K R X_b
  CK(launch_lincomb(M2, nang, d_c1, d_c2, 1, G1 + (size_t)colB * M2, M2, G2 + (size_t)colB * M2, M2, nullptr, 0, Wv, M2, st));
  if (P) {
    CR(neighbour_K(RXp + (size_t)colB * nr, RXm + (size_t)colB * nr, yy));
    std::vector<GemmDesc> g;
    for (int gg = 0; gg < ng; ++gg)
      g.push_back(gd(CV + (size_t)gg * M2 * nr, M2, 0, yy + (size_t)goff[gg] * nr, nr, Wv + (size_t)goff[gg] * M2, M2, M2,
                     gcnt[gg], nr, minus1c, onec));
    CR(gemm(g));
  }
  // Bragg groups of >= 4 angles share one basis of diffraction orders (rows qlo .. qlo + nq - 1
  // relative to the group's first angle).  The bases depend only on the nodes and the orders:
  // when they all fit one buffer they are computed here, where the main stream would otherwise
  // wait for the side stream's Woodbury factors.
  const size_t bragg_ecap = ((size_t)4 << 30) / sizeof(cplx);
  auto bragg_orders = [&](int g, int* qlo, int* nq, std::vector<int>* sl) {
    const int q0 = goff[g], cnt = gcnt[g];
    int lo = 1 << 30, hi = -(1 << 30);
    if (sl) sl->assign(cnt, 0);
    for (int a = 0; a < cnt; ++a) {
      const int mshift = (int)std::llround((kx[q0 + a] - kx[q0]) * period / (2 * M_PI));
      const int s0 = mshift + nlo[q0 + a];
      if (sl) (*sl)[a] = s0;
      lo = std::min(lo, s0);
      hi = std::max(hi, s0 + nm[q0 + a] - 1);
    }
    *qlo = lo;
    *nq = hi - lo + 1;
  };
  DevBuf bragg_pre;
  bool bragg_early = false;
  {
    size_t et = 0;
    for (int g = 0; g < ng; ++g)
      if (gcnt[g] >= 4) {
        int qlo, nq;
        bragg_orders(g, &qlo, &nq, nullptr);
        et += (size_t)2 * nq * N;
      }
    if (et > 0 && et <= bragg_ecap) {
      CK(bragg_pre.reserve(sizeof(cplx) * et));
      size_t eoff = 0;
      ProfScope ps("bragg", st, 0.0, 0.0);
      for (int g = 0; g < ng; ++g)
        if (gcnt[g] >= 4) {
          int qlo, nq;
          bragg_orders(g, &qlo, &nq, nullptr);
          CK(launch_bragg_basis(Q, kx[goff[g]], qlo, nq, bragg_pre.as<cplx>() + eoff, st));
          eoff += (size_t)2 * nq * N;
        }
      bragg_early = true;
    }
  }
  if (overlap) CK(hipStreamWaitEvent(st, h->side_ev[1], 0));
  CR(solve_S(Wv, xi, minus1c));
  // eta = X_b - X(alpha) xi - V K (R X_b - R X(alpha) xi)
  CK(launch_stack(M2, nang, d_al, xi, stk, st));
  if (overlap) {
    // eta = A^{-1} b - A^{-1} U (B_J v): one downward pass from the root vector
    // U^T A^{-1} b - R^{-1} B_J v (the upward results of b are still in the apply workspace)
    CR(gemm({gd(BJ, nu, 0, stk, M4, t1, nu, nu, nang, M4, onec, zero)}));
    CR(gemm({gd(Zt, nu, 0, t1, nu, t2, nu, nu, nang, nu, onec, zero)}));
    CK(launch_axpby(nu, nang, onec, Zt + (size_t)nu * nu, nu, minus1c, t2, nu, st));
    CR(apply_inverse_down(h, Y + (size_t)ycolB * N, N, eta, N, nang, t2));
  } else {
    CK(launch_axpby(N, nang, onec, X + (size_t)ycolB * N, N, zero, eta, N, st));
    CR(sub_Xv(stk, eta));
  }
  // eta -= V K [R b - R X(alpha) xi], assembled in uu/yy
  auto nb_correction = [&](const cplx* Rz, const cplx* xs, cplx sign) -> int {
    // vv = Rz - RAX xs (per group), yy = K vv, eta += sign * V yy
    CK(hipMemcpyAsync(vv, Rz, sizeof(cplx) * (size_t)nr * nang, hipMemcpyDeviceToDevice, st));
    std::vector<GemmDesc> g, g2;
    for (int gg = 0; gg < ng; ++gg)
      g.push_back(gd(RAX + (size_t)gg * nr * M2, nr, 0, xs + (size_t)goff[gg] * M2, M2, vv + (size_t)goff[gg] * nr, nr, nr,
                     gcnt[gg], M2, minus1c, onec));
    CR(gemm(g));
    for (int gg = 0; gg < ng; ++gg)
      g2.push_back(gd(Kg + (size_t)gg * nr * nr, nr, 0, vv + (size_t)goff[gg] * nr, nr, yy + (size_t)goff[gg] * nr, nr, nr,
                      gcnt[gg], nr, onec, zero));
    CR(gemm(g2));
    return gemm({gd(Vc, N, 0, yy, nr, eta, N, N, nang, nr, sign, onec)});
  };
  if (P) {
    CK(launch_lincomb(nr, nang, d_al, d_ainv, 1, RXp + (size_t)colB * nr, nr, RXm + (size_t)colB * nr, nr, nullptr, 0, Rb, nr,
                      st));
    CR(nb_correction(Rb, xi, minus1c));
  }
  // iterative refinement of the bordered system
  int maxit = o->refine_max_iter < 0 ? 0 : (o->refine_max_iter == 0 ? (fp32 ? 3 : 2) : o->refine_max_iter);
  const double rtol = o->refine_tol > 0 ? o->refine_tol : 1e-13;
  std::vector<double> hn(3 * nang);
  CK(launch_colnorm2(N, nang, Y + (size_t)ycolB * N, N, nrm + 2 * nang, st));
  double relres = -1;
  int iters = 0;
  for (int it = 0; it <= maxit; ++it) {
    // R1 = b - A~ eta - B(alpha) xi ;  R2 = -C~(alpha) eta - Q(alpha) xi
    if (cw && !xw) {
      // every U-term enters at the root of one forward apply: F = A eta + U (B_J v [+ R(alpha) eta]),
      // and the same apply's upward result at the root is U^T eta (C eta = C_J U^T eta)
      CR(gemm({gd(BJ, nu, 0, stk, M4, t1, nu, nu, nang, M4, onec, zero)}));
      if (P) {
        CR(gemm({gd(Rp, nr, 0, eta, N, uu, nr, nr, nang, N, onec, zero), gd(Rm, nr, 0, eta, N, yy, nr, nr, nang, N, onec, zero)}));
        CK(launch_lincomb(nr, nang, d_al, d_ainv, 1, uu, nr, yy, nr, nullptr, 0, vv, nr, st));
        CK(launch_axpby(nr, nang, onec, vv, nr, onec, t1, nu, st));
      }
      CR(apply_forward_root(h, eta, N, F, N, nang, t1, t2));
      CK(launch_axpby(N, nang, onec, Y + (size_t)ycolB * N, N, zero, R1, N, st));
      CK(launch_axpby(N, nang, minus1c, F, N, onec, R1, N, st));
      CR(gemm({gd(C1, M2, 0, t2, nu, T1, M2, M2, nang, nu, onec, zero), gd(C2, M2, 0, t2, nu, T2, M2, M2, nang, nu, onec, zero)}));
    } else {
      CR(apply_factors(h, false, eta, N, F, N, nang));
      if (P) {
        CR(gemm({gd(Rp, nr, 0, eta, N, uu, nr, nr, nang, N, onec, zero), gd(Rm, nr, 0, eta, N, yy, nr, nr, nang, N, onec, zero)}));
        CK(launch_lincomb(nr, nang, d_al, d_ainv, 1, uu, nr, yy, nr, nullptr, 0, vv, nr, st));
        CR(apply_interp(h, vv, nr, Z1, N, nang));
        CK(launch_axpby(N, nang, onec, Z1, N, onec, F, N, st));
      }
      CK(launch_axpby(N, nang, onec, Y + (size_t)ycolB * N, N, zero, R1, N, st));
      CK(launch_axpby(N, nang, minus1c, F, N, onec, R1, N, st));
      if (xw) {
        CR(gemm({gd(Yx, N, 0, stk, M4, R1, N, N, nang, M4, minus1c, onec)}));
        CR(gemm({gd(C1x, M2, 0, eta, N, T1, M2, M2, nang, N, onec, zero), gd(C2x, M2, 0, eta, N, T2, M2, M2, nang, N, onec, zero)}));
      } else {
        CR(sub_Bv(stk, R1));
        CR(C_v(eta, T1, T2));
      }
    }
    CK(launch_resid2(Q, nang, d_al, d_c1, d_c2, T1, T2, xi, R2, st));
    CK(launch_colnorm2(N, nang, R1, N, nrm, st));
    CK(launch_colnorm2(M2, nang, R2, M2, nrm + nang, st));
    CK(hipMemcpyAsync(hn.data(), nrm, sizeof(double) * 3 * nang, hipMemcpyDeviceToHost, st));
    // the side stream's flags: the capacitance matrices, then the root matrix when it was deferred
    const int nflag = ng + (defer ? 1 : 0);
    std::vector<int> sinfo(side_dinfo && it == 0 ? nflag : 0);
    // the main stream has waited for the side stream's inversion: its flags are final
    if (!sinfo.empty()) CK(hipMemcpyAsync(sinfo.data(), side_dinfo, sizeof(int) * nflag, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (!sinfo.empty() && defer) {
      h->root_state = sinfo[ng] ? 3 : 0;
      if (sinfo[ng]) {
        set_error("qp_solve: singular root matrix");
        return HBS_E_SINGULAR;
      }
    }
    for (int g = 0; g < ng && !sinfo.empty(); ++g)
      if (sinfo[g] != 0) {
        set_error("qp_solve: singular Schur complement");
        return HBS_E_SINGULAR;
      }
    relres = 0;
    for (int q = 0; q < nang; ++q) relres = std::max(relres, std::sqrt((hn[q] + hn[nang + q]) / hn[2 * nang + q]));
    if (relres < rtol || it == maxit) break;
    ++iters;
    // correction by the block solve: Z1 = A~^{-1} R1; dxi = S^{-1}(R2 - C~ Z1); deta = Z1 - X~(alpha) dxi
    CR(apply_factors(h, true, R1, N, Z1, N, nang));
    if (P) {
      CR(gemm({gd(Rp, nr, 0, Z1, N, uu, nr, nr, nang, N, onec, zero), gd(Rm, nr, 0, Z1, N, vv, nr, nr, nang, N, onec, zero)}));
      CK(hipMemcpyAsync(Rb, uu, sizeof(cplx) * (size_t)nr * nang, hipMemcpyDeviceToDevice, st));
      CR(neighbour_K(Rb, vv, yy));
      CR(gemm({gd(Vc, N, 0, yy, nr, Z1, N, N, nang, nr, minus1c, onec)}));
    }
    CR(C_v(Z1, U1, U2));
    CK(launch_lincomb(M2, nang, d_c1, d_c2, 1, U1, M2, U2, M2, R2, M2, Wv, M2, st));
    CR(solve_S(Wv, dxi, onec));
    CK(launch_stack(M2, nang, d_al, dxi, stk, st));
    CK(launch_axpby(N, nang, onec, Z1, N, onec, eta, N, st));
    CR(sub_Xv(stk, eta));
    if (P) {
      // + V K R X(alpha) dxi  (X~(alpha) = X(alpha) - V K R X(alpha))
      CK(hipMemsetAsync(Rb, 0, sizeof(cplx) * (size_t)nr * nang, st));
      CR(nb_correction(Rb, dxi, minus1c));
    }
    CK(launch_axpby(M2, nang, onec, dxi, M2, onec, xi, M2, st));
    CK(launch_stack(M2, nang, d_al, xi, stk, st));
  }
  h->stats.refine_iters = iters;
  h->stats.refine_residual = relres;
  h->stats.contour_M = M;
  h->stats.walls_compressed = cw ? (xw ? 2 : 1) : 0;
  if (maxit > 0 && relres >= rtol && relres > 1e-8) {
    set_error("qp_solve: refinement stalled at relative residual " + std::to_string(relres));
    return HBS_E_NOT_CONVERGED;
  }
  // Bragg amplitudes
  {
    ProfScope ps("bragg", st, 0.0, 0.0);
    // groups of >= 4 angles share one basis of diffraction orders (one batched GEMM for all such
    // groups); smaller groups sum directly
    struct BG { int q0, cnt, qlo, nq; double kref; size_t eoff, coff, soff; };
    std::vector<BG> bg;
    std::vector<int> slots;
    size_t etot = 0, ctot = 0;
    // bases of at most ~4 GiB at a time
    const size_t ecap = bragg_ecap;
    auto flush = [&]() -> int {
      if (bg.empty()) return HBS_OK;
      // with the bases computed early (one buffer, so this is the only flush) only the
      // coefficients and slots go to the work buffer
      const size_t ewk = bragg_early ? 0 : etot;
      CK(h->work.reserve(sizeof(cplx) * (ewk + ctot) + sizeof(int) * slots.size() + 512));
      cplx* E = bragg_early ? bragg_pre.as<cplx>() : h->work.as<cplx>();
      cplx* Cg = h->work.as<cplx>() + ewk;
      int* dslot = (int*)(Cg + ctot);
      CK(hipMemcpyAsync(dslot, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice, st));
      std::vector<GemmDesc> g;
      for (const BG& b : bg) {
        if (!bragg_early) CK(launch_bragg_basis(Q, b.kref, b.qlo, b.nq, E + b.eoff, st));
        g.push_back(gd(E + b.eoff, 2 * b.nq, 0, eta + (size_t)b.q0 * N, N, Cg + b.coff, 2 * b.nq, 2 * b.nq, b.cnt, N, onec,
                       zero));
      }
      CR(gemm(g));
      for (const BG& b : bg)
        CK(launch_bragg_gather(Q, b.kref, b.qlo, b.nq, dslot + b.soff, dnm + b.q0, maxm, b.cnt, Cg + b.coff, pl.y0,
                               brg + (size_t)b.q0 * 2 * maxm, st));
      CK(hipStreamSynchronize(st));
      bg.clear();
      slots.clear();
      etot = ctot = 0;
      return HBS_OK;
    };
    for (int g = 0; g < ng; ++g) {
      const int q0 = goff[g], cnt = gcnt[g];
      if (cnt < 4) {
        CK(launch_bragg(Q, dkap + q0, dnlo + q0, dnm + q0, maxm, cnt, eta + (size_t)q0 * N, N, pl.y0,
                        brg + (size_t)q0 * 2 * maxm, st));
        continue;
      }
      BG b{q0, cnt, 0, 0, kx[q0], 0, 0, 0};
      std::vector<int> sl;
      bragg_orders(g, &b.qlo, &b.nq, &sl);
      if (etot + (size_t)2 * b.nq * N > ecap) CR(flush());
      b.soff = slots.size();
      for (int a = 0; a < cnt; ++a) slots.push_back(sl[a] - b.qlo);
      b.eoff = etot;
      b.coff = ctot;
      etot += (size_t)2 * b.nq * N;
      ctot += (size_t)2 * b.nq * cnt;
      bg.push_back(b);
    }
    CR(flush());
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
