// Entries of the Nystrom matrix A = I/2 + D - i omega S (Sec. 2.2 below Eq. 2.15).
#pragma once
#include "hankel.h"
#include "internal.h"

#define QPS_PI 3.14159265358979323846264338327950288
#define QPS_EULER 0.577215664901532860606512090082402431

// Kernel K(x, y, n_y) = dG/dn_y - i omega G with G = (i/4) H0(omega |x - y|) (Eqs. 2.7-2.9):
//   K = (i omega / 4) H1(omega r) n_y.(x - y)/r + (omega / 4) H0(omega r).
__device__ inline cplx helm_kernel(double omega, double dx, double dy, double nx, double ny) {
  const double r = sqrt(dx * dx + dy * dy);
  cplx h0, h1;
  hankel01(omega * r, h0, h1);
  const double nd = (nx * dx + ny * dy) / r;
  const double q = 0.25 * omega;
  return mkc(q * (h0.x - h1.y * nd), q * (h0.y + h1.x * nd));
}

// Kapur-Rokhlin discretization (Sec. 2.3): A_ij = delta_ij/2 + R_{(i-j) mod N} K(y_i, y_j, n_j) w_j,
// R_0 = 0, R_m = R_{N-m} = 1 + g_m (1 <= m <= 6), 1 otherwise.
__device__ inline cplx a_entry_kr6(const Geo& G, int i, int j) {
  if (i == j) return mkc(0.5, 0.0);
  cplx K = helm_kernel(G.omega, G.x[i] - G.x[j], G.y[i] - G.y[j], G.nx[j], G.ny[j]);
  int m = i - j;
  if (m < 0) m += G.N;
  double R = 1.0;
  if (m <= 6) R += G.g[m - 1];
  else if (m >= G.N - 6) R += G.g[G.N - m - 1];
  return cscale(K, R * G.w[j]);
}

// Kress' spectral log-split discretization, N = 2n nodes (Colton & Kress, Sec. 3.5), with
// speed s_j = N w_j / (2 pi) and z'(t_j) = s_j (-n_y, n_x):
//   M = (i/4) H0 s_j,  L = (i omega/4) H1 s_j nd,  M1 = -J0 s_j / (4 pi),  L1 = -omega J1 s_j nd / (4 pi),
//   M2 = M - M1 ln(4 sin^2((t_i - t_j)/2)), L2 = L - L1 ln(...), and on the diagonal
//   M1 = -s/(4 pi), L1 = 0, M2 = [i/4 - C_E/(2 pi) - ln(omega s / 2)/(2 pi)] s, L2 = -kappa s / (4 pi);
//   A_ij = delta_ij/2 + Rk_{(i-j)} (L1 - i omega M1) + (pi / n) (L2 - i omega M2).
__device__ inline cplx a_entry_kress(const Geo& G, int i, int j) {
  const int N = G.N;
  const double pin = QPS_PI / (0.5 * N);
  const double s = G.w[j] * N / (2.0 * QPS_PI);
  int m = i - j;
  if (m < 0) m += N;
  const double Rk = G.kressR[m];
  const double om = G.omega;
  if (i == j) {
    // -i om M1 = i om s/(4pi)
    cplx t1 = mkc(0.0, om * s / (4.0 * QPS_PI));
    double m2r = (-QPS_EULER / (2.0 * QPS_PI) - log(0.5 * om * s) / (2.0 * QPS_PI)) * s;
    double m2i = 0.25 * s;
    double l2 = -G.kap[j] * s / (4.0 * QPS_PI);
    // L2 - i om M2 = (l2 + om m2i) - i om m2r
    cplx t2 = mkc(l2 + om * m2i, -om * m2r);
    return mkc(0.5 + Rk * t1.x + pin * t2.x, Rk * t1.y + pin * t2.y);
  }
  const double dx = G.x[i] - G.x[j], dy = G.y[i] - G.y[j];
  const double r = sqrt(dx * dx + dy * dy);
  cplx h0, h1;
  hankel01(om * r, h0, h1);
  const double nd = (G.nx[j] * dx + G.ny[j] * dy) / r;
  // M = (i/4) h0 s ; L = (i om/4) h1 s nd
  const cplx M = mkc(-0.25 * h0.y * s, 0.25 * h0.x * s);
  const cplx L = mkc(-0.25 * om * h1.y * s * nd, 0.25 * om * h1.x * s * nd);
  const double M1 = -h0.x * s / (4.0 * QPS_PI);
  const double L1 = -om * h1.x * s * nd / (4.0 * QPS_PI);
  const double t = 2.0 * QPS_PI * (double)m / (double)N;
  const double sh = sin(0.5 * t);
  const double lg = log(4.0 * sh * sh);
  const cplx M2 = mkc(M.x - M1 * lg, M.y);
  const cplx L2 = mkc(L.x - L1 * lg, L.y);
  // R (L1 - i om M1) + (pi/n)(L2 - i om M2); M1, L1 real
  const cplx a = mkc(Rk * L1, -Rk * om * M1);
  const cplx b = mkc(L2.x + om * M2.y, L2.y - om * M2.x);
  return mkc(a.x + pin * b.x, a.y + pin * b.y);
}

// Alpert's hybrid Gauss-trapezoidal correction (Sec. 2.3 names it beside Kapur-Rokhlin): the grid
// nodes closer than a to the target (periodic index distance) are left out, and the off-grid nodes
// t_i +- x_l h carry the density as its Lagrange interpolant from the G.alpnl grid values at
// offsets G.alpo[q] .. G.alpo[q] + alpnl - 1 (q = one of the 2m off-grid nodes), weights G.alpL.
// The kernel part of node q of row i, h w_l K(y_i, z(t_i + u_q h), n(...)) |z'(...)|, is the table
// G.alpT[i + q N] built once per handle, so
//   A_ij = delta_ij/2 + [dist(i, j) >= a] K(y_i, y_j, n_j) w_j + sum_q alpT[i, q] L_q(j - i).
__device__ inline cplx a_entry_alpert(const Geo& G, int i, int j) {
  const int N = G.N;
  int d = j - i;
  if (d > N / 2) d -= N;
  if (d < -(N - 1) / 2) d += N;
  cplx v = mkc(i == j ? 0.5 : 0.0, 0.0);
  if (d >= G.alpa || -d >= G.alpa) {
    const cplx K = helm_kernel(G.omega, G.x[i] - G.x[j], G.y[i] - G.y[j], G.nx[j], G.ny[j]);
    v = cadd(v, cscale(K, G.w[j]));
  }
  for (int q = 0; q < G.alpn; ++q) {
    const int r = d - G.alpo[q];
    if (r >= 0 && r < G.alpnl) v = cadd(v, cscale(G.alpT[i + (size_t)q * N], G.alpL[q * G.alpnl + r]));
  }
  return v;
}

__device__ inline cplx a_entry(const Geo& G, int i, int j) {
  if (G.quad == HBS_QUAD_ALPERT) return a_entry_alpert(G, i, j);
  return G.quad == HBS_QUAD_KRESS ? a_entry_kress(G, i, j) : a_entry_kr6(G, i, j);
}

// Transmission problem (Sec. 5): the four difference kernels of the interlaced 2 x 2 operator, with
// H0, H1 taken at k0 r and k1 r (k0 = omega outside, k1 = n omega inside), a = n_x.(x - y)/r,
// b = n_y.(x - y)/r, nn = n_x.n_y, d1 = k0 H1(k0 r) - k1 H1(k1 r), d0 = k0^2 H0(k0 r) - k1^2 H0(k1 r),
// kb = max(k0, k1) (the single layer carries kb and the normal-derivative row is divided by it, so
// that all four blocks are of one size in the far field):
//   (row 0, col 0)  D0 - D1            = (i/4) b d1
//   (0, 1)          kb (S0 - S1)       = (i/4) kb [H0(k0 r) - H0(k1 r)]
//   (1, 0)          -(T0 - T1) / kb    = -(i/4) [a b d0 + (nn - 2 a b) d1 / r] / kb
//   (1, 1)          -(D0* - D1*)       = (i/4) a d1
// (T = d^2 G / dn_x dn_y, D* = dG/dn_x; the 1/r^2 parts of T0 and T1 cancel in d1 / r).
__device__ inline cplx tr_kernel(double k0, double k1, double kb, double dx, double dy, double tnx, double tny, double snx,
                                 double sny, int cr, int cc) {
  const double r = sqrt(dx * dx + dy * dy);
  cplx a0, a1, b0, b1;
  hankel01(k0 * r, a0, a1);
  hankel01(k1 * r, b0, b1);
  cplx v;
  if (cr == 0 && cc == 1) {
    v = mkc(kb * (a0.x - b0.x), kb * (a0.y - b0.y));
  } else {
    const cplx d1 = mkc(k0 * a1.x - k1 * b1.x, k0 * a1.y - k1 * b1.y);
    const double a = (tnx * dx + tny * dy) / r, b = (snx * dx + sny * dy) / r;
    if (cr == 0) {
      v = cscale(d1, b);
    } else if (cc == 1) {
      v = cscale(d1, a);
    } else {
      const double k02 = k0 * k0, k12 = k1 * k1;
      const cplx d0 = mkc(k02 * a0.x - k12 * b0.x, k02 * a0.y - k12 * b0.y);
      const double ab = a * b, c = (tnx * snx + tny * sny - 2.0 * ab) / r, ikb = 1.0 / kb;
      v = mkc(-(ab * d0.x + c * d1.x) * ikb, -(ab * d0.y + c * d1.y) * ikb);
    }
  }
  return mkc(-0.25 * v.y, 0.25 * v.x);  // (i/4) v
}

// Entry (u, v) of the transmission operator I + K (u = 2 i + c_r, v = 2 j + c_c) with the
// Kapur-Rokhlin weights R_{(i-j) mod N} of Sec. 2.3 on every block (R_0 = 0: the kernel drops at i = j).
__device__ inline cplx a_entry_tr(const Geo& G, int u, int v) {
  const int i = u >> 1, j = v >> 1, cr = u & 1, cc = v & 1;
  if (i == j) return mkc(cr == cc ? 1.0 : 0.0, 0.0);
  const cplx K = tr_kernel(G.omega, G.omega1, G.kbar, G.x[i] - G.x[j], G.y[i] - G.y[j], G.nx[i], G.ny[i], G.nx[j], G.ny[j],
                           cr, cc);
  int m = i - j;
  if (m < 0) m += G.N;
  double R = 1.0;
  if (m <= 6) R += G.g[m - 1];
  else if (m >= G.N - 6) R += G.g[G.N - m - 1];
  return cscale(K, R * G.w[j]);
}

// The exterior field's rows alone (wavenumber k = omega; neighbour images and the far-field circle
// see only u+): target unknown t = 2 i + c_r at x_i + (tsx, 0), source unknown s = 2 j + c_c at
// x_j + (ssx, 0), plain trapezoid weight w_j, the normalization kb of tr_kernel:
//   (0, 0) dG/dn_y = (i/4) k H1 b,  (0, 1) kb G = (i/4) kb H0,
//   (1, 0) -T / kb = -(i/4) [k^2 H0 a b + (k H1 / r)(nn - 2 a b)] / kb,  (1, 1) -dG/dn_x = (i/4) k H1 a.
__device__ inline cplx a_ext_tr(const Geo& G, int t, int s, double tsx, double ssx) {
  const int i = t >> 1, j = s >> 1, cr = t & 1, cc = s & 1;
  const double dx = G.x[i] + tsx - G.x[j] - ssx, dy = G.y[i] - G.y[j];
  const double r = sqrt(dx * dx + dy * dy);
  const double k = G.omega;
  cplx h0, h1;
  hankel01(k * r, h0, h1);
  cplx v;
  if (cr == 0 && cc == 1) {
    v = cscale(h0, G.kbar);
  } else {
    const double a = (G.nx[i] * dx + G.ny[i] * dy) / r, b = (G.nx[j] * dx + G.ny[j] * dy) / r;
    if (cr == 0) {
      v = cscale(h1, k * b);
    } else if (cc == 1) {
      v = cscale(h1, k * a);
    } else {
      const double ab = a * b, c = k * (G.nx[i] * G.nx[j] + G.ny[i] * G.ny[j] - 2.0 * ab) / r, ikb = 1.0 / G.kbar;
      v = mkc(-(k * k * ab * h0.x + c * h1.x) * ikb, -(k * k * ab * h0.y + c * h1.y) * ikb);
    }
  }
  return cscale(mkc(-0.25 * v.y, 0.25 * v.x), G.w[j]);
}

__device__ inline cplx a_entry_any(const Geo& G, int i, int j) { return G.two ? a_entry_tr(G, i, j) : a_entry(G, i, j); }
