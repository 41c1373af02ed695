// Device kernels of the periodizing scheme (Sec. 2.2-2.4) and the block solve (Sec. 3.1):
// Sommerfeld-contour wall blocks B (Eq. 2.16) and C (Eq. 2.17), incident data, the Schur
// complement S(alpha) = Q(alpha) - C(alpha) A^{-1} B(alpha) assembled from alpha-free products,
// and Bragg amplitudes from the lattice-summed Green's function.
#include "hankel.h"
#include "qp_kernels.h"

namespace {

constexpr int NT = 256;
constexpr double PI = 3.14159265358979323846264338327950288;

// exp(i z) for complex z
__device__ inline cplx cexpi_c(cplx z) {
  const double e = exp(-z.y);
  double s, c;
  sincos(z.x, &s, &c);
  return mkc(e * c, e * s);
}

// Y[:, 0:4M] = [B^S_L, B^D_L, B^S_R, B^D_R] with
//   B^S_W[i,m] = (i/2) wk_m e^{i k_m y_i} e^{i s_m |x_i - x_W|} / s_m,
//   B^D_W[i,m] = (1/2) sign(x_i - x_W) wk_m e^{i k_m y_i} e^{i s_m |x_i - x_W|}   (Eqs. 2.12-2.13).
// Transmission problem: row 2i is the value above at node i, row 2i + 1 minus its normal derivative
// over Q.kb, d/dn e^{i k y + i s |x - x_W|} = i (s sign(x - x_W) n_x + k n_y) e^{...}.
__global__ __launch_bounds__(NT) void k_gen_B(QPGeo Q, cplx* __restrict__ Y, int64_t ldy) {
  // rows: every unknown, or the Q.N unknowns idx[] (a skeleton subset)
  const int nrow = (Q.two && !Q.idx) ? 2 * Q.N : Q.N;
  const int64_t total = (int64_t)nrow * 4 * Q.M;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int i = (int)(e % nrow);
    const int col = (int)(e / nrow);
    const int wall = col / (2 * Q.M);          // 0 = L, 1 = R
    const int dbl = (col / Q.M) & 1;           // 0 = single, 1 = double
    const int m = col % Q.M;
    const int u = Q.idx ? Q.idx[i] : i;
    const int nd = Q.two ? u >> 1 : u;
    const double xw = wall ? 0.5 * Q.period : -0.5 * Q.period;
    const double dx = Q.x[nd] + Q.shift - xw;
    const cplx k = Q.k[m], s = Q.s[m], wk = Q.wk[m];
    // i (k y + s |dx|)
    const cplx z = mkc(k.x * Q.y[nd] + s.x * fabs(dx), k.y * Q.y[nd] + s.y * fabs(dx));
    const cplx ex = cmul(wk, cexpi_c(z));
    cplx v;
    if (!dbl) v = cmul(mkc(0.0, 0.5), cmul(ex, cinv(s)));
    else v = cscale(ex, dx > 0 ? 0.5 : -0.5);
    if (Q.two && (u & 1)) {
      const double sg = dx > 0 ? 1.0 : -1.0;
      // -i (s sg n_x + k n_y) v / kb
      const cplx f = cscale(cadd(cscale(s, sg * Q.nx[nd]), cscale(k, Q.ny[nd])), 1.0 / Q.kb);
      v = cmul(mkc(f.y, -f.x), v);
    }
    Y[i + (size_t)col * ldy] = v;
  }
}

// b = -exp(i (kx x + ky y)) for each column; ky may be complex (ky_im nullable): the Rayleigh-Bloch
// waves of evanescent orders that the Wood's-anomaly scheme adds as extra right-hand sides
__global__ __launch_bounds__(NT) void k_gen_inc(QPGeo Q, const double* __restrict__ kx, const double* __restrict__ ky,
                                                const double* __restrict__ ky_im, int nang, cplx* __restrict__ Y, int64_t ldy) {
  // transmission problem (Eqs. 5.3-5.4): row 2i = -u^i, row 2i + 1 = +(du^i/dn) / kb = -i (kx n_x + ky n_y) (-u^i) / kb
  const int nrow = Q.two ? 2 * Q.N : Q.N;
  const int64_t total = (int64_t)nrow * nang;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e % nrow);
    const int a = (int)(e / nrow);
    const int i = Q.two ? r >> 1 : r;
    double s, c;
    sincos(kx[a] * Q.x[i] + ky[a] * Q.y[i], &s, &c);
    const double amp = ky_im ? -exp(-ky_im[a] * Q.y[i]) : -1.0;
    cplx v = mkc(amp * c, amp * s);
    if (Q.two && (r & 1)) {
      const double f = (kx[a] * Q.nx[i] + ky[a] * Q.ny[i]) / Q.kb;
      v = mkc(f * v.y, -f * v.x);
    }
    Y[r + (size_t)a * ldy] = v;
  }
}

// C_W (2M x N): rows m (value) and M + m (x-derivative) of the wall Fourier data of the density
// at node j on dOmega + shift e_1, with E = e^{-i k y_j} e^{i s |x_j - x_W|} / (4 pi), sigma = sign(x_j - x_W):
//   value = [E (-sigma n_x + (k/s) n_y) + omega E / s] w_j
//   deriv = [i E (s n_x - k sigma n_y) - i omega E sigma] w_j          (Sec. 2.2, Eq. 2.17)
// Transmission problem: column 2j carries the double layer alone (value E (-sigma n_x + (k/s) n_y),
// deriv i E (s n_x - k sigma n_y)) and column 2j + 1 the single layer times Q.kb (value i kb E / s,
// deriv kb E sigma), both times w_j: the Dirichlet column is their combination D - i omega S.
__global__ __launch_bounds__(NT) void k_gen_C(QPGeo Q, int wall, double shift, cplx* __restrict__ C) {
  const int ncol = (Q.two && !Q.idx) ? 2 * Q.N : Q.N;
  const int64_t total = (int64_t)ncol * Q.M;
  const double xw = wall ? 0.5 * Q.period : -0.5 * Q.period;
  const int ldc = 2 * Q.M;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int m = (int)(e % Q.M);
    const int j = (int)(e / Q.M);
    const int uj = Q.idx ? Q.idx[j] : j;
    const int nd = Q.two ? uj >> 1 : uj;
    const double dx = Q.x[nd] + shift - xw;
    const double sg = dx > 0 ? 1.0 : -1.0;
    const cplx k = Q.k[m], s = Q.s[m];
    // i(-k y + s |dx|)
    const cplx z = mkc(-k.x * Q.y[nd] + s.x * fabs(dx), -k.y * Q.y[nd] + s.y * fabs(dx));
    const cplx E = cscale(cexpi_c(z), 1.0 / (4.0 * PI));
    const cplx is = cinv(s);
    const double nx = Q.nx[nd], ny = Q.ny[nd], w = Q.w[nd];
    if (Q.two && (uj & 1)) {
      const cplx ve = cmul(mkc(0.0, 1.0), cmul(E, is));
      C[m + (size_t)j * ldc] = cscale(ve, w * Q.kb);
      C[Q.M + m + (size_t)j * ldc] = cscale(E, sg * w * Q.kb);
      continue;
    }
    const double om = Q.two ? 0.0 : Q.omega;  // no single-layer part in a transmission tau column
    // value
    cplx t = cadd(mkc(-sg * nx, 0.0), cscale(cmul(k, is), ny));
    cplx val = cadd(cmul(E, t), cscale(cmul(E, is), om));
    // derivative: i E (s nx - k sg ny) - i omega E sg
    cplx u = csub(cscale(s, nx), cscale(k, sg * ny));
    cplx der = cmul(mkc(0.0, 1.0), csub(cmul(E, u), cscale(E, om * sg)));
    C[m + (size_t)j * ldc] = cscale(val, w);
    C[Q.M + m + (size_t)j * ldc] = cscale(der, w);
  }
}

// Q(alpha) entry (r, c) with E = e^{i s d}, a(+/-) = alpha +/- 1/alpha (Eq. 2.18 with the identity
// blocks placed as the wall self-terms require):
//   [[ i E a- /(2 s),  1 - E a+/2 ], [ -1 + E a+/2,  i E s a-/2 ]]
__device__ inline cplx q_entry(const QPGeo& Q, cplx alpha, int r, int c) {
  const int M = Q.M;
  const int m = r % M;
  if (c % M != m) return mkc(0, 0);
  const cplx s = Q.s[m];
  const cplx E = cexpi_c(cscale(s, Q.period));
  const cplx ainv = cinv(alpha);
  const cplx ap = cadd(alpha, ainv), am = csub(alpha, ainv);
  const int br = r / M, bc = c / M;
  if (br == 0 && bc == 0) return cmul(mkc(0.0, 0.5), cmul(cmul(E, am), cinv(s)));
  if (br == 1 && bc == 1) return cmul(mkc(0.0, 0.5), cmul(cmul(E, am), s));
  const cplx h = cscale(cmul(E, ap), 0.5);
  if (br == 0) return mkc(1.0 - h.x, -h.y);
  return mkc(h.x - 1.0, h.y);
}

// out[:, a] = Q(alpha_a)^{-1} in[:, a]: Q couples rows m and M + m only, so each contour node is a
// 2 x 2 solve (in and out may alias).  alpha_a = alpha[a * cs].
__global__ __launch_bounds__(NT) void k_qsolve(QPGeo Q, const cplx* __restrict__ alpha, int cs, int ncol, const cplx* in,
                                               int64_t ldi, cplx* out, int64_t ldo) {
  const int M = Q.M;
  const int64_t total = (int64_t)M * ncol;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int m = (int)(e % M), a = (int)(e / M);
    const cplx al = alpha[(size_t)a * cs];
    const cplx q00 = q_entry(Q, al, m, m), q01 = q_entry(Q, al, m, M + m);
    const cplx q10 = q_entry(Q, al, M + m, m), q11 = q_entry(Q, al, M + m, M + m);
    const cplx id = cinv(csub(cmul(q00, q11), cmul(q01, q10)));
    const cplx x0 = in[m + (size_t)a * ldi], x1 = in[M + m + (size_t)a * ldi];
    out[m + (size_t)a * ldo] = cmul(id, csub(cmul(q11, x0), cmul(q01, x1)));
    out[M + m + (size_t)a * ldo] = cmul(id, csub(cmul(q00, x1), cmul(q10, x0)));
  }
}

// S_g = Q(alpha_g) - C(alpha_g) X(alpha_g) with C(alpha) = c1 C1 + c2 C2, X(alpha) = X_L + alpha X_R:
//   S_g = Q - [c1 (G1_L + alpha G1_R) + c2 (G2_L + alpha G2_R)],  G1 = C1 [X_L | X_R | ...], G2 = C2 [...]
// (ld 2M).  coef holds (alpha, c1, c2) per group.
__global__ __launch_bounds__(NT) void k_form_S(QPGeo Q, const cplx* __restrict__ coef, const cplx* __restrict__ G1,
                                               const cplx* __restrict__ G2, cplx* __restrict__ S) {
  const int g = blockIdx.y;
  const int M2 = 2 * Q.M;
  const cplx al = coef[3 * g], c1 = coef[3 * g + 1], c2 = coef[3 * g + 2];
  const int64_t total = (int64_t)M2 * M2;
  cplx* Sg = S + (size_t)g * total;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e % M2), c = (int)(e / M2);
    const cplx x1 = cadd(G1[r + (size_t)c * M2], cmul(al, G1[r + (size_t)(M2 + c) * M2]));
    const cplx x2 = cadd(G2[r + (size_t)c * M2], cmul(al, G2[r + (size_t)(M2 + c) * M2]));
    const cplx cx = cadd(cmul(c1, x1), cmul(c2, x2));
    Sg[e] = csub(q_entry(Q, al, r, c), cx);
  }
}

// W[:, a] = c1_a U1[:, a] + c2_a U2[:, a]  (or R - (...) when R is given), rows of length `rows`
__global__ __launch_bounds__(NT) void k_lincomb(int rows, int ncol, const cplx* __restrict__ c1, const cplx* __restrict__ c2,
                                                int cs, const cplx* __restrict__ U1, int64_t ld1, const cplx* __restrict__ U2,
                                                int64_t ld2, const cplx* R, int64_t ldr, cplx* W, int64_t ldw) {
  const int64_t total = (int64_t)rows * ncol;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e % rows), a = (int)(e / rows);
    cplx v = cadd(cmul(c1[a * cs], U1[r + (size_t)a * ld1]), cmul(c2[a * cs], U2[r + (size_t)a * ld2]));
    if (R) v = csub(R[r + (size_t)a * ldr], v);
    W[r + (size_t)a * ldw] = v;
  }
}

// Xi_stack (4M x nang) = [xi; alpha xi]
__global__ __launch_bounds__(NT) void k_stack(int M2, int nang, const cplx* __restrict__ alpha_col,
                                              const cplx* __restrict__ xi, cplx* __restrict__ st) {
  const int64_t total = (int64_t)M2 * nang;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e % M2), a = (int)(e / M2);
    const cplx v = xi[e];
    st[r + (size_t)a * 2 * M2] = v;
    st[M2 + r + (size_t)a * 2 * M2] = cmul(alpha_col[a], v);
  }
}

// R2[:, a] = -(c1_a T1 + c2_a T2)[:, a] - Q(alpha_a) xi[:, a]
__global__ __launch_bounds__(NT) void k_resid2(QPGeo Q, int nang, const cplx* __restrict__ alpha_col,
                                               const cplx* __restrict__ c1, const cplx* __restrict__ c2,
                                               const cplx* __restrict__ T1, const cplx* __restrict__ T2,
                                               const cplx* __restrict__ xi, cplx* __restrict__ R2) {
  const int M = Q.M, M2 = 2 * M;
  const int64_t total = (int64_t)M2 * nang;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e % M2), a = (int)(e / M2);
    const cplx al = alpha_col[a];
    const cplx* x = xi + (size_t)a * M2;
    const int m = r % M;
    cplx qx = cadd(cmul(q_entry(Q, al, r, m), x[m]), cmul(q_entry(Q, al, r, M + m), x[M + m]));
    cplx cv = cadd(cmul(c1[a], T1[e]), cmul(c2[a], T2[e]));
    R2[e] = mkc(-cv.x - qx.x, -cv.y - qx.y);
  }
}

// A_g = I + B_g for ng square n x n blocks (ld n), B_g at B + g*bstride with column stride ldb
__global__ __launch_bounds__(NT) void k_eye_plus(int n, int ng, const cplx* __restrict__ B, int64_t ldb, int64_t bstride,
                                                 cplx* __restrict__ A) {
  const int64_t total = (int64_t)n * n * ng;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int g = (int)(e / ((int64_t)n * n));
    const int64_t q = e % ((int64_t)n * n);
    const int r = (int)(q % n), c = (int)(q / n);
    cplx v = B[(size_t)g * bstride + r + (size_t)c * ldb];
    if (r == c) v.x += 1.0;
    A[e] = v;
  }
}

// y = a*x + b*y elementwise over n complex entries (strided columns)
__global__ __launch_bounds__(NT) void k_axpby(int64_t rows, int cols, cplx a, const cplx* __restrict__ x, int64_t ldx,
                                              cplx b, cplx* __restrict__ y, int64_t ldy) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t r = e % rows;
    const int64_t c = e / rows;
    const cplx xv = x[r + c * ldx];
    cplx* yp = y + r + c * ldy;
    *yp = (b.x == 0.0 && b.y == 0.0) ? cmul(a, xv) : cadd(cmul(a, xv), cmul(b, *yp));
  }
}

// column-wise squared norms (one workgroup per column)
// one 1024-thread workgroup per column, four independent partial sums per thread (more loads in
// flight per CU); fixed summation order
constexpr int NT_NORM = 1024;
__global__ __launch_bounds__(NT_NORM) void k_colnorm2(int64_t rows, const cplx* __restrict__ x, int64_t ldx,
                                                      double* __restrict__ out) {
  const cplx* col = x + (size_t)blockIdx.x * ldx;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t r = threadIdx.x;
  for (; r + 3 * NT_NORM < rows; r += 4 * NT_NORM) {
    a0 += cabs2(col[r]);
    a1 += cabs2(col[r + NT_NORM]);
    a2 += cabs2(col[r + 2 * NT_NORM]);
    a3 += cabs2(col[r + 3 * NT_NORM]);
  }
  for (; r < rows; r += NT_NORM) a0 += cabs2(col[r]);
  double a = wave_sum((a0 + a1) + (a2 + a3));
  __shared__ double red[NT_NORM / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NT_NORM / 64; ++w) t += red[w];
    out[blockIdx.x] = t;
  }
}

// ---- radiation rows of the Wood's-anomaly scheme (Sec. 2.4, second improvement)
// For each listed order m (kappa_m, k_m) the row of the condition "no up-going part of order m below
// the obstacle": row . [eta; xi] = i k_m U_m(-y0) + U_m'(-y0), where U_m is the discrete Fourier
// coefficient of order m of the representation (Eq. 2.14, Eq. 2.20 with P images) sampled at
// x_l = -d/2 + (l + 1/2) d / ns on the line y = -y0 (Remark 2.3), U_m' that of its y-derivative.
//
// Obstacle part, one thread per (node i, order m):
//   R[m + i ldr] = w_i sum_{j=-P..P} alpha^j (1/ns) sum_l e^{-i kappa_m x_l} [i k_m K + dK/dy](p_l; y_i + j d e_1, n_i)
// with K = (i omega/4) H1(omega r) n.D/r + (omega/4) H0(omega r), D = p - y, and its derivative in the
// target's second coordinate (H1' = H0 - H1/z):
//   dK/dy = (i omega/4) [(omega H1'(omega r)/r - H1/r^2)(D_2/r) n.D + H1 n_2/r] - (omega^2/4) H1 D_2/r.
__global__ __launch_bounds__(NT) void k_rad_rows_eta(QPGeo Q, const RadOrder* __restrict__ ord, int ns, int P, cplx alpha,
                                                     double y0, cplx* __restrict__ R, int64_t ldr) {
  const int i = blockIdx.x * NT + threadIdx.x;
  const int m = blockIdx.y;
  if (i >= Q.N) return;
  const RadOrder o = ord[m];
  const cplx ikm = mkc(-o.kn.y, o.kn.x);
  const double nx = Q.nx[i], ny = Q.ny[i];
  const double q = 0.25 * Q.omega;
  cplx acc = mkc(0, 0);
  cplx aj = mkc(1, 0);
  for (int j = 0; j < P; ++j) aj = cmul(aj, cinv(alpha));  // alpha^{-P}
  for (int j = -P; j <= P; ++j) {
    const double sx = Q.x[i] + j * Q.period, sy = Q.y[i];
    cplx part = mkc(0, 0);
    for (int l = 0; l < ns; ++l) {
      const double xl = -0.5 * Q.period + (l + 0.5) * Q.period / ns;
      const double dx = xl - sx, dy = -y0 - sy;
      const double r = sqrt(dx * dx + dy * dy);
      const double z = Q.omega * r;
      cplx h0, h1;
      hankel01(z, h0, h1);
      const double nd = nx * dx + ny * dy;
      // K = q (H0 + i H1 nd / r)
      const cplx K = cscale(cadd(h0, cmul(mkc(0, 1), cscale(h1, nd / r))), q);
      // dK/dy = i q [(omega H1'/r - H1/r^2)(dy/r) nd + H1 ny / r] - q omega H1 dy / r
      const cplx dh1 = csub(h0, cscale(h1, 1.0 / z));
      const cplx br = cadd(cscale(csub(cscale(dh1, Q.omega / r), cscale(h1, 1.0 / (r * r))), dy * nd / r), cscale(h1, ny / r));
      const cplx dK = csub(cmul(mkc(0, q), br), cscale(h1, q * Q.omega * dy / r));
      double s, c;
      sincos(-o.kap * xl, &s, &c);
      part = cadd(part, cmul(mkc(c, s), cadd(cmul(ikm, K), dK)));
    }
    acc = cadd(acc, cmul(aj, part));
    aj = cmul(aj, alpha);
  }
  R[m + (size_t)i * ldr] = cscale(acc, Q.w[i] / ns);
}

// Wall part, one thread per (contour column k in [0, 2M), order m): the Fourier wall potentials
// (Eqs. 2.12-2.13) of mu (k < M) and nu (k >= M) on both walls, L with factor 1 and R with alpha,
// sampled on y = -y0; d/dy multiplies node kk's term by i k_kk:
//   mu:  (i/2) wk e^{-i kk y0} [e^{i s (x_l + d/2)} + alpha e^{i s (d/2 - x_l)}] / s
//   nu:  (1/2) wk e^{-i kk y0} [e^{i s (x_l + d/2)} - alpha e^{i s (d/2 - x_l)}]
__global__ __launch_bounds__(NT) void k_rad_rows_xi(QPGeo Q, const RadOrder* __restrict__ ord, int ns, cplx alpha, double y0,
                                                    cplx* __restrict__ R, int64_t ldr) {
  const int col = blockIdx.x * NT + threadIdx.x;
  const int m = blockIdx.y;
  if (col >= 2 * Q.M) return;
  const RadOrder o = ord[m];
  const int kk = col % Q.M;
  const bool dbl = col >= Q.M;
  const cplx k = Q.k[kk], sq = Q.s[kk], wk = Q.wk[kk];
  // i k_m + i k
  const cplx fac = mkc(-(o.kn.y + k.y), o.kn.x + k.x);
  // wk e^{-i k y0}
  const cplx base = cmul(wk, cexpi_c(mkc(-k.x * y0, -k.y * y0)));
  cplx acc = mkc(0, 0);
  for (int l = 0; l < ns; ++l) {
    const double xl = -0.5 * Q.period + (l + 0.5) * Q.period / ns;
    const cplx eL = cexpi_c(cscale(sq, xl + 0.5 * Q.period));
    const cplx eR = cmul(alpha, cexpi_c(cscale(sq, 0.5 * Q.period - xl)));
    double s, c;
    sincos(-o.kap * xl, &s, &c);
    acc = cadd(acc, cmul(mkc(c, s), dbl ? csub(eL, eR) : cadd(eL, eR)));
  }
  cplx v = cmul(cmul(base, fac), acc);
  v = dbl ? cscale(v, 0.5) : cmul(mkc(0.0, 0.5), cmul(v, cinv(sq)));
  R[m + (size_t)col * ldr] = cscale(v, 1.0 / ns);
}

// Bragg amplitudes (lattice-summed Green's function), one workgroup per (mode slot, angle):
//   c_n = pre sum_j w_j eta_j e^{-i(kap_n x_j + k_n y_j)} [-i(kap_n n_x + k_n n_y) - i omega]
//   d_n = pre sum_j w_j eta_j e^{-i(kap_n x_j - k_n y_j)} [ i(-kap_n n_x + k_n n_y) - i omega]
//   pre = i e^{i k_n y0} / (2 d k_n),  kap_n = kappa + 2 pi n / d, k_n = sqrt(omega^2 - kap_n^2).
__global__ __launch_bounds__(NT) void k_bragg(QPGeo Q, const double* __restrict__ kappa, const int* __restrict__ nlo,
                                              const int* __restrict__ nmodes, int maxmodes, const cplx* __restrict__ eta,
                                              int64_t ldeta, double y0, cplx* __restrict__ out) {
  const int slot = blockIdx.x, a = blockIdx.y;
  cplx* oc = out + (size_t)a * 2 * maxmodes;
  if (slot >= nmodes[a]) {
    if (threadIdx.x == 0) {
      oc[slot] = mkc(0, 0);
      oc[maxmodes + slot] = mkc(0, 0);
    }
    return;
  }
  const double kn_x = kappa[a] + 2.0 * PI * (nlo[a] + slot) / Q.period;
  const double kn = sqrt(fmax(Q.omega * Q.omega - kn_x * kn_x, 0.0));
  const cplx* et = eta + (size_t)a * ldeta;
  cplx su = mkc(0, 0), sd = mkc(0, 0);
  for (int j = threadIdx.x; j < Q.N; j += NT) {
    double s1, c1, s2, c2;
    sincos(-(kn_x * Q.x[j] + kn * Q.y[j]), &s1, &c1);
    sincos(-(kn_x * Q.x[j] - kn * Q.y[j]), &s2, &c2);
    if (Q.two) {
      // tau (double layer) with the factors above less the -i omega; sigma (single layer) with kb
      const cplx wt = cscale(et[2 * j], Q.w[j]), ws = cscale(et[2 * j + 1], Q.w[j] * Q.kb);
      const cplx fu = cadd(cmul(wt, mkc(0.0, -(kn_x * Q.nx[j] + kn * Q.ny[j]))), ws);
      const cplx fd = cadd(cmul(wt, mkc(0.0, -kn_x * Q.nx[j] + kn * Q.ny[j])), ws);
      su = cadd(su, cmul(mkc(c1, s1), fu));
      sd = cadd(sd, cmul(mkc(c2, s2), fd));
      continue;
    }
    const cplx we = cscale(et[j], Q.w[j]);
    const cplx fu = mkc(0.0, -(kn_x * Q.nx[j] + kn * Q.ny[j]) - Q.omega);
    const cplx fd = mkc(0.0, (-kn_x * Q.nx[j] + kn * Q.ny[j]) - Q.omega);
    su = cadd(su, cmul(we, cmul(mkc(c1, s1), fu)));
    sd = cadd(sd, cmul(we, cmul(mkc(c2, s2), fd)));
  }
  su = wave_csum(su);
  sd = wave_csum(sd);
  __shared__ cplx ru[NT / 64], rd[NT / 64];
  if ((threadIdx.x & 63) == 0) { ru[threadIdx.x >> 6] = su; rd[threadIdx.x >> 6] = sd; }
  __syncthreads();
  if (threadIdx.x == 0) {
    cplx tu = mkc(0, 0), td = mkc(0, 0);
    for (int w = 0; w < NT / 64; ++w) { tu = cadd(tu, ru[w]); td = cadd(td, rd[w]); }
    double s, c;
    sincos(kn * y0, &s, &c);
    const cplx pre = cscale(cmul(mkc(0.0, 1.0), mkc(c, s)), 1.0 / (2.0 * Q.period * kn));
    oc[slot] = cmul(pre, tu);
    oc[maxmodes + slot] = cmul(pre, td);
  }
}

// Bragg basis of one Bloch-phase group: the orders shared by its angles are kap_q = kref + 2 pi (qlo + q) / d,
// q < nq.  E (2 nq x N, col-major): row q = w_j e^{-i(kap_q x_j + k_q y_j)} [-i(kap_q n_x + k_q n_y) - i omega],
// row nq + q = w_j e^{-i(kap_q x_j - k_q y_j)} [i(-kap_q n_x + k_q n_y) - i omega]; E eta gives the sums of k_bragg.
// Transmission problem: 2N columns, column 2j (tau) without the -i omega term, column 2j + 1
// (sigma) with the factor Q.kb.
__global__ __launch_bounds__(NT) void k_bragg_basis(QPGeo Q, double kref, int qlo, int nq, cplx* __restrict__ E) {
  const int64_t rows = 2 * (int64_t)nq;
  const int64_t total = rows * (Q.two ? 2 * Q.N : Q.N);
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e % rows);
    const int jc = (int)(e / rows);
    const int j = Q.two ? jc >> 1 : jc;
    const bool up = r < nq;
    const int q = up ? r : r - nq;
    const double kx = kref + 2.0 * PI * (qlo + q) / Q.period;
    const double kn = sqrt(fmax(Q.omega * Q.omega - kx * kx, 0.0));
    const double ky = up ? kn : -kn;
    double sn, cs;
    sincos(-(kx * Q.x[j] + ky * Q.y[j]), &sn, &cs);
    const double om = Q.two ? 0.0 : Q.omega;
    const cplx f = (Q.two && (jc & 1)) ? mkc(Q.kb, 0.0)
                   : up ? mkc(0.0, -(kx * Q.nx[j] + kn * Q.ny[j]) - om) : mkc(0.0, (-kx * Q.nx[j] + kn * Q.ny[j]) - om);
    E[e] = cscale(cmul(mkc(cs, sn), f), Q.w[j]);
  }
}

// out slot s of angle a (a < nang of one group) = pre(k) * Cg[slot0[a] + s, a] (c_n) and the same from
// row nq + slot0[a] + s (d_n), pre = i e^{i k y0} / (2 d k); slots >= nmodes[a] are zero.
__global__ __launch_bounds__(NT) void k_bragg_gather(QPGeo Q, double kref, int qlo, int nq, const int* __restrict__ slot0,
                                                     const int* __restrict__ nmodes, int maxmodes, int nang,
                                                     const cplx* __restrict__ Cg, double y0, cplx* __restrict__ out) {
  const int64_t total = (int64_t)maxmodes * nang;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int sl = (int)(e % maxmodes), a = (int)(e / maxmodes);
    cplx* oc = out + (size_t)a * 2 * maxmodes;
    if (sl >= nmodes[a]) {
      oc[sl] = mkc(0, 0);
      oc[maxmodes + sl] = mkc(0, 0);
      continue;
    }
    const int q = slot0[a] + sl;
    const double kx = kref + 2.0 * PI * (qlo + q) / Q.period;
    const double kn = sqrt(fmax(Q.omega * Q.omega - kx * kx, 0.0));
    double sn, cs;
    sincos(kn * y0, &sn, &cs);
    const cplx pre = cscale(cmul(mkc(0.0, 1.0), mkc(cs, sn)), 1.0 / (2.0 * Q.period * kn));
    const cplx* col = Cg + (size_t)a * 2 * nq;
    oc[sl] = cmul(pre, col[q]);
    oc[maxmodes + sl] = cmul(pre, col[nq + q]);
  }
}

// permute columns: dst[:, perm[a]] = src[:, a]
__global__ __launch_bounds__(NT) void k_permute_cols(int64_t rows, int cols, const int* __restrict__ perm,
                                                     const cplx* __restrict__ src, int64_t lds, cplx* __restrict__ dst,
                                                     int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t r = e % rows;
    const int a = (int)(e / rows);
    dst[r + (size_t)perm[a] * ldd] = src[r + (size_t)a * lds];
  }
}

inline int grid_for(int64_t elems, int cap = 8192) {
  int64_t g = (elems + NT - 1) / NT;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

namespace qps {

hipError_t launch_gen_B(const QPGeo& q, cplx* Y, int64_t ldy, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_B, dim3(grid_for((int64_t)((q.two && !q.idx) ? 2 : 1) * q.N * 4 * q.M)), dim3(NT), 0, s, q, Y, ldy);
  return hipGetLastError();
}
hipError_t launch_gen_inc(const QPGeo& q, const double* kx, const double* ky, const double* ky_im, int nang, cplx* Y,
                          int64_t ldy, hipStream_t s) {
  if (nang == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gen_inc, dim3(grid_for((int64_t)(q.two ? 2 : 1) * q.N * nang)), dim3(NT), 0, s, q, kx, ky, ky_im, nang, Y, ldy);
  return hipGetLastError();
}
hipError_t launch_gen_C(const QPGeo& q, int wall, double shift, cplx* C, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_C, dim3(grid_for((int64_t)((q.two && !q.idx) ? 2 : 1) * q.N * q.M)), dim3(NT), 0, s, q, wall, shift, C);
  return hipGetLastError();
}
hipError_t launch_form_S(const QPGeo& q, const cplx* coef, int ng, const cplx* G1, const cplx* G2, cplx* S, hipStream_t s) {
  if (ng == 0) return hipSuccess;
  int64_t tot = (int64_t)4 * q.M * q.M;
  hipLaunchKernelGGL(k_form_S, dim3(grid_for(tot, 4096), ng), dim3(NT), 0, s, q, coef, G1, G2, S);
  return hipGetLastError();
}
hipError_t launch_lincomb(int rows, int ncol, const cplx* c1, const cplx* c2, int cs, const cplx* U1, int64_t ld1,
                          const cplx* U2, int64_t ld2, const cplx* R, int64_t ldr, cplx* W, int64_t ldw, hipStream_t s) {
  if ((int64_t)rows * ncol == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lincomb, dim3(grid_for((int64_t)rows * ncol)), dim3(NT), 0, s, rows, ncol, c1, c2, cs, U1, ld1, U2,
                     ld2, R, ldr, W, ldw);
  return hipGetLastError();
}
hipError_t launch_qsolve(const QPGeo& q, const cplx* alpha, int cs, int ncol, const cplx* in, int64_t ldi, cplx* out,
                         int64_t ldo, hipStream_t s) {
  if ((int64_t)q.M * ncol == 0) return hipSuccess;
  hipLaunchKernelGGL(k_qsolve, dim3(grid_for((int64_t)q.M * ncol)), dim3(NT), 0, s, q, alpha, cs, ncol, in, ldi, out, ldo);
  return hipGetLastError();
}
hipError_t launch_eye_plus(int n, int ng, const cplx* B, int64_t ldb, int64_t bstride, cplx* A, hipStream_t s) {
  if ((int64_t)n * n * ng == 0) return hipSuccess;
  hipLaunchKernelGGL(k_eye_plus, dim3(grid_for((int64_t)n * n * ng)), dim3(NT), 0, s, n, ng, B, ldb, bstride, A);
  return hipGetLastError();
}
hipError_t launch_stack(int M2, int nang, const cplx* alpha_col, const cplx* xi, cplx* st, hipStream_t s) {
  if (nang == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stack, dim3(grid_for((int64_t)M2 * nang)), dim3(NT), 0, s, M2, nang, alpha_col, xi, st);
  return hipGetLastError();
}
hipError_t launch_resid2(const QPGeo& q, int nang, const cplx* alpha_col, const cplx* c1, const cplx* c2, const cplx* T1,
                         const cplx* T2, const cplx* xi, cplx* R2, hipStream_t s) {
  if (nang == 0) return hipSuccess;
  hipLaunchKernelGGL(k_resid2, dim3(grid_for((int64_t)2 * q.M * nang)), dim3(NT), 0, s, q, nang, alpha_col, c1, c2, T1, T2,
                     xi, R2);
  return hipGetLastError();
}
hipError_t launch_axpby(int64_t rows, int cols, cplx a, const cplx* x, int64_t ldx, cplx b, cplx* y, int64_t ldy, hipStream_t s) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(rows * cols)), dim3(NT), 0, s, rows, cols, a, x, ldx, b, y, ldy);
  return hipGetLastError();
}
hipError_t launch_colnorm2(int64_t rows, int cols, const cplx* x, int64_t ldx, double* out, hipStream_t s) {
  if (cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_colnorm2, dim3(cols), dim3(NT_NORM), 0, s, rows, x, ldx, out);
  return hipGetLastError();
}
hipError_t launch_bragg(const QPGeo& q, const double* kappa, const int* nlo, const int* nmodes, int maxmodes, int nang,
                        const cplx* eta, int64_t ldeta, double y0, cplx* out, hipStream_t s) {
  if (nang == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bragg, dim3(maxmodes, nang), dim3(NT), 0, s, q, kappa, nlo, nmodes, maxmodes, eta, ldeta, y0, out);
  return hipGetLastError();
}
hipError_t launch_bragg_basis(const QPGeo& q, double kref, int qlo, int nq, cplx* E, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bragg_basis, dim3(grid_for((int64_t)2 * nq * (q.two ? 2 : 1) * q.N)), dim3(NT), 0, s, q, kref, qlo, nq, E);
  return hipGetLastError();
}
hipError_t launch_bragg_gather(const QPGeo& q, double kref, int qlo, int nq, const int* slot0, const int* nmodes, int maxmodes,
                               int nang, const cplx* Cg, double y0, cplx* out, hipStream_t s) {
  if (nang == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bragg_gather, dim3(grid_for((int64_t)maxmodes * nang)), dim3(NT), 0, s, q, kref, qlo, nq, slot0, nmodes,
                     maxmodes, nang, Cg, y0, out);
  return hipGetLastError();
}
hipError_t launch_rad_rows(const QPGeo& q, const RadOrder* ord, int c, int ns, int P, cplx alpha, double y0, cplx* Reta,
                           cplx* Rxi, hipStream_t s) {
  if (c == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rad_rows_eta, dim3((q.N + NT - 1) / NT, c), dim3(NT), 0, s, q, ord, ns, P, alpha, y0, Reta, (int64_t)c);
  hipLaunchKernelGGL(k_rad_rows_xi, dim3((2 * q.M + NT - 1) / NT, c), dim3(NT), 0, s, q, ord, ns, alpha, y0, Rxi, (int64_t)c);
  return hipGetLastError();
}

hipError_t launch_permute_cols(int64_t rows, int cols, const int* perm, const cplx* src, int64_t lds, cplx* dst, int64_t ldd,
                               hipStream_t s) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute_cols, dim3(grid_for(rows * cols)), dim3(NT), 0, s, rows, cols, perm, src, lds, dst, ldd);
  return hipGetLastError();
}

}  // namespace qps
