// FP64 evaluation of the Hankel functions H0(x), H1(x) of the first kind for real x > 0,
// the kernel of the free-space Helmholtz Green's function G(x) = (i/4) H0(omega |x|)
// (Eq. 2.9) and of its normal derivative.
//
// Three ranges (tables from gen_hankel_tables.py, accurate to < 1e-18 in exact arithmetic):
//   x < HK_XS          ascending series of J0, J1, Y0, Y1 in u = x^2/4 (Horner), with the
//                      logarithmic terms of Y0, Y1 written out;
//   HK_XS <= x < HK_XA piecewise Chebyshev series (Clenshaw) of the slowly varying factor
//                      f_nu(x) = sqrt(pi x/2) exp(-i(x - nu pi/2 - pi/4)) H_nu(x);
//   x >= HK_XA         Hankel's asymptotic series for f_nu in powers of i/x.
// In the last two ranges H_nu = sqrt(2/(pi x)) exp(i(x - nu pi/2 - pi/4)) f_nu(x), and one
// sincos(x) serves both orders.  The absolute error is a few ulp of max(|J|,|Y|) at the
// series / Chebyshev seam (x = 3) and a few ulp of |H| elsewhere.
#pragma once
#include "qps_common.h"
#include "hankel_tables.inc"

#define HK_PI 3.14159265358979323846264338327950288
#define HK_TWO_OVER_PI 0.636619772367581343075535053490057448
#define HK_INV_SQRT2 0.707106781186547524400844362104849039

struct Bessel01 {
  double j0, y0, j1, y1;
};

__device__ inline Bessel01 bessel01_series(double x) {
  const double u = 0.25 * x * x;
  double c0 = hk_c0[HK_NSER - 1], d0 = hk_d0[HK_NSER - 1];
  double c1 = hk_c1[HK_NSER - 1], d1 = hk_d1[HK_NSER - 1];
#pragma unroll
  for (int k = HK_NSER - 2; k >= 0; --k) {
    c0 = fma(c0, u, hk_c0[k]);
    d0 = fma(d0, u, hk_d0[k]);
    c1 = fma(c1, u, hk_c1[k]);
    d1 = fma(d1, u, hk_d1[k]);
  }
  const double L = log(0.5 * x) + HK_EULER_GAMMA;
  Bessel01 b;
  b.j0 = c0;
  b.y0 = HK_TWO_OVER_PI * fma(L, c0, d0);
  b.j1 = 0.5 * x * c1;
  b.y1 = -HK_TWO_OVER_PI / x + HK_TWO_OVER_PI * L * b.j1 - (0.5 / HK_PI) * x * d1;
  return b;
}

// f0 = sqrt(pi x/2) e^{-i(x-pi/4)} H0, f1 = sqrt(pi x/2) e^{-i(x-3pi/4)} H1
__device__ inline void hankel_factor(double x, cplx& f0, cplx& f1) {
  if (x < HK_XA) {
    int j = 0;
#pragma unroll
    for (int q = 1; q < HK_NINT; ++q) j += (x >= hk_edges[q]) ? 1 : 0;
    const double a = hk_edges[j], b = hk_edges[j + 1];
    const double t = (2.0 * x - (a + b)) / (b - a);
    const double t2 = 2.0 * t;
    double v[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const double* c = hk_cheb[j][f];
      double b1 = 0.0, b2 = 0.0;
#pragma unroll
      for (int k = HK_NCHEB - 1; k >= 1; --k) {
        double b0 = fma(t2, b1, c[k] - b2);
        b2 = b1;
        b1 = b0;
      }
      v[f] = fma(t, b1, c[0] - b2);
    }
    f0 = mkc(v[0], v[1]);
    f1 = mkc(v[2], v[3]);
  } else {
    // sum_k i^k a_k / x^k, Horner in z = i/x
    const double r = 1.0 / x;
    cplx s0 = mkc(hk_asym0[HK_NASYM - 1], 0.0), s1 = mkc(hk_asym1[HK_NASYM - 1], 0.0);
#pragma unroll
    for (int k = HK_NASYM - 2; k >= 0; --k) {
      // s = s * (i r) + a_k
      s0 = mkc(hk_asym0[k] - s0.y * r, s0.x * r);
      s1 = mkc(hk_asym1[k] - s1.y * r, s1.x * r);
    }
    f0 = s0;
    f1 = s1;
  }
}

// H0(x), H1(x) of the first kind, x > 0.
__device__ inline void hankel01(double x, cplx& h0, cplx& h1) {
  if (x < HK_XS) {
    Bessel01 b = bessel01_series(x);
    h0 = mkc(b.j0, b.y0);
    h1 = mkc(b.j1, b.y1);
    return;
  }
  cplx f0, f1;
  hankel_factor(x, f0, f1);
  double s, c;
  sincos(x, &s, &c);
  const double amp = sqrt(HK_TWO_OVER_PI / x);
  // e^{i(x - pi/4)} = ((c + s) + i (s - c)) / sqrt(2)
  const cplx e = mkc((c + s) * HK_INV_SQRT2 * amp, (s - c) * HK_INV_SQRT2 * amp);
  h0 = cmul(e, f0);
  // e^{i(x - 3pi/4)} = -i e^{i(x - pi/4)}
  const cplx e1 = mkc(e.y, -e.x);
  h1 = cmul(e1, f1);
}

// J0(x), J1(x) (real parts), needed by the Kress log split.
__device__ inline void bessel_j01(double x, double& j0, double& j1) {
  cplx h0, h1;
  hankel01(x, h0, h1);
  j0 = h0.x;
  j1 = h1.x;
}
