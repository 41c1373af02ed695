// Declarations of the periodizing-scheme kernels (kernels_qp.hip).
#pragma once
#include "internal.h"

// Geometry and contour data for the wall blocks (device pointers).
struct QPGeo {
  const double *x, *y, *nx, *ny, *w;
  const cplx *k, *s, *wk;  // contour nodes, sqrt(omega^2 - k^2), quadrature weights
  const int* idx;  // nullable: row / column i of a generated block is node idx[i] (a skeleton subset)
  int N, M;
  double omega, period, shift;
  // transmission problem (Sec. 5): vectors over the obstacle have 2N entries, node by node [tau; sigma]
  // (columns) or [value; minus normal derivative] (rows); the walls see the exterior field only
  int two;
  double kb;  // the transmission normalization max(omega, n omega): sigma columns x kb, derivative rows / kb
};

// An order of the Wood's-anomaly radiation rows: kappa_m = kappa + 2 pi m / d and k_m (complex).
struct RadOrder {
  double kap;
  double pad;
  cplx kn;
};

namespace qps {
// Rows (c x N and c x 2M, column-major, leading dimension c) of the radiation conditions of the
// orders ord[0..c) for the representation with P images and Bloch phase alpha, from ns samples on y = -y0
hipError_t launch_rad_rows(const QPGeo& q, const RadOrder* ord, int c, int ns, int P, cplx alpha, double y0, cplx* Reta,
                           cplx* Rxi, hipStream_t s);
hipError_t launch_gen_B(const QPGeo& q, cplx* Y, int64_t ldy, hipStream_t s);
hipError_t launch_gen_inc(const QPGeo& q, const double* kx, const double* ky, const double* ky_im, int nang, cplx* Y,
                          int64_t ldy, hipStream_t s);
hipError_t launch_gen_C(const QPGeo& q, int wall, double shift, cplx* C, hipStream_t s);
hipError_t launch_form_S(const QPGeo& q, const cplx* coef, int ng, const cplx* G1, const cplx* G2, cplx* S, hipStream_t s);
// W[:, a] = c1[a*cs] U1[:, a] + c2[a*cs] U2[:, a], or R[:, a] - (...) when R != nullptr (W may alias R)
hipError_t launch_lincomb(int rows, int ncol, const cplx* c1, const cplx* c2, int cs, const cplx* U1, int64_t ld1,
                          const cplx* U2, int64_t ld2, const cplx* R, int64_t ldr, cplx* W, int64_t ldw, hipStream_t s);
// out[:, a] = Q(alpha[a cs])^{-1} in[:, a] (2M rows; may alias)
hipError_t launch_qsolve(const QPGeo& q, const cplx* alpha, int cs, int ncol, const cplx* in, int64_t ldi, cplx* out,
                         int64_t ldo, hipStream_t s);
hipError_t launch_eye_plus(int n, int ng, const cplx* B, int64_t ldb, int64_t bstride, cplx* A, hipStream_t s);
hipError_t launch_stack(int M2, int nang, const cplx* alpha_col, const cplx* xi, cplx* st, hipStream_t s);
hipError_t launch_resid2(const QPGeo& q, int nang, const cplx* alpha_col, const cplx* c1, const cplx* c2, const cplx* T1,
                         const cplx* T2, const cplx* xi, cplx* R2, hipStream_t s);
hipError_t launch_axpby(int64_t rows, int cols, cplx a, const cplx* x, int64_t ldx, cplx b, cplx* y, int64_t ldy, hipStream_t s);
hipError_t launch_colnorm2(int64_t rows, int cols, const cplx* x, int64_t ldx, double* out, hipStream_t s);
hipError_t launch_bragg(const QPGeo& q, const double* kappa, const int* nlo, const int* nmodes, int maxmodes, int nang,
                        const cplx* eta, int64_t ldeta, double y0, cplx* out, hipStream_t s);
// Bragg amplitudes of a group of angles sharing a Bloch phase through one basis matrix and a GEMM
hipError_t launch_bragg_basis(const QPGeo& q, double kref, int qlo, int nq, cplx* E, hipStream_t s);
hipError_t launch_bragg_gather(const QPGeo& q, double kref, int qlo, int nq, const int* slot0, const int* nmodes, int maxmodes,
                               int nang, const cplx* Cg, double y0, cplx* out, hipStream_t s);
hipError_t launch_permute_cols(int64_t rows, int cols, const int* perm, const cplx* src, int64_t lds, cplx* dst, int64_t ldd,
                               hipStream_t s);
}  // namespace qps
