// The solver handle: geometry, tree, per-level skeletonization factors, periodizing cache.
#pragma once
#include <complex>
#include "internal.h"

#include <memory>
#include <vector>

namespace qps {

struct Level {
  int nb = 0;
  std::vector<int> n, k;
  std::vector<int64_t> aoff, soff;  // offsets of active / skeleton lists (prefix sums of n / k)
  int64_t ntot = 0, ktot = 0;
  std::vector<int> hact, hskel;     // host copies of the index lists (global node indices)
  DevBuf act, skel;
  // factors (element offsets into the buffers, per box)
  DevBuf P, E, Ft, G, Df, Dh;
  DevBuf E32, Ft32, G32;            // complex64 inverse factors (FP32-preconditioner mode)
  std::vector<int64_t> oP, oE, oFt, oG, oDh;
  // bounding circles of the boxes' original points
  std::vector<double> cx, cy, rad, aspect;
  std::vector<int> lo, hi;          // original index range
};

}  // namespace qps

// A captured application of the telescoping factorization (HIP graph), replayed while the call
// uses the same operands and the apply workspaces have not moved.
struct ApplyGraph {
  bool inv = false;
  bool root_acc = false;  // the root product accumulates (beta = 1)
  int phase = 0;          // whole apply, upward + root only, or downward only
  int split = 0;
  const void* B = nullptr;
  void* X = nullptr;
  int64_t ldb = 0, ldx = 0, r = 0;
  const void* ws[8] = {};
  hipGraphExec_t exec = nullptr;
  qps::DevBuf d64, d32;  // the graph's own descriptor arrays
};

struct hbs_handle {
  ~hbs_handle();
  // declared first, so destroyed after every buffer charged to it
  qps::MemBudget budget;
  int64_t N = 0;   // nodes
  int64_t NU = 0;  // unknowns: N, or 2N for the transmission problem (two densities per node)
  int nc = 1;      // unknowns per node
  double omega = 0, tol = 0;
  hbs_opts opts{};
  hipStream_t stream = nullptr;
  int L = 0;
  std::vector<double> hx, hy, hnx, hny, hw, hkap;
  qps::DevBuf dgeo, dkressR;
  qps::DevBuf dalp, dalpT;  // Alpert correction: Lagrange weights + node weights, kernel table (N x 2m)
  Geo geo{};
  std::vector<qps::Level> lv;  // lv[1..L]
  int nroot = 0;
  qps::DevBuf Rinv, Rfwd;
  // Rinv: 0 = the root inverse; 1 = still the root matrix (hbs_opts.defer_root); 2 = its inversion is
  // enqueued on the side stream, flag (device) not yet read; 3 = the root matrix was singular
  int root_state = 0;
  const int* root_flag = nullptr;
  int fp64_top = 0;               // levels 1..fp64_top hold complex128 inverse factors, deeper ones complex64
  bool top_identity = false;      // level 1 left uncompressed (root over the level-2 skeletons)
  std::vector<float> rank_model;  // rank-predictor parameters (when hbs_opts.rank_predictor)
  // per box of every level (leaves first): predictor features, CPQR rank, level, predicted rank
  std::vector<float> feat, feat_pred;
  std::vector<int> feat_rank, feat_level;
  qps::DevBuf arena, arena32, work, scratch, splitws, qp32;
  qps::DevBuf ab_up, ab_x0, ab_x1, ab_root;          // apply workspaces
  qps::DevBuf ab_in32, ab_up32, ab_x32a, ab_x32b;    // complex64 stage of a mixed-precision inverse apply
  std::vector<std::unique_ptr<ApplyGraph>> graphs;   // hbs_opts.graph: captured applies (at most 4)
  hipStream_t cap_stream = nullptr;                 // private stream the applies are captured on
  // second stream for work that does not depend on a concurrent apply, with its own descriptor
  // arena and workspaces; side_ev: [ready on the main stream, done on the side stream]
  hipStream_t side_stream = nullptr;
  hipEvent_t side_ev[2] = {nullptr, nullptr};
  qps::DevBuf arena_s, splitws_s, work_s;
  int64_t graph_captures = 0, graph_replays = 0;
  hbs_stats_t stats{};
  double c0x = 0, c0y = 0, robs = 0;  // obstacle centre and radius about it
  int64_t factor_bytes = 0;
  double build_seconds = 0;
};

namespace qps {
// apply the telescoping factorization: inverse (F^T, E, G, root inverse) or forward (P^T, P, D, root coupling)
int apply_factors(hbs_handle* h, bool inverse, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r);
// X = A^{-1} B with whichever inverse factors the handle holds (complex64 levels run on casts)
int apply_inverse(hbs_handle* h, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r);
int build(hbs_handle* h);
int apply_interp(hbs_handle* h, const cplx* Z, int64_t ldz, cplx* X, int64_t ldx, int64_t r);
int apply_interp_t(hbs_handle* h, const cplx* X, int64_t ldx, cplx* Z, int64_t ldz, int64_t r);
// X = E_L ... E_1 Z (complex128 levels only): A^{-1} U from Z = R^{-1}
int apply_down_E(hbs_handle* h, const cplx* Z, int64_t ldz, cplx* X, int64_t ldx, int64_t r);
// X = A^{-1} B and root (nroot x r) = U^T A^{-1} B, the root solution of the same apply
// X = A B (compressed forward operator) with root_add (nroot x r, or null) added to the root's
// downward input, so that X = A B + U root_add, and root_up (nroot x r, or null) = U^T B, the
// upward result at the root (U: the nested interpolation).  Stream-ordered, no host wait.
int apply_forward_root(hbs_handle* h, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r, const cplx* root_add,
                       cplx* root_up);
// A^{-1} B in two calls (complex128 factors only): the upward pass and the root product, with the
// root solution U^T A^{-1} B (nroot x r) copied to root; later the downward pass from root_in
// (nroot x r, ld nroot) instead of that root solution, writing X.  The upward results of B stay
// in the handle's apply workspace in between: no other apply may run on the handle meanwhile.
// root_wait (nullable): an event the root product waits for (the root inverse is formed elsewhere)
int apply_inverse_up(hbs_handle* h, const cplx* B, int64_t ldb, int64_t r, cplx* root, int64_t ldr,
                     hipEvent_t root_wait = nullptr);
// bring Rinv to the root inverse (root_state 0) before it is read; HBS_E_SINGULAR for a singular root
int ensure_root(hbs_handle* h);
int apply_inverse_down(hbs_handle* h, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r, const cplx* root_in);
// (sync = false leaves the work stream-ordered on the handle's stream without waiting for it)
int apply_inverse_root(hbs_handle* h, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r, cplx* root, int64_t ldr,
                       bool sync = true);
// create the side stream and its two events on first use
int side_stream_init(hbs_handle* h);
int qp_max_modes_impl(double om, double period);
struct QPPlan;
// Columns of the Wood's-anomaly scheme (Sec. 2.4): plane waves -exp(i (kx x + ky y)), ky complex, sharing
// the Bloch phase alpha, on the contour displaced to cross the real axis at delta.
struct QPCols {
  double delta = 0.0;
  std::complex<double> alpha{1.0, 0.0};
  std::vector<double> kx;
  std::vector<std::complex<double>> ky;
};
int qp_solve_core(hbs_handle* h, double period, const std::vector<double>& th, const qp_opts* o, const QPCols* cols,
                  cplx* eta_out, cplx* xi_out, cplx* bragg_out, int32_t* nlo_out, int32_t* nm_out, double* flux_out);
int qp_solve_impl(hbs_handle* h, double period, const std::vector<double>& th, const qp_opts* o, cplx* eta_out,
                  cplx* xi_out, cplx* bragg_out, int32_t* nlo_out, int32_t* nm_out, double* flux_out);
int qp_contour_M(const hbs_handle* h, double period, const qp_opts* o);
}  // namespace qps
