/* qpscatter.h -- C ABI of the MI355X (gfx950) fast direct solver for 2D quasi-periodic
 * Dirichlet scattering (Gillman & Barnett, "A fast direct solver for quasi-periodic
 * scattering problems").
 *
 * Conventions for every entry point:
 *  - Complex arrays are interleaved (re, im) doubles, column-major.  Point arrays are
 *    N x 2 row-major ((x0, y0, x1, y1, ...)).
 *  - With opts->ptr_mode == HBS_PTR_HOST (default) array arguments are host pointers,
 *    borrowed for the duration of the call and copied to / from the GPU.  With
 *    HBS_PTR_DEVICE they are device pointers (e.g. torch tensors' data_ptr()) and no
 *    copies are made.  The mode given at hbs_build applies to every later call on
 *    that handle.
 *  - All GPU work of a handle runs on opts->stream (a hipStream_t; NULL = the default
 *    stream).  Calls return after the results are complete.
 *  - Status codes: 0 on success, a negative HBS_E_* code otherwise; the text of the last
 *    error of the calling thread is returned by hbs_last_error().  Validation errors are
 *    detected on the host before any GPU work.
 *  - A handle may be used by one call at a time; distinct handles may be used
 *    concurrently from different threads.
 */
#ifndef QPSCATTER_H
#define QPSCATTER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HBS_OK = 0,
  HBS_E_INVALID_ARG = -1,   /* bad size, pointer, option or non-unit normal */
  HBS_E_NONFINITE = -2,     /* NaN / Inf in an input array */
  HBS_E_OOM = -3,           /* device allocation failed or mem_limit exceeded */
  HBS_E_DEVICE = -4,        /* HIP runtime error (text in hbs_last_error) */
  HBS_E_SINGULAR = -6,      /* zero pivot in a diagonal block, the root or a Schur complement */
  HBS_E_NOT_CONVERGED = -7, /* refinement did not reach qp_opts.refine_tol */
  HBS_E_ALPHA_MISMATCH = -8,/* |alpha - exp(i omega d cos theta)| > 1e-12 for some theta */
  HBS_E_WOOD = -9           /* an angle is within qp_opts.wood_min_kn of a Wood's anomaly */
};

enum { HBS_QUAD_KR6 = 0, HBS_QUAD_KRESS = 1, HBS_QUAD_ALPERT = 2 };
enum { HBS_COMPRESS_PROXY = 0, HBS_COMPRESS_EXACT = 1 };
enum { HBS_PTR_HOST = 0, HBS_PTR_DEVICE = 1 };
enum { HBS_FP64 = 0, HBS_FP32_PRECOND = 1 };

typedef struct hbs_handle hbs_handle;

typedef struct {
  int32_t struct_size;      /* sizeof(hbs_opts); set by hbs_opts_init */
  int32_t quad;             /* HBS_QUAD_KR6 (Sec. 2.3), HBS_QUAD_KRESS (needs curvature) or
                               HBS_QUAD_ALPERT (Alpert's hybrid Gauss-trapezoidal correction, the
                               alternative Sec. 2.3 names: 5 off-grid nodes on each side of the target,
                               grid nodes closer than 6 left out, order about 11; the off-grid density
                               and position are 12-point Lagrange interpolants of the node arrays, the
                               normal and speed come from the interpolant's derivative) */
  int32_t compress;         /* HBS_COMPRESS_PROXY (proxy circles) or HBS_COMPRESS_EXACT
                               (true off-diagonal blocks; required with KRESS, O(N^2)) */
  int32_t leaf_size;        /* max points per leaf box; 0 -> 64 */
  double proxy_ratio;       /* proxy circle radius / box radius; 0 -> 2.0 */
  int32_t proxy_min;        /* minimum proxy points per circle; 0 -> 64 */
  int32_t ptr_mode;         /* HBS_PTR_HOST or HBS_PTR_DEVICE */
  const double* curvature;  /* KRESS only: signed curvature at the N nodes (ptr_mode) */
  void* stream;             /* hipStream_t, NULL = default stream */
  uint64_t seed;            /* seed of the sketching matrices of the interpolative decompositions */
  double far_radius;        /* > 0: every skeleton also represents sources and targets outside the
                               circle of this radius about the centre of the nodes' bounding box
                               (needed by qp_solve with P >= 1, whose neighbour images must lie
                               outside it unless image_period is set, and by
                               qp_opts.compress_walls); 0 = off */
  int32_t precision;        /* HBS_FP64: inverse factors in complex128.  HBS_FP32_PRECOND: the inverse
                               factors of the deep levels are built and applied in complex64 on FP32
                               matrix cores and serve as a preconditioner; skeletons, the forward
                               operator, the top levels, the root and all residuals stay FP64, and
                               refinement (hbs_apply's `refine`, qp_solve's refine_max_iter) recovers
                               FP64 accuracy */
  int32_t fp64_top_levels;  /* HBS_FP32_PRECOND only: levels 1..t below the root keep complex128
                               factors (their reduced systems are the worst conditioned), deeper
                               levels complex64; <0 -> 0, 0 -> 3 */
  int32_t rank_predictor;   /* 1: size each box's sketch from the rank predicted by a small MLP
                               (16 geometric features -> log k) instead of the worst case 2n + 8;
                               a box whose CPQR rank reaches the sketch size is redone at full size,
                               so ranks and skeletons stay those of the adaptive CPQR.  0 = off */
  double rank_scale;        /* factor on the predicted rank (0 -> 1); values < 1 force the fallback */
  const float* rank_model;  /* host pointer to qps_rank_model_size() floats (layout of qps_mlp_forward);
                               NULL -> the library's built-in model */
  int32_t root_level;       /* 1: the root holds the skeletons of the two level-1 boxes (Sec. 4);
                               2: level 1 is left uncompressed (P = I) and the root holds the
                               level-2 skeletons; 0 (default): 2 when the rank predictor expects
                               the level-1 decomposition to keep >= 60% of its points and the root
                               stays within 1024 points, else 1 */
  int32_t graph;            /* 1: each application of the factorization (hbs_apply, hbs_forward and the
                               applies inside qp_solve) is captured into a HIP graph on a private
                               stream and replayed while a later call uses the same operands and
                               workspaces (up to 4 captured operand sets per handle); 0 = off */
  uint64_t mem_limit;       /* > 0: largest number of device bytes the handle may hold at once, its
                               factors and the workspaces of the calls made on it together (buffers
                               are counted at the size requested from the library's pool); a call
                               that would exceed it fails with HBS_E_OOM before allocating, and
                               hbs_last_error names the limit.  0 = no limit */
  double image_period;      /* > 0: the skeletons also represent the obstacle's two neighbour images at
                               +-image_period along x (Sec. 3.2, the near points of Fig. 3.1): the
                               active points of every image box that comes inside a box's proxy circle
                               (inside far_radius for a box without proxies) are explicit columns of
                               its interpolative decomposition, in both directions.  Then
                               A_{+-1} = U A_{+-1}(J, :) holds however close the images come, and
                               qp_solve with P = 1 and this period needs no separation of the images
                               from far_radius.  Needs far_radius > 0; 0 = off */
  int32_t defer_root;       /* 1: hbs_build leaves the inversion of the root matrix (Sec. 4) to the first
                               call that needs it: qp_solve on compressed walls runs it in one batch with
                               its Woodbury capacitance inversions, on a second stream while the first
                               stream applies the tree's upward pass; other calls invert it on entry.
                               A singular root is then reported by that call (HBS_E_SINGULAR), and
                               build_seconds leaves the root inversion out.  0 = in hbs_build */
  double index;             /* > 0: the transmission problem of Sec. 5 instead of the Dirichlet problem:
                               refractive index n of the obstacle (wavenumber n omega inside, omega
                               outside), matching conditions of Eqs. 5.3-5.4.  The unknowns are the
                               densities tau (double layer) and sigma (single layer) of both sides'
                               potentials (u = D tau + kb S sigma on both sides, kb = max(omega,
                               n omega)), interlaced node by node as Sec. 5.3 asks: 2N unknowns
                               [tau_1; sigma_1; tau_2; ...], row 2i the value jump at node i and row
                               2i + 1 minus the normal-derivative jump divided by kb, so that the
                               operator is I + [[D0 - D1, kb (S0 - S1)], [-(T0 - T1) / kb,
                               -(D0* - D1*)]] (T the normal derivative of D, D* that of S; 0 and 1 the
                               two wavenumbers), every block with the Kapur-Rokhlin weights; the factor
                               kb brings the four blocks to one size, which the decompositions'
                               relative tolerance needs.  Every N-sized vector of the other calls
                               (hbs_apply's rhs, qp_solve's eta) then has 2N rows, and leaf_size counts
                               unknowns.  Needs HBS_QUAD_KR6 and rank_predictor = 0.  qp_solve takes
                               P = 0 or 1 and refuses angles near a Wood's anomaly (HBS_E_WOOD).  It
                               compresses the wall blocks only when compress_walls = 1 or 2 (at
                               omega = 60 they then lose accuracy to about 6e-10 with 1; 2 refines
                               that away).
                               0 = the Dirichlet problem */
} hbs_opts;

typedef struct {
  int32_t struct_size;      /* sizeof(qp_opts) */
  int32_t P;                /* neighbour images on each side (Sec. 2.4): 0 or 1 */
  int32_t M;                /* contour nodes; 0 -> ceil(2K/h) */
  double K;                 /* contour half-width in Re k; 0 -> sqrt(omega^2 + (37/g)^2) */
  double h;                 /* contour spacing; 0 -> 0.1 */
  double ca, cb;            /* contour k(t) = t - i ca tanh(t / cb); 0 -> 1, 1 */
  double y0;                /* Bragg reference height; 0 -> max|y| + 0.5 */
  double wood_min_kn;       /* angles with min_n |k_n| below this are within reach of a Wood's
                               anomaly (the undisplaced contour loses accuracy there); 0 -> 0.75 */
  int32_t refine_max_iter;  /* iterative refinement steps of the bordered system; <0 -> 0,
                               0 -> 2 (3 for a handle built with HBS_FP32_PRECOND) */
  double refine_tol;        /* stop when the relative residual is below; 0 -> 1e-13 */
  int32_t compress_walls;   /* the wall blocks B (Eq. 2.16) and C (Eq. 2.17) through the root skeletons:
                               B = U B(J, :), C = C(:, J) U^T with U the nested interpolation of the
                               tree, valid when the handle's far_radius circle excludes the walls
                               (far_radius <= d/2 - |c_x|, c = centre of the nodes' bounding box).
                               Then A^{-1} is applied to root-size + q columns instead of 4M + q and
                               no N-sized Schur product is formed.  0 = when valid (the Dirichlet
                               problem; never for the transmission problem, see hbs_opts.index),
                               1 = required (HBS_E_INVALID_ARG otherwise), -1 = never,
                               2 = as 1 for the solve, while the refinement's residual takes B and C
                               uncompressed (formed in full: 16 (4M N + 4M N) bytes more device
                               memory), so that its corrections remove what the skeletons leave out
                               of the wall blocks; the displaced-contour solves of Wood's-anomaly
                               angles, and calls with refine_max_iter < 0, take 1 */
  int32_t wood;             /* angles within wood_min_kn of a Wood's anomaly (Sec. 2.4, second
                               improvement): 0 = solve them on the Sommerfeld contour displaced to cross
                               the real axis at wood_shift, with one added Rayleigh-Bloch wave and one
                               no-incoming-radiation row per order whose pole the contour crossed (the
                               angles of each Bloch phase in one extra pass); -1 = refuse (HBS_E_WOOD).
                               Their xi holds the densities at the displaced contour's nodes */
  double wood_shift;        /* real-axis crossing of the displaced contour; 0 -> chosen per Bloch phase
                               in [0.25, 3] to keep every pole +-k_n farthest from the real axis of the
                               contour's parameter t */
  int32_t wood_samples;     /* samples on y = -y0 of the radiation rows' Fourier coefficients; 0 -> the
                               smallest count >= 64 whose aliases of the propagating orders decay by
                               e^-37 between y = -y0 and the obstacle:
                               (omega + sqrt(omega^2 + (37 / (y0 - max|y|))^2)) d / (2 pi) */
} qp_opts;

typedef struct {
  int32_t struct_size;
  int32_t levels;           /* tree depth L (leaves at level L, root at 0) */
  int64_t N;
  int32_t root_size;        /* size of the dense root matrix */
  int32_t max_rank;         /* largest skeleton rank over all boxes */
  int64_t factor_bytes;     /* device bytes held by the factors */
  double build_seconds;
  int32_t ranks_per_level_max[32];
  double ranks_per_level_mean[32];
  int32_t refine_iters;     /* refinement iterations of the last qp_solve */
  double refine_residual;   /* relative residual after the last qp_solve */
  int32_t contour_M;        /* contour size of the last qp_solve */
  int32_t walls_compressed; /* 1 if the last qp_solve took B and C through the root skeletons, 2 if
                               its refinement also took them uncompressed (compress_walls = 2) */
  int32_t rank_fallbacks;   /* boxes whose predicted sketch was too short (rank_predictor) */
  int64_t sketch_bytes_max; /* largest per-level sketch buffer of the build */
  double cpqr_work;         /* sum over boxes of sketch rows x n x k (CPQR cost measure) */
  int32_t root_level;       /* 1 or 2 (see hbs_opts.root_level) */
  int64_t graph_captures;   /* applies captured into HIP graphs (hbs_opts.graph) */
  int64_t graph_replays;    /* applies served by replaying a captured graph */
  int64_t device_bytes_peak;/* largest device bytes held at once by the handle and its calls */
  int32_t wood_angles;      /* angles of the last qp_solve solved on a displaced contour */
  int32_t wood_orders;      /* Rayleigh-Bloch waves added for them (summed over Bloch phases) */
  double wood_shift;        /* real-axis crossing of the last displaced contour (0 = none) */
  int64_t image_samples;    /* image points taken as explicit columns over all boxes and levels
                               (hbs_opts.image_period) */
  int64_t unknowns;         /* length of the handle's vectors: N, or 2N for the transmission problem */
} hbs_stats_t;

void hbs_opts_init(hbs_opts* o);
void qp_opts_init(qp_opts* o);

/* Build the compressed (HBS) inverse of the Nystrom matrix A = I/2 + D - i omega S of the
 * isolated obstacle (Sec. 2.2 below Eq. 2.15, discretized as in Sec. 2.3) by recursive
 * skeletonization (Sec. 4, Eqs. 4.1-4.8; interpolative decomposition of Def. 3.1 with proxy
 * circles as in Sec. 3.2).
 *   nodes   N x 2   trapezoid nodes y_j = z(2 pi j / N), counter-clockwise
 *   weights N       w_j = (2 pi / N) |z'(t_j)|  (> 0)
 *   normals N x 2   outward unit normals
 *   omega > 0, tol in [1e-15, 1e-2] (relative tolerance of each interpolative decomposition).
 *   N >= 2 * leaf_size and N >= 13 (KR6) / even (KRESS).
 * On success *out holds a handle owning all device memory of the factors. */
int hbs_build(const double* nodes, const double* weights, const double* normals, int64_t N,
              double omega, double tol, const hbs_opts* opts, hbs_handle** out);

/* out = A^{-1} rhs through the compressed inverse (Eq. 4.3 applied level by level),
 * followed by `refine` steps of iterative refinement against the compressed forward operator.
 *   rhs, out: N x nrhs complex (may not alias); nrhs = 0 returns HBS_OK and touches nothing
 *   (hbs_forward and hbs_apply_noalloc likewise). */
int hbs_apply(hbs_handle* h, const double* rhs, int64_t nrhs, double* out, int32_t refine);

/* hbs_apply for callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same result as hbs_apply(h, rhs, nrhs, out, refine)
 * (the same kernels), but every workspace of the call is carved from a static per-device scratch
 * array of 64 MiB (each GPU holds it from the first such call on it until the process ends) and the
 * call makes no hipMalloc / hipFree.  The handle must be built with HBS_PTR_DEVICE; rhs and out are
 * device pointers (N x nrhs complex, may not alias); refine in [0, 16]; graph capture of the handle
 * (hbs_opts.graph) is not used for this call.  Returns HBS_E_OOM, before any GPU work when the level,
 * root and refinement buffers alone are too large, when the workspaces of nrhs columns exceed the
 * scratch (about 5-8 MB per column at N = 1e5).  All calls on one GPU share its scratch, which keeps the
 * last call's contents (every workspace is written before it is read): calls that overlap on one GPU
 * (other threads, other streams) race and must be serialised by the caller. */
int hbs_apply_noalloc(hbs_handle* h, const double* rhs, int64_t nrhs, double* out, int32_t refine);

/* out = A x with the compressed forward operator (the telescoping factorization of Eq. 4.8
 * built from the same skeletons); relative accuracy ~ tol.  x, out: N x nrhs complex. */
int hbs_forward(hbs_handle* h, const double* x, int64_t nrhs, double* out);

/* Solve the quasi-periodic problem (Eq. 1.1 restricted to the unit cell, Sec. 2.1) for the q
 * incident angles thetas[q] in (-pi, 0) that share the Bloch phase alpha = alpha_re + i alpha_im
 * (Eq. 1.2), with period d, by the block solve of Sec. 3.1 (Eq. 3.1) on the bordered system of
 * Eq. 2.19 (Eq. 2.21 with P = 1 neighbour images, Woodbury form of Eq. 3.2) and iterative
 * refinement of the bordered system.
 *   eta      N x q complex   obstacle densities (required)
 *   xi       2M x q complex  wall densities [mu; nu] (nullable)
 *   bragg    (2 mx) x q complex, mx = qp_max_modes(omega, d) (nullable): for angle a, rows
 *            0..n_modes_out[a]-1 hold c_n (Eq. 2.5) and rows mx..mx+n_modes_out[a]-1 hold d_n
 *            (Eq. 2.6) of the propagating orders n = nlo_out[a], nlo_out[a]+1, ...; other rows unset
 *   flux_err q doubles, energy-balance error of Remark 6.1 (nullable)
 * q = 0 returns HBS_OK at once and writes nothing (thetas and eta may then be NULL). */
int qp_solve(hbs_handle* h, double period, double alpha_re, double alpha_im, const double* thetas,
             int64_t q, const qp_opts* opts, double* eta, double* xi, double* bragg,
             int32_t* nlo_out, int32_t* n_modes_out, double* flux_err);

/* Same for n angles with any Bloch phases: the angles are grouped by alpha internally and all
 * groups share one application of A^{-1} to [B_L | B_R | b_1..b_n] (Remark 3.1). */
int qp_solve_many(hbs_handle* h, double period, const double* thetas, int64_t n, const qp_opts* opts,
                  double* eta, double* xi, double* bragg, int32_t* nlo_out, int32_t* n_modes_out,
                  double* flux_err);

/* Number of contour nodes M that qp_solve will use for this handle and options (xi is 2M x q). */
int32_t qp_contour_size(const hbs_handle* h, double period, const qp_opts* opts);
/* Upper bound on the number of Bragg orders returned per angle. */
int32_t qp_max_modes(double omega, double period);

int hbs_stats(const hbs_handle* h, hbs_stats_t* s);
void hbs_free(hbs_handle* h);                 /* NULL is a no-op */
const char* hbs_last_error(void);             /* thread-local; "" if none */

/* Device memory of freed handles and workspaces is kept by the library (per device, up to
 * QPS_POOL_MAX_GB GiB, default 64; when the blocks of the latest call do not fit, blocks cached
 * earlier are returned first) and reused by later builds and solves.  qps_pool_release
 * returns the cached blocks of the current device to HIP; qps_pool_cached_bytes reports them. */
int qps_pool_release(void);
int64_t qps_pool_cached_bytes(void);

/* ------------------------------------------------------------- rank predictor -------
 * A 16-64-64-1 tanh MLP in FP32 predicting log(rank) of a box from 16 geometric features.
 * Parameter vector (qps_rank_model_size() floats): mu[16], sd[16] (input normalisation
 * (x - mu) / sd), W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3.  The features of every box
 * of a built handle, with the CPQR ranks as targets, are the training data.  All arrays are host
 * or device pointers by ptr_mode; x is n x 16 row-major. */
int32_t qps_rank_model_size(void);
/* copies the built-in model into out (qps_rank_model_size() floats); HBS_E_INVALID_ARG if the
 * library was built without one */
int qps_rank_model_default(float* out);
/* features (count x 16, row-major), CPQR ranks, levels and predicted ranks (0 without the
 * predictor) of the boxes of h, leaves first; host pointers, capacity cap boxes (NULL to query
 * *count only) */
int qps_rank_features(const hbs_handle* h, float* feats, int32_t* ranks, int32_t* levels, float* predicted,
                      int64_t cap, int64_t* count);
/* y[b] = model(x[b]) (log of the rank) */
int qps_mlp_forward(const float* params, const float* x, int64_t n, float* y, int32_t ptr_mode);
/* pinball loss at quantile tau summed over the n samples (r = t - y: tau r if r > 0 else
 * (tau - 1) r) and its gradient with respect to the parameters (zero for mu, sd) */
int qps_mlp_grad(const float* params, const float* x, const float* t, int64_t n, float tau, float* grad, float* loss,
                 int32_t ptr_mode);
/* steps of full-batch Adam (lr; betas 0.9, 0.999) on the mean pinball loss, params updated in
 * place (mu, sd kept); loss_hist (steps floats, nullable) receives the mean loss before each step */
int qps_mlp_train(float* params, const float* x, const float* t, int64_t n, float tau, int32_t steps, float lr,
                  float* loss_hist, int32_t ptr_mode);

/* ---------------------------------------------------------------- diagnostics ---------
 * Unit-level access to the device kernels, used by the parity tests. */

/* H0(x_i), H1(x_i) for x_i > 0 evaluated on the GPU; out = 2 x n complex (H0 row then H1). */
int qps_hankel01(const double* x, int64_t n, double* out, int32_t ptr_mode);
/* The symmetric Kapur-Rokhlin 6th-order corrections g_1..g_6 (R_m = 1 + g_m, Sec. 2.3) as
 * derived by the library (host, long double). */
int qps_kr6_corrections(double out[6]);
/* Nodes x[m] (ascending, in (0, a)) and weights w[m] of Alpert's correction with m off-grid nodes
 * per side and the grid nodes closer than a left out, as the library derives them (Newton's method in
 * long double on the conditions of the generalized Euler-Maclaurin expansion, Sec. 2.3's named
 * alternative to Kapur-Rokhlin); m in [1, 8], a in [1, 12]; HBS_E_NOT_CONVERGED if Newton fails. */
int qps_alpert_rule(int32_t m, int32_t a, double* x, double* w);
/* Entries A(rows[t], cols[t]) of the Nystrom matrix of the handle, evaluated on the GPU (indices of
 * the handle's unknowns: 0 .. hbs_stats.unknowns - 1). */
int qps_matrix_entries(hbs_handle* h, const int32_t* rows, const int32_t* cols, int64_t n, double* out);
/* Batched complex GEMM C_b = A_b B_b (+ C_b if accumulate) on the GPU with the library's
 * MFMA kernel: nbatch equal-size problems, A: m x k, B: k x n, C: m x n, col-major, packed. */
int qps_zgemm(const double* A, const double* B, double* C, int32_t m, int32_t n, int32_t k,
              int32_t nbatch, int32_t transA, int32_t accumulate, int32_t ptr_mode);
/* In-place inversion of nbatch square n x n complex matrices (Gauss-Jordan, partial pivoting). */
int qps_zinv(double* A, int32_t n, int32_t nbatch, int32_t ptr_mode);
/* The complex64 variants used by HBS_FP32_PRECOND (interleaved (re, im) floats, FP32 MFMA). */
int qps_cgemm(const float* A, const float* B, float* C, int32_t m, int32_t n, int32_t k,
              int32_t nbatch, int32_t transA, int32_t accumulate, int32_t ptr_mode);
int qps_cinv(float* A, int32_t n, int32_t nbatch, int32_t ptr_mode);

/* Kernel-time profiling with HIP events on the handle's stream.  When enabled, each launch
 * of a kernel family is bracketed by events; qps_profile_read returns the summed time (ms),
 * launch count and summed algorithmic flops of the family ("zgemm", "cgemm", "zinv", "cinv",
 * "cpqr", "sketch", "assemble", "apply", "bragg").  Enabling resets the counters. */
int qps_profile_enable(int32_t on);
int qps_profile_read(const char* family, double* ms, int64_t* launches, double* flops, double* bytes);

/* Tile configurations of the batched complex GEMM that carries every block product of the
 * factorization and its application (the per-level products of the telescoping factorization,
 * Sec. 4, and the Schur products of the block solve of the periodizing step, Sec. 3).  Configuration c:
 * 0 = 64 x 64 output tiles (2 x 2 wavefronts), 1 = 32 x 32 (one wavefront), 2 = 64 x 32 (2 x 1),
 * 3 = 32 x 64 (1 x 2).  Each launch picks one from its shape class through a tuning table; all
 * configurations give bitwise equal results, so the table affects run time only.
 *
 * qps_gemm_class: the class key of a launch (complex64 != 0 for the complex64 kernel; the largest
 *   m, n, k of its entries and the entry count; all >= 0).  Key = prec << 24 | ceil(log2 m) << 18
 *   | ceil(log2 n) << 12 | ceil(log2 k) << 6 | ceil(log2 count), each ceil(log2) of max(x, 1).
 * qps_gemm_tune_lookup: *cfg = the table's configuration for key, or -1 (configuration 0 is used).
 * qps_gemm_tune_set: replace the table by n (key, cfg) pairs (host arrays; cfg outside 0..3 is
 *   an error); n = 0 empties it, n < 0 restores the built-in table.  Launches planned afterwards
 *   use the new table (captured apply graphs keep the configuration they were captured with).
 * qps_gemm_tune_get: copy up to cap entries (keys ascending) into keys/cfgs (may be NULL when
 *   cap = 0); *n = the table size.
 * qps_gemm_tune_begin: start a sweep: every launch uses configuration cfg, and each class's
 *   launches outside graph capture are timed with HIP events.  qps_gemm_tune_end: wait for
 *   the timed launches, return up to cap classes (keys ascending) with their summed ms and
 *   launch counts, *n = the number of classes timed, and end the sweep (table lookups again).
 *   One sweep at a time per process; calls from other threads during a sweep are forced too. */
#define QPS_GEMM_CONFIGS 4
int qps_gemm_class(int32_t complex64, int64_t max_m, int64_t max_n, int64_t max_k, int64_t count, int32_t* key);
int qps_gemm_tune_lookup(int32_t key, int32_t* cfg);
int qps_gemm_tune_set(const int32_t* keys, const int32_t* cfgs, int32_t n);
int qps_gemm_tune_get(int32_t* keys, int32_t* cfgs, int32_t cap, int32_t* n);
int qps_gemm_tune_begin(int32_t cfg);
int qps_gemm_tune_end(int32_t* keys, double* ms, int64_t* launches, int32_t cap, int32_t* n);

#ifdef __cplusplus
}
#endif
#endif
