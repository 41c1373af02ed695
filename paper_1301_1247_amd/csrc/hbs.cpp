// Recursive skeletonization (Sec. 4) of the Nystrom matrix on the GPU, and the application of
// its telescoping factorizations.
//
// Tree: level l has 2^l boxes of contiguous node ranges (curve order); leaves at level L.
// Per level, for every box (all boxes of a level batched into one launch per step):
//   1. D = A(I, I) at the leaves, or [[Dh_a, A(J_a, J_b)], [A(J_b, J_a), Dh_b]] above (Eq. 4.8):
//      the diagonal block of the reduced matrix on the active set I = J_a u J_b.
//   2. W^T = [A(I, near)^T | A(near, I) | proxy columns] (Sec. 3.2 proxy idea applied per box),
//      sketched to 2n+8 rows with a complex Rademacher matrix when longer.
//   3. Interpolative decomposition (Def. 3.1) by column-pivoted QR: skeleton J, P = Pi [I; T^T].
//   4. With U = V = P (one joint skeleton for rows and columns), Eqs. 4.4-4.7:
//      Dh = (P^T D^{-1} P)^{-1}, E = D^{-1} P Dh, F^T = Dh P^T D^{-1}, G = D^{-1} - E P^T D^{-1}.
// The root holds [[Dh_1, A(J_1, J_2)], [A(J_2, J_1), Dh_2]], inverted densely.
// The forward operator of Eq. 4.8 uses the same skeletons: P, the leaf blocks A(I, I), the
// sibling couplings and the root coupling.
#include "hbs.h"
#include "mlp.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>

namespace qps {

namespace {

struct LaunchRec {
  size_t off;
  int cnt;
  GemmPlan plan;
  double flops;
};

GemmDesc gd(const cplx* A, int lda, int transA, const cplx* B, int ldb, cplx* C, int ldc, int m, int n, int k,
            cplx alpha = mkc(1, 0), cplx beta = mkc(0, 0)) {
  GemmDesc g;
  g.A = A; g.B = B; g.C = C;
  g.m = m; g.n = n; g.k = k;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc;
  g.transA = transA; g.pad = 0;
  g.alpha = alpha; g.beta = beta;
  return g;
}

#define CK(expr)                                                                                  \
  do {                                                                                            \
    hipError_t _e = (expr);                                                                       \
    if (_e != hipSuccess) {                                                                       \
      set_error(std::string("hbs_build: ") + #expr + ": " + hipGetErrorString(_e));               \
      return _e == hipErrorOutOfMemory ? HBS_E_OOM : HBS_E_DEVICE;                                \
    }                                                                                             \
  } while (0)

// Descriptor upload into the arena.  The copy from pageable host memory is staged before the call
// returns and is ordered on the stream after the kernels that read the previous contents, so no
// host synchronisation is needed between consecutive uploads and launches.
template <class T>
hipError_t up_sync(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  return upload(b, v, s);
}

}  // namespace

int build(hbs_handle* h) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = h->stream;
  const int64_t N = h->N;
  const int leaf = h->opts.leaf_size;
  // leaf_size counts unknowns (two per node for the transmission problem); boxes split the nodes
  int L = (int)std::ceil(std::log2((double)h->NU / (double)leaf));
  if (L < 1) L = 1;
  while ((N >> L) < 2 && L > 1) --L;
  h->L = L;
  if (h->opts.precision == HBS_FP32_PRECOND) {
    const int t = h->opts.fp64_top_levels;
    h->fp64_top = std::min(L, t < 0 ? 0 : (t == 0 ? 3 : t));
  } else {
    h->fp64_top = L;
  }
  h->lv.clear();
  h->lv.resize(L + 1);
  const bool exact = h->opts.compress == HBS_COMPRESS_EXACT;
  const double ratio = h->opts.proxy_ratio;
  const int pmin = h->opts.proxy_min;
  const double om = h->omega;
  const double om_max = h->geo.two ? std::max(om, h->geo.omega1) : om;  // the proxies resolve both wavenumbers

  // far-field circle (neighbour images lie outside radius far_radius about the obstacle's centre)
  {
    double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
    for (int64_t i = 0; i < N; ++i) {
      x0 = std::min(x0, h->hx[i]); x1 = std::max(x1, h->hx[i]);
      y0 = std::min(y0, h->hy[i]); y1 = std::max(y1, h->hy[i]);
    }
    h->c0x = 0.5 * (x0 + x1);
    h->c0y = 0.5 * (y0 + y1);
    double r = 0;
    for (int64_t i = 0; i < N; ++i) {
      const double dx = h->hx[i] - h->c0x, dy = h->hy[i] - h->c0y;
      r = std::max(r, dx * dx + dy * dy);
    }
    r = std::sqrt(r);
    h->robs = r;
    if (h->opts.far_radius > 0 && !(h->opts.far_radius > 1.05 * r)) {
      set_error("hbs_build: far_radius must exceed the obstacle's radius about its centre");
      return HBS_E_INVALID_ARG;
    }
  }
  const bool far_on = h->opts.far_radius > 0;
  const bool img_on = h->opts.image_period > 0;
  const double Rfar = far_on ? std::sqrt(h->robs * h->opts.far_radius) : 0.0;
  const int npfar = far_on ? std::max(pmin, 2 * (int)std::ceil(om_max * Rfar + std::log(1.0 / h->tol) /
                                                                  std::log(Rfar / h->robs)) + 8) : 0;

  // box ranges, bounding circles and the predictor's geometric features (max and mean |curvature|,
  // arc length) of the original points, all levels in one launch
  std::vector<std::vector<double>> kmaxb(L + 1), kmeanb(L + 1), arcb(L + 1);
  {
    std::vector<int> blo, bhi;
    for (int l = 1; l <= L; ++l) {
      Level& V = h->lv[l];
      V.nb = 1 << l;
      V.lo.resize(V.nb);
      V.hi.resize(V.nb);
      for (int b = 0; b < V.nb; ++b) {
        V.lo[b] = (int)((int64_t)b * N / V.nb);
        V.hi[b] = (int)((int64_t)(b + 1) * N / V.nb);
        blo.push_back(V.lo[b]);
        bhi.push_back(V.hi[b]);
      }
    }
    const int nbox = (int)blo.size();
    DevBuf dlo, dhi, dcirc;
    CK(dlo.reserve(sizeof(int) * nbox));
    CK(dhi.reserve(sizeof(int) * nbox));
    CK(dcirc.reserve(sizeof(double) * 10 * nbox));
    CK(hipMemcpyAsync(dlo.p, blo.data(), sizeof(int) * nbox, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(dhi.p, bhi.data(), sizeof(int) * nbox, hipMemcpyHostToDevice, st));
    CK(launch_box_circles(h->geo, dlo.as<int>(), dhi.as<int>(), nbox, dcirc.as<double>(), st));
    std::vector<double> circ(10 * (size_t)nbox);
    CK(hipMemcpyAsync(circ.data(), dcirc.p, sizeof(double) * 10 * nbox, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    size_t q = 0;
    for (int l = 1; l <= L; ++l) {
      Level& V = h->lv[l];
      V.cx.resize(V.nb);
      V.cy.resize(V.nb);
      V.rad.resize(V.nb);
      V.aspect.resize(V.nb);
      kmaxb[l].resize(V.nb);
      kmeanb[l].resize(V.nb);
      arcb[l].resize(V.nb);
      for (int b = 0; b < V.nb; ++b, ++q) {
        const double* c = &circ[10 * q];
        V.cx[b] = c[0];
        V.cy[b] = c[1];
        V.rad[b] = c[2];
        const double wx = c[4] - c[3], wy = c[6] - c[5];
        V.aspect[b] = std::max(wx, wy) > 0 ? std::min(wx, wy) / std::max(wx, wy) : 1.0;
        kmaxb[l][b] = c[7];
        kmeanb[l][b] = c[8];
        arcb[l][b] = c[9];
      }
    }
  }

  const bool predict = h->opts.rank_predictor != 0;
  const double rscale = h->opts.rank_scale > 0 ? h->opts.rank_scale : 1.0;
  DevBuf dmodel, dfeat, dpred;
  // predictions land in pinned host memory behind an event, so the host can build and launch a
  // level's block and proxy evaluation (which do not depend on them) before it waits
  struct PredHost {
    float* p = nullptr;
    hipEvent_t ev = nullptr;
    ~PredHost() {
      if (ev) (void)hipEventSynchronize(ev);  // a copy into p may still be in flight after an error
      if (p) (void)hipHostFree(p);
      if (ev) (void)hipEventDestroy(ev);
    }
  } ph;
  if (predict) {
    CK(dmodel.reserve(sizeof(float) * MLP_NPARAM));
    CK(hipMemcpyAsync(dmodel.p, h->rank_model.data(), sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, st));
  }
  h->feat.clear();
  h->feat_rank.clear();
  h->feat_level.clear();
  h->feat_pred.clear();
  h->stats.rank_fallbacks = 0;
  h->stats.sketch_bytes_max = 0;
  h->stats.cpqr_work = 0.0;
  h->stats.image_samples = 0;

  DevBuf dnear, wt, zb, zb2, kout, tmpY, tmpZt;
  DevBuf& arena = h->arena;
  // Two chains per level: the compression (W, sketch, column-pivoted QR, P) on the main stream,
  // and the factors (diagonal blocks, their inverses, the products with P, the reduced blocks) on
  // the side stream, which trails.  A level's compression needs only its children's skeletons, so
  // the main stream never waits for the side stream; the side stream waits for the active set
  // of each level (event 0) and for its P (event 1).
  {
    const int rc = side_stream_init(h);
    if (rc != HBS_OK) return rc;
  }
  hipStream_t sf = h->side_stream;
  DevBuf& arena_f = h->arena_s;
  DevBuf& work_f = h->work_s;
  hipEvent_t ev_act = h->side_ev[0], ev_P = h->side_ev[1];
  // singularity flags of every batched inversion of the build (two per box and level, the root),
  // read once after the final synchronisation so that the host never waits on an inversion
  int64_t nflag = 1;
  for (int l = 1; l <= L; ++l) nflag += 2 * (int64_t)h->lv[l].nb;
  DevBuf dflags;
  CK(dflags.reserve(sizeof(int) * nflag));
  CK(hipMemsetAsync(dflags.p, 0, sizeof(int) * nflag, st));
  struct FlagRange { int64_t off; int cnt, level; const char* what; };
  std::vector<FlagRange> franges;
  int64_t foff = 0;
  auto flags_for = [&](int cnt, int level, const char* what) {
    int* p = dflags.as<int>() + foff;
    franges.push_back({foff, cnt, level, what});
    foff += cnt;
    return p;
  };
  // The side-stream part of level lf's factor phase (it needs lf's P: event 1).  Enqueued one level
  // late, after the next level's predictor round trip, so that the large products of the side
  // stream do not share the GPU with the main stream's short critical kernels at that moment.
  auto factor_chain = [&](int lf) -> int {
    Level& V = h->lv[lf];
    const int l = lf, nb = V.nb;
    const bool fp32 = lf > h->fp64_top;
    const bool ident = lf == 1 && h->top_identity;
    cplx* dG = V.G.as<cplx>();
    cplx* dP = V.P.as<cplx>();
    CK(hipStreamWaitEvent(sf, ev_P, 0));
      if (fp32) {
        // complex64 inverse factors from the FP64 blocks D and interpolation matrices P
        CK(V.G32.reserve(sizeof(cplxf) * V.oG[nb]));
        CK(V.E32.reserve(sizeof(cplxf) * V.oP[nb]));
        CK(V.Ft32.reserve(sizeof(cplxf) * V.oP[nb]));
        DevBuf p32, y32, z32, dh32;
        CK(p32.reserve(sizeof(cplxf) * V.oP[nb]));
        CK(y32.reserve(sizeof(cplxf) * V.oP[nb]));
        CK(z32.reserve(sizeof(cplxf) * V.oP[nb]));
        CK(dh32.reserve(sizeof(cplxf) * std::max<int64_t>(1, V.oDh[nb])));
        cplxf* G32 = V.G32.as<cplxf>();
        cplxf* P32 = p32.as<cplxf>();
        cplxf* Y32 = y32.as<cplxf>();
        cplxf* Z32 = z32.as<cplxf>();
        cplxf* Dh32 = dh32.as<cplxf>();
        cplxf* E32 = V.E32.as<cplxf>();
        cplxf* F32 = V.Ft32.as<cplxf>();
        CK(launch_cast_d2f(dG, G32, V.oG[nb], sf));
        CK(launch_cast_d2f(dP, P32, V.oP[nb], sf));
        std::vector<InvDesc32> iv;
        for (int b = 0; b < nb; ++b) iv.push_back({G32 + V.oG[b], V.n[b], V.n[b]});
        CK(inv_batched_flags<float>(arena_f, work_f, iv, sf, flags_for(nb, l, "diagonal block")));
        const cplxf one = mkcf(1, 0), zero = mkcf(0, 0), mone = mkcf(-1, 0);
        auto g32 = [&](const cplxf* A, int lda, int tA, const cplxf* B, int ldb, cplxf* C, int ldc, int m, int n, int k,
                       cplxf al, cplxf be) {
          GemmDesc32 g;
          g.A = A; g.B = B; g.C = C; g.m = m; g.n = n; g.k = k; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
          g.transA = tA; g.pad = 0; g.alpha = al; g.beta = be;
          return g;
        };
        std::vector<GemmDesc32> g1, g2, g3, g4;
        for (int b = 0; b < nb; ++b) {
          const int n = V.n[b], k = V.k[b];
          g1.push_back(g32(G32 + V.oG[b], n, 0, P32 + V.oP[b], n, Y32 + V.oP[b], n, n, k, n, one, zero));
          g1.push_back(g32(P32 + V.oP[b], n, 1, G32 + V.oG[b], n, Z32 + V.oP[b], k, k, n, n, one, zero));
        }
        CK(gemm_batched<float>(arena_f, g1, sf));
        for (int b = 0; b < nb; ++b)
          g2.push_back(g32(Z32 + V.oP[b], V.k[b], 0, P32 + V.oP[b], V.n[b], Dh32 + V.oDh[b], V.k[b], V.k[b], V.k[b], V.n[b],
                           one, zero));
        CK(gemm_batched<float>(arena_f, g2, sf));
        std::vector<InvDesc32> iv2;
        for (int b = 0; b < nb; ++b) iv2.push_back({Dh32 + V.oDh[b], V.k[b], V.k[b]});
        CK(inv_batched_flags<float>(arena_f, work_f, iv2, sf, flags_for(nb, l, "reduced block")));
        for (int b = 0; b < nb; ++b) {
          const int n = V.n[b], k = V.k[b];
          g3.push_back(g32(Y32 + V.oP[b], n, 0, Dh32 + V.oDh[b], k, E32 + V.oP[b], n, n, k, k, one, zero));
          g3.push_back(g32(Dh32 + V.oDh[b], k, 0, Z32 + V.oP[b], k, F32 + V.oP[b], k, k, n, k, one, zero));
        }
        CK(gemm_batched<float>(arena_f, g3, sf));
        for (int b = 0; b < nb; ++b)
          g4.push_back(g32(E32 + V.oP[b], V.n[b], 0, Z32 + V.oP[b], V.k[b], G32 + V.oG[b], V.n[b], V.n[b], V.n[b], V.k[b],
                           mone, one));
        CK(gemm_batched<float>(arena_f, g4, sf));
        // the parent's diagonal block needs D^ in FP64
        CK(launch_cast_f2d(Dh32, V.Dh.as<cplx>(), V.oDh[nb], sf));
        V.G.release();  // D itself is not a factor in this mode
      } else if (ident) {
        // P = I: the reduced block is D itself, E = F^T = I and G = D^{-1} - D^{-1} = 0
        CK(hipMemcpyAsync(V.Dh.p, dG, sizeof(cplx) * V.oG[nb], hipMemcpyDeviceToDevice, sf));
        std::vector<CopyDesc> ce, cz;
        int maxe = 0;
        for (int b = 0; b < nb; ++b) {
          const int n = V.n[b];
          ce.push_back({nullptr, V.E.as<cplx>() + V.oP[b], n, n, n, n});
          ce.push_back({nullptr, V.Ft.as<cplx>() + V.oP[b], n, n, n, n});
          cz.push_back({nullptr, dG + V.oG[b], n, n, n, n});
          maxe = std::max(maxe, n * n);
        }
        CK(up_sync(arena_f, ce, sf));
        CK(launch_eye(arena_f.as<CopyDesc>(), (int)ce.size(), maxe, sf));
        CK(up_sync(arena_f, cz, sf));
        CK(launch_copy(arena_f.as<CopyDesc>(), (int)cz.size(), maxe, sf));
      } else {
      cplx* Y = tmpY.as<cplx>();
      cplx* Zt = tmpZt.as<cplx>();
      cplx* Dh = V.Dh.as<cplx>();
      cplx* E = V.E.as<cplx>();
      cplx* Ft = V.Ft.as<cplx>();
      {
        std::vector<GemmDesc> g1, g2;
        for (int b = 0; b < nb; ++b) {
          const int n = V.n[b], k = V.k[b];
          const cplx* Di = dG + V.oG[b];
          // Y = D^{-1} P  (n x k)
          g1.push_back(gd(Di, n, 0, dP + V.oP[b], n, Y + V.oP[b], n, n, k, n));
          // Zt = P^T D^{-1}  (k x n)
          g1.push_back(gd(dP + V.oP[b], n, 1, Di, n, Zt + V.oP[b], k, k, n, n));
        }
        CK(gemm_batched(arena_f, g1, sf));
        for (int b = 0; b < nb; ++b) {
          const int n = V.n[b], k = V.k[b];
          // S = Zt P (k x k) -> Dh
          g2.push_back(gd(Zt + V.oP[b], k, 0, dP + V.oP[b], n, Dh + V.oDh[b], k, k, k, n));
        }
        CK(gemm_batched(arena_f, g2, sf));
        std::vector<InvDesc> iv;
        for (int b = 0; b < nb; ++b) iv.push_back({Dh + V.oDh[b], V.k[b], V.k[b]});
        CK(inv_batched_flags(arena_f, work_f, iv, sf, flags_for(nb, l, "reduced block")));
        std::vector<GemmDesc> g3, g4;
        for (int b = 0; b < nb; ++b) {
          const int n = V.n[b], k = V.k[b];
          // E = Y Dh (n x k); Ft = Dh Zt (k x n)
          g3.push_back(gd(Y + V.oP[b], n, 0, Dh + V.oDh[b], k, E + V.oP[b], n, n, k, k));
          g3.push_back(gd(Dh + V.oDh[b], k, 0, Zt + V.oP[b], k, Ft + V.oP[b], k, k, n, k));
        }
        CK(gemm_batched(arena_f, g3, sf));
        for (int b = 0; b < nb; ++b) {
          const int n = V.n[b], k = V.k[b];
          // G = D^{-1} - E Zt  (in place)
          g4.push_back(gd(E + V.oP[b], n, 0, Zt + V.oP[b], k, dG + V.oG[b], n, n, n, k, mkc(-1, 0), mkc(1, 0)));
        }
        CK(gemm_batched(arena_f, g4, sf));
      }
      }
    return HBS_OK;
  };
  int pending = 0;  // the level whose factor chain is still to be enqueued
  h->factor_bytes = 0;
  std::memset(h->stats.ranks_per_level_max, 0, sizeof(h->stats.ranks_per_level_max));
  std::memset(h->stats.ranks_per_level_mean, 0, sizeof(h->stats.ranks_per_level_mean));

  DevBuf cpqrws;  // workspace of the one-launch-per-pivot QR of the top levels
  for (int l = L; l >= 1; --l) {
    Level& V = h->lv[l];
    const int nb = V.nb;
    V.n.assign(nb, 0);
    V.aoff.assign(nb + 1, 0);
    if (l == L) {
      for (int b = 0; b < nb; ++b) V.n[b] = (V.hi[b] - V.lo[b]) * h->nc;
      V.hact.resize(h->NU);
      for (int64_t i = 0; i < h->NU; ++i) V.hact[i] = (int)i;
    } else {
      Level& C = h->lv[l + 1];
      for (int b = 0; b < nb; ++b) V.n[b] = C.k[2 * b] + C.k[2 * b + 1];
      V.hact = C.hskel;
    }
    for (int b = 0; b < nb; ++b) V.aoff[b + 1] = V.aoff[b] + V.n[b];
    V.ntot = V.aoff[nb];
    for (int b = 0; b < nb; ++b)
      if (V.n[b] > 2048) {
        set_error("hbs_build: a box's active set exceeds 2048 points (raise tol or the leaf count)");
        return HBS_E_INVALID_ARG;
      }
    CK(V.act.reserve(sizeof(int) * V.ntot));
    CK(hipMemcpyAsync(V.act.p, V.hact.data(), sizeof(int) * V.ntot, hipMemcpyHostToDevice, st));
    const int* dact = V.act.as<int>();
    CK(hipEventRecord(ev_act, st));
    CK(hipStreamWaitEvent(sf, ev_act, 0));

    // ---- compression matrices
    std::vector<int> nnear(nb), np(nb), npf(nb), m(nb), s(nb), nimg(nb, 0), nimgp(nb, 0);
    std::vector<int64_t> noff(nb + 1, 0), woff(nb + 1, 0), zoff(nb + 1, 0), ioff(nb + 1, 0);
    std::vector<int> hnear, himg;
    // candidate boxes from a uniform grid of box centres (cell = the largest near distance), so
    // the near lists cost O(nb) instead of O(nb^2); exact compression takes every box
    double maxrad = 0, gx0 = 1e300, gy0 = 1e300;
    for (int b = 0; b < nb; ++b) {
      maxrad = std::max(maxrad, V.rad[b]);
      gx0 = std::min(gx0, V.cx[b]);
      gy0 = std::min(gy0, V.cy[b]);
    }
    const double cell = std::max((ratio + 1.0) * maxrad, 1e-300);
    // cells of side `cell` holding linked lists of box centres: a dense array of list heads, or a
    // hash of the occupied cells when the obstacle spans very many cells
    double gx1 = -1e300, gy1 = -1e300;
    for (int b = 0; b < nb; ++b) {
      gx1 = std::max(gx1, V.cx[b]);
      gy1 = std::max(gy1, V.cy[b]);
    }
    // a cell grid beyond 1e9 cells per side (degenerate, tiny boxes) takes every box as a candidate
    const double fcx = (gx1 - gx0) / cell, fcy = (gy1 - gy0) / cell;
    const bool allc = exact || !(fcx < 1e9 && fcy < 1e9);
    const int64_t ncx = allc ? 1 : (int64_t)std::floor(fcx) + 1;
    const int64_t ncy = allc ? 1 : (int64_t)std::floor(fcy) + 1;
    const bool dense = !allc && ncx * ncy <= ((int64_t)1 << 23);
    std::vector<int> cell_head(dense ? ncx * ncy : 0, -1), cell_next(nb, -1);
    std::unordered_map<int64_t, int> cell_hash;
    auto head = [&](int64_t c) -> int& { return dense ? cell_head[c] : cell_hash.emplace(c, -1).first->second; };
    auto head_find = [&](int64_t c) -> int {
      if (dense) return cell_head[c];
      auto it = cell_hash.find(c);
      return it == cell_hash.end() ? -1 : it->second;
    };
    auto cell_of = [&](double x, double y, int64_t* ix, int64_t* iy) {
      *ix = std::min<int64_t>(ncx - 1, std::max<int64_t>(0, (int64_t)std::floor((x - gx0) / cell)));
      *iy = std::min<int64_t>(ncy - 1, std::max<int64_t>(0, (int64_t)std::floor((y - gy0) / cell)));
    };
    if (!allc)
      for (int c = nb - 1; c >= 0; --c) {
        int64_t ix, iy;
        cell_of(V.cx[c], V.cy[c], &ix, &iy);
        int& hd = head(ix + ncx * iy);
        cell_next[c] = hd;
        hd = c;
      }
    std::vector<int> cand;
    std::vector<double> mind(nb);
    for (int b = 0; b < nb; ++b) {
      const double Rp = ratio * V.rad[b];
      int cnt = 0;
      double md = std::max(0.0, Rp - V.rad[b]);
      const int64_t total_other = V.ntot - V.n[b];
      cand.clear();
      if (allc) {
        for (int c = 0; c < nb; ++c) cand.push_back(c);
      } else {
        int64_t ix, iy;
        cell_of(V.cx[b], V.cy[b], &ix, &iy);
        for (int64_t jy = std::max<int64_t>(0, iy - 1); jy <= std::min<int64_t>(ncy - 1, iy + 1); ++jy)
          for (int64_t jx = std::max<int64_t>(0, ix - 1); jx <= std::min<int64_t>(ncx - 1, ix + 1); ++jx)
            for (int c = head_find(jx + ncx * jy); c >= 0; c = cell_next[c]) cand.push_back(c);
        cand.push_back((b + 1) % nb);
        cand.push_back((b + nb - 1) % nb);
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      }
      for (int c : cand) {
        if (c == b) continue;
        const int dd = ((c - b) % nb + nb) % nb;
        const bool adj = (dd == 1 || dd == nb - 1);
        const double ex = V.cx[c] - V.cx[b], ey = V.cy[c] - V.cy[b];
        const bool nr = exact || adj || std::sqrt(ex * ex + ey * ey) < Rp + V.rad[c];
        if (nr) {
          hnear.insert(hnear.end(), V.hact.begin() + V.aoff[c], V.hact.begin() + V.aoff[c] + V.n[c]);
          cnt += V.n[c];
          if (!adj) md = std::min(md, std::max(0.0, std::sqrt(ex * ex + ey * ey) - V.rad[c] - V.rad[b]));
        }
      }
      mind[b] = md;
      nnear[b] = cnt;
      const bool full = (cnt == total_other);
      np[b] = full ? 0 : std::max(pmin, (int)std::ceil(1.5 * om_max * Rp) + 50);
      // sources beyond far_radius must be represented too: by the box's own proxies when its
      // circle lies inside far_radius, else by proxies on the far-field circle
      const bool inside = !full && std::hypot(V.cx[b] - h->c0x, V.cy[b] - h->c0y) + Rp < h->opts.far_radius;
      npf[b] = (far_on && !inside) ? npfar : 0;
      // near points of the neighbour images (Sec. 3.2, Fig. 3.1): the active points of every image
      // box that comes inside this box's proxy circle (inside far_radius when the box has no
      // proxies of its own) join the sample in both directions, like the near boxes above; the
      // images at +d first, then at -d
      if (img_on)
        for (int sg = 0; sg < 2; ++sg) {
          const double sx = sg == 0 ? h->opts.image_period : -h->opts.image_period;
          cand.clear();
          if (allc || np[b] == 0) {
            for (int c = 0; c < nb; ++c) cand.push_back(c);
          } else {
            int64_t ix, iy;
            cell_of(V.cx[b] - sx, V.cy[b], &ix, &iy);
            for (int64_t jy = std::max<int64_t>(0, iy - 1); jy <= std::min<int64_t>(ncy - 1, iy + 1); ++jy)
              for (int64_t jx = std::max<int64_t>(0, ix - 1); jx <= std::min<int64_t>(ncx - 1, ix + 1); ++jx)
                for (int c = head_find(jx + ncx * jy); c >= 0; c = cell_next[c]) cand.push_back(c);
          }
          for (int c : cand) {
            const double ix = V.cx[c] + sx, iy = V.cy[c];
            const bool nr = np[b] > 0 ? std::hypot(ix - V.cx[b], iy - V.cy[b]) < Rp + V.rad[c]
                                      : std::hypot(ix - h->c0x, iy - h->c0y) < h->opts.far_radius + V.rad[c];
            if (!nr) continue;
            himg.insert(himg.end(), V.hact.begin() + V.aoff[c], V.hact.begin() + V.aoff[c] + V.n[c]);
            nimg[b] += V.n[c];
            if (sg == 0) nimgp[b] += V.n[c];
          }
        }
      ioff[b + 1] = ioff[b] + nimg[b];
      h->stats.image_samples += nimg[b];
      m[b] = 2 * cnt + 2 * nimg[b] + 3 * h->nc * (np[b] + npf[b]);
      s[b] = (m[b] > 2 * V.n[b] + 8) ? 2 * V.n[b] + 8 : m[b];
      // the transmission operator (no rank model): n + 16 sketch rows; its ranks stay below 0.8 n
      // on every level measured, so the rows exceed the rank by at least 0.2 n + 16
      if (h->nc == 2) s[b] = std::min(s[b], V.n[b] + 16);
      noff[b + 1] = noff[b] + cnt;
      woff[b + 1] = woff[b] + (int64_t)m[b] * V.n[b];
    }
    // features of every box (kept on the handle: training data for the predictor)
    const std::vector<int> sfull = s;
    std::vector<float> F((size_t)nb * MLP_IN);
    for (int b = 0; b < nb; ++b) {
      const double Rp = ratio * V.rad[b];
      const double len = arcb[l][b];
      const double chx = h->hx[V.hi[b] - 1] - h->hx[V.lo[b]], chy = h->hy[V.hi[b] - 1] - h->hy[V.lo[b]];
      int ksum = 0;
      if (l < L) ksum = h->lv[l + 1].k[2 * b] + h->lv[l + 1].k[2 * b + 1];
      float* f = &F[(size_t)b * MLP_IN];
      f[0] = (float)std::log2((double)V.n[b]);
      f[1] = (float)l / (float)L;
      f[2] = (float)(om * len);
      f[3] = (float)(om * V.rad[b]);
      f[4] = (float)(om * Rp);
      f[5] = (float)nnear[b] / (float)V.n[b];
      f[6] = (float)np[b] / 100.f;
      f[7] = (float)std::log10(h->tol);
      f[8] = (float)(kmaxb[l][b] * V.rad[b]);
      f[9] = (float)(kmeanb[l][b] * V.rad[b]);
      f[10] = (float)(om * mind[b]);
      f[11] = (float)(om / 100.0);
      f[12] = (float)(len > 0 ? std::sqrt(chx * chx + chy * chy) / len : 1.0);
      f[13] = (float)V.aspect[b];
      f[14] = (float)(npf[b] > 0 ? om * Rfar : 0.0);
      f[15] = (float)std::log2(1.0 + ksum);
    }
    h->feat.insert(h->feat.end(), F.begin(), F.end());
    std::vector<float> kpred;
    // level 1 decides on the predictions whether it is compressed at all: it waits for them first
    const bool early_pred = predict && l != 1;
    if (predict) {
      CK(dfeat.reserve(sizeof(float) * F.size()));
      CK(dpred.reserve(sizeof(float) * nb));
      CK(hipMemcpyAsync(dfeat.p, F.data(), sizeof(float) * F.size(), hipMemcpyHostToDevice, st));
      CK(mlp_forward(dmodel.as<float>(), dfeat.as<float>(), nb, dpred.as<float>(), st));
      if (!ph.p) {
        CK(hipHostMalloc((void**)&ph.p, sizeof(float) * std::max(1, h->lv[L].nb), hipHostMallocDefault));
        CK(hipEventCreateWithFlags(&ph.ev, hipEventDisableTiming));
      }
      CK(hipMemcpyAsync(ph.p, dpred.p, sizeof(float) * nb, hipMemcpyDeviceToHost, st));
      CK(hipEventRecord(ph.ev, st));
    }
    // predicted rank -> sketch rows 1.25 k^ + 16 (at least 32, at most the full 2n + 8)
    auto take_pred = [&]() -> int {
      CK(hipEventSynchronize(ph.ev));
      kpred.resize(nb);
      for (int b = 0; b < nb; ++b) {
        const double kp = std::exp(std::min(20.0, (double)ph.p[b])) * rscale;
        kpred[b] = (float)kp;
        const int sp = (int)std::max(32.0, std::ceil(1.25 * kp) + 16.0);
        s[b] = std::min(sfull[b], sp);
      }
      return HBS_OK;
    };
    if (predict && !early_pred) {
      const int rc = take_pred();
      if (rc != HBS_OK) return rc;
    }
    // The top level is left uncompressed (P = I, root over the level-2 skeletons) when its
    // interpolative decomposition would keep most points anyway: requested by root_level = 2, or
    // chosen when the predicted ranks reach 0.6 n and the root stays within 1024 points.
    bool ident = false;
    if (l == 1 && L >= 2 && l <= h->fp64_top) {
      if (h->opts.root_level == 2) {
        ident = true;
      } else if (h->opts.root_level == 0 && predict && V.ntot <= 1024) {
        ident = true;
        for (int b = 0; b < nb; ++b) ident = ident && kpred[b] >= 0.6 * V.n[b];
      }
    }
    h->top_identity = ident;
    if (ident)
      for (int b = 0; b < nb; ++b) s[b] = m[b];  // no sketch
    auto size_sketches = [&]() {
      for (int b = 0; b < nb; ++b) zoff[b + 1] = zoff[b] + ((s[b] < m[b]) ? (int64_t)s[b] * V.n[b] : 0);
      h->stats.sketch_bytes_max = std::max<int64_t>(h->stats.sketch_bytes_max, (int64_t)sizeof(cplx) * zoff[nb]);
    };
    if (!early_pred) size_sketches();
    cplx* dwt = nullptr;
    cplx* dz = nullptr;
    if (!ident) {
    CK(dnear.reserve(sizeof(int) * std::max<int64_t>(1, noff[nb] + ioff[nb])));
    if (noff[nb] > 0)
      CK(hipMemcpyAsync(dnear.p, hnear.data(), sizeof(int) * noff[nb], hipMemcpyHostToDevice, st));
    if (ioff[nb] > 0)
      CK(hipMemcpyAsync(dnear.as<int>() + noff[nb], himg.data(), sizeof(int) * ioff[nb], hipMemcpyHostToDevice, st));
    CK(wt.reserve(sizeof(cplx) * std::max<int64_t>(1, woff[nb])));
    dwt = wt.as<cplx>();
    const int* dn = dnear.as<int>();
    {
      std::vector<BlockDesc> bd;
      int maxb = 0;
      for (int b = 0; b < nb; ++b) {
        if (nnear[b] == 0) continue;
        const int n = V.n[b];
        if (h->opts.quad == HBS_QUAD_KR6 && !h->geo.two) {
          // both directions from one Hankel evaluation per pair (no point of b is near itself)
          bd.push_back({dn + noff[b], dact + V.aoff[b], dwt + woff[b], nnear[b], n, m[b], 2, 0.0, nnear[b]});
        } else {
          bd.push_back({dn + noff[b], dact + V.aoff[b], dwt + woff[b], nnear[b], n, m[b], 1});
          bd.push_back({dn + noff[b], dact + V.aoff[b], dwt + woff[b] + nnear[b], nnear[b], n, m[b], 0});
        }
        maxb = std::max(maxb, nnear[b] * n);
      }
      // image rows [2 nnear, 2 nnear + 2 nimg): sources at the images, then targets there; each
      // in the +d part and the -d part
      for (int b = 0; b < nb; ++b) {
        const int n = V.n[b];
        const int* ib = dn + noff[nb] + ioff[b];
        cplx* w0 = dwt + woff[b] + 2 * nnear[b];
        const int part[2] = {nimgp[b], nimg[b] - nimgp[b]};
        const double sxs[2] = {h->opts.image_period, -h->opts.image_period};
        for (int sg = 0, o = 0; sg < 2; o += part[sg], ++sg) {
          if (part[sg] == 0) continue;
          bd.push_back({ib + o, dact + V.aoff[b], w0 + o, part[sg], n, m[b], 2, sxs[sg], nimg[b]});
          maxb = std::max(maxb, part[sg] * n);
        }
      }
      if (!bd.empty()) {
        CK(up_sync(arena, bd, st));
        ProfScope ps("assemble", st, 0.0, 0.0);
        CK(launch_eval_blocks(h->geo, arena.as<BlockDesc>(), (int)bd.size(), maxb, st));
      }
      std::vector<ProxyDesc> pd;
      int maxp = 0;
      for (int b = 0; b < nb; ++b) {
        if (np[b] == 0) continue;
        pd.push_back({dact + V.aoff[b], dwt + woff[b], V.n[b], m[b], 2 * nnear[b] + 2 * nimg[b], np[b], V.cx[b], V.cy[b],
                      ratio * V.rad[b], 2});
        maxp = std::max(maxp, np[b] * V.n[b]);
      }
      for (int b = 0; b < nb; ++b) {
        if (npf[b] == 0) continue;
        // the far-field circle stands for the walls and the neighbour images, whose fields are exterior
        // ones; for the transmission operator it takes both wavenumbers all the same (with the exterior
        // one alone, the skeletons reproduced the wall blocks to 1e-8 at tol 1e-12, with both to 1e-11)
        pd.push_back({dact + V.aoff[b], dwt + woff[b], V.n[b], m[b], 2 * nnear[b] + 2 * nimg[b] + 3 * h->nc * np[b], npf[b],
                      h->c0x, h->c0y, Rfar, 2});
        maxp = std::max(maxp, npf[b] * V.n[b]);
      }
      if (!pd.empty()) {
        CK(up_sync(arena, pd, st));
        ProfScope ps("assemble", st, 0.0, 0.0);
        CK(launch_proxy(h->geo, arena.as<ProxyDesc>(), (int)pd.size(), maxp, st));
      }
      // the sketch sizes need the predictions
      if (early_pred) {
        const int rc = take_pred();
        if (rc != HBS_OK) return rc;
        size_sketches();
      }
      CK(zb.reserve(sizeof(cplx) * std::max<int64_t>(1, zoff[nb])));
      dz = zb.as<cplx>();
      std::vector<SketchDesc> sd;
      int maxs = 0, maxn = 0;
      for (int b = 0; b < nb; ++b) {
        if (s[b] >= m[b]) continue;
        sd.push_back({dwt + woff[b], dz + zoff[b], m[b], V.n[b], s[b], b + (l << 24)});
        maxs = std::max(maxs, s[b]);
        maxn = std::max(maxn, V.n[b]);
      }
      if (!sd.empty()) {
        double fl = 0;
        for (auto& x : sd) fl += 8.0 * x.s * (double)x.m * x.n;
        CK(up_sync(arena, sd, st));
        ProfScope ps("sketch", st, fl, 0.0);
        CK(launch_sketch(arena.as<SketchDesc>(), (int)sd.size(), maxs, maxn, h->opts.seed, st));
      }
    }
    }
    // ---- interpolative decompositions
    std::vector<int> hperm(V.ntot);
    DevBuf dperm;
    CK(dperm.reserve(sizeof(int) * V.ntot));
    CK(kout.reserve(sizeof(int) * nb));
    std::vector<cplx*> zptr(nb, nullptr);
    if (ident) {
      std::vector<int> idp(V.ntot);
      for (int b = 0; b < nb; ++b)
        for (int j = 0; j < V.n[b]; ++j) idp[V.aoff[b] + j] = j;
      std::vector<int> kk(V.n.begin(), V.n.end());
      CK(hipMemcpyAsync(dperm.p, idp.data(), sizeof(int) * V.ntot, hipMemcpyHostToDevice, st));
      CK(hipMemcpyAsync(kout.p, kk.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
      CK(hipStreamSynchronize(st));
    } else {
      std::vector<CpqrDesc> qd;
      double fl = 0;
      for (int b = 0; b < nb; ++b) {
        zptr[b] = (s[b] < m[b]) ? dz + zoff[b] : dwt + woff[b];
        qd.push_back({zptr[b], dperm.as<int>() + V.aoff[b], s[b], V.n[b]});
        fl += 8.0 * 2.0 * s[b] * (double)V.n[b] * V.n[b];
      }
      CK(up_sync(arena, qd, st));
      int ms = 0, mn = 0;
      for (const auto& q : qd) { ms = std::max(ms, q.s); mn = std::max(mn, q.n); }
      ProfScope ps("cpqr", st, fl, 0.0);
      CK(launch_cpqr(arena.as<CpqrDesc>(), nb, ms, mn, h->tol, kout.as<int>(), st, &cpqrws, &ps.launches));
    }
    // the side stream: the children's factor chain (their reduced blocks D^ enter this level's
    // diagonal blocks), then this level's diagonal blocks and their inverses.  Enqueued after the
    // level's compression kernels, so that the host builds these launches while the GPU
    // compresses and the main stream's kernels reach the GPU first.
    if (pending) {
      const int rc = factor_chain(pending);
      if (rc != HBS_OK) return rc;
      pending = 0;
    }
    // ---- diagonal blocks D (into G, inverted in place later) and forward blocks Df
    V.oG.assign(nb + 1, 0);
    for (int b = 0; b < nb; ++b) V.oG[b + 1] = V.oG[b] + (int64_t)V.n[b] * V.n[b];
    CK(V.G.reserve(sizeof(cplx) * V.oG[nb]));
    CK(V.Df.reserve(sizeof(cplx) * V.oG[nb]));
    cplx* dG = V.G.as<cplx>();
    cplx* dDf = V.Df.as<cplx>();
    {
      std::vector<BlockDesc> bd;
      std::vector<CopyDesc> cz, cp, cd;
      int maxe = 0;
      for (int b = 0; b < nb; ++b) {
        const int n = V.n[b];
        maxe = std::max(maxe, n * n);
        if (l == L) {
          bd.push_back({dact + V.aoff[b], dact + V.aoff[b], dG + V.oG[b], n, n, n, 0});
          cp.push_back({dG + V.oG[b], dDf + V.oG[b], n, n, n, n});
        } else {
          Level& C = h->lv[l + 1];
          const int a = 2 * b, c = 2 * b + 1;
          const int ka = C.k[a], kc = C.k[c];
          const int* sa = C.skel.as<int>() + C.soff[a];
          const int* sc = C.skel.as<int>() + C.soff[c];
          cz.push_back({nullptr, dDf + V.oG[b], n, n, n, n});
          bd.push_back({sa, sc, dDf + V.oG[b] + (int64_t)ka * n, ka, kc, n, 0});
          bd.push_back({sc, sa, dDf + V.oG[b] + ka, kc, ka, n, 0});
          cp.push_back({dDf + V.oG[b], dG + V.oG[b], n, n, n, n});
          cd.push_back({C.Dh.as<cplx>() + C.oDh[a], dG + V.oG[b], ka, ka, ka, n});
          cd.push_back({C.Dh.as<cplx>() + C.oDh[c], dG + V.oG[b] + (int64_t)ka * n + ka, kc, kc, kc, n});
        }
      }
      if (!cz.empty()) {
        CK(up_sync(arena_f, cz, sf));
        CK(launch_copy(arena_f.as<CopyDesc>(), (int)cz.size(), maxe, sf));
      }
      {
        int maxb = 0;
        for (auto& d : bd) maxb = std::max(maxb, d.nr * d.nc);
        CK(up_sync(arena_f, bd, sf));
        ProfScope ps("assemble", sf, 0.0, 0.0);
        CK(launch_eval_blocks(h->geo, arena_f.as<BlockDesc>(), (int)bd.size(), maxb, sf));
      }
      CK(up_sync(arena_f, cp, sf));
      CK(launch_copy(arena_f.as<CopyDesc>(), (int)cp.size(), maxe, sf));
      if (!cd.empty()) {
        int maxc = 0;
        for (auto& d : cd) maxc = std::max(maxc, d.nr * d.nc);
        CK(up_sync(arena_f, cd, sf));
        CK(launch_copy(arena_f.as<CopyDesc>(), (int)cd.size(), maxc, sf));
      }
    }

    // complex128 levels: the diagonal blocks D are inverted on the side stream (after their
    // assembly there) while the main stream compresses the level
    if (!ident && l <= h->fp64_top) {
      std::vector<InvDesc> iv;
      for (int b = 0; b < nb; ++b) iv.push_back({dG + V.oG[b], V.n[b], V.n[b]});
      CK(inv_batched_flags(arena_f, work_f, iv, sf, flags_for(nb, l, "diagonal block")));
    }
    V.k.assign(nb, 0);
    CK(hipMemcpyAsync(V.k.data(), kout.p, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(hperm.data(), dperm.p, sizeof(int) * V.ntot, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    bool perm_stale = false;  // a redone box rewrites its part of the permutation
    if (predict && !ident) {
      // a sketch that was too short for the box's rank reveals no gap: redo it at full size
      std::vector<int> redo;
      for (int b = 0; b < nb; ++b)
        if (s[b] < sfull[b] && V.k[b] >= s[b] - 8) redo.push_back(b);
      if (!redo.empty()) {
        h->stats.rank_fallbacks += (int)redo.size();
        std::vector<int64_t> z2off(redo.size() + 1, 0);
        for (size_t r = 0; r < redo.size(); ++r) {
          const int b = redo[r];
          s[b] = sfull[b];
          z2off[r + 1] = z2off[r] + ((s[b] < m[b]) ? (int64_t)s[b] * V.n[b] : 0);
        }
        CK(zb2.reserve(sizeof(cplx) * std::max<int64_t>(1, z2off.back())));
        std::vector<SketchDesc> sd;
        int maxs = 0, maxn = 0;
        for (size_t r = 0; r < redo.size(); ++r) {
          const int b = redo[r];
          if (s[b] >= m[b]) continue;
          sd.push_back({dwt + woff[b], zb2.as<cplx>() + z2off[r], m[b], V.n[b], s[b], b + (l << 24)});
          maxs = std::max(maxs, s[b]);
          maxn = std::max(maxn, V.n[b]);
        }
        if (!sd.empty()) {
          CK(up_sync(arena, sd, st));
          CK(launch_sketch(arena.as<SketchDesc>(), (int)sd.size(), maxs, maxn, h->opts.seed, st));
        }
        std::vector<CpqrDesc> qd;
        for (size_t r = 0; r < redo.size(); ++r) {
          const int b = redo[r];
          zptr[b] = (s[b] < m[b]) ? zb2.as<cplx>() + z2off[r] : dwt + woff[b];
          qd.push_back({zptr[b], dperm.as<int>() + V.aoff[b], s[b], V.n[b]});
        }
        CK(up_sync(arena, qd, st));
        CK(kout.reserve(sizeof(int) * nb + sizeof(int) * redo.size()));
        int* k2 = kout.as<int>() + nb;
        int ms = 0, mn = 0;
        for (const auto& q : qd) { ms = std::max(ms, q.s); mn = std::max(mn, q.n); }
        double fl2 = 0;
        for (const auto& q : qd) fl2 += 8.0 * 2.0 * q.s * (double)q.n * q.n;
        ProfScope ps2("cpqr", st, fl2, 0.0);
        CK(launch_cpqr(arena.as<CpqrDesc>(), (int)qd.size(), ms, mn, h->tol, k2, st, &cpqrws, &ps2.launches));
        std::vector<int> hk2(redo.size());
        CK(hipMemcpyAsync(hk2.data(), k2, sizeof(int) * redo.size(), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        for (size_t r = 0; r < redo.size(); ++r) V.k[redo[r]] = hk2[r];
        perm_stale = true;
      }
    }
    if (perm_stale) {
      CK(hipMemcpyAsync(hperm.data(), dperm.p, sizeof(int) * V.ntot, hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
    }
    for (int b = 0; b < nb; ++b) {
      h->feat_rank.push_back(V.k[b]);
      h->feat_level.push_back(l);
      h->feat_pred.push_back(predict ? kpred[b] : 0.f);
      if (!ident) h->stats.cpqr_work += (double)s[b] * V.n[b] * V.k[b];
    }
    V.soff.assign(nb + 1, 0);
    for (int b = 0; b < nb; ++b) V.soff[b + 1] = V.soff[b] + V.k[b];
    V.ktot = V.soff[nb];
    V.hskel.resize(V.ktot);
    int kmax = 0;
    double ksum = 0;
    for (int b = 0; b < nb; ++b) {
      for (int j = 0; j < V.k[b]; ++j) V.hskel[V.soff[b] + j] = V.hact[V.aoff[b] + hperm[V.aoff[b] + j]];
      kmax = std::max(kmax, V.k[b]);
      ksum += V.k[b];
    }
    if (l < 32) {
      h->stats.ranks_per_level_max[l] = kmax;
      h->stats.ranks_per_level_mean[l] = ksum / nb;
    }
    CK(V.skel.reserve(sizeof(int) * std::max<int64_t>(1, V.ktot)));
    CK(hipMemcpyAsync(V.skel.p, V.hskel.data(), sizeof(int) * V.ktot, hipMemcpyHostToDevice, st));

    // ---- factors
    V.oP.assign(nb + 1, 0);
    V.oDh.assign(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
      V.oP[b + 1] = V.oP[b] + (int64_t)V.n[b] * V.k[b];
      V.oDh[b + 1] = V.oDh[b] + (int64_t)V.k[b] * V.k[b];
    }
    V.oE = V.oP;
    V.oFt = V.oP;
    const bool fp32 = l > h->fp64_top;  // this level's inverse factors in complex64
    CK(V.P.reserve(sizeof(cplx) * V.oP[nb]));
    if (!fp32) {
      CK(V.E.reserve(sizeof(cplx) * V.oP[nb]));
      CK(V.Ft.reserve(sizeof(cplx) * V.oP[nb]));
      CK(tmpY.reserve(sizeof(cplx) * V.oP[nb]));
      CK(tmpZt.reserve(sizeof(cplx) * V.oP[nb]));
    }
    CK(V.Dh.reserve(sizeof(cplx) * std::max<int64_t>(1, V.oDh[nb])));
    cplx* dP = V.P.as<cplx>();
    {
      std::vector<PDesc> pd;
      int maxe = 0;
      for (int b = 0; b < nb; ++b) {
        pd.push_back({zptr[b], dperm.as<int>() + V.aoff[b], dP + V.oP[b], V.n[b], V.k[b], s[b]});
        maxe = std::max(maxe, V.n[b] * V.k[b]);
      }
      CK(up_sync(arena, pd, st));
      CK(launch_buildP(arena.as<PDesc>(), nb, maxe, st));
    }
    CK(hipEventRecord(ev_P, st));
    pending = l;  // its factor chain is enqueued after the next level's predictor
    if (l < L) h->lv[l + 1].Dh.release();
    h->factor_bytes += fp32 ? (int64_t)sizeof(cplx) * (V.oP[nb] + V.oG[nb]) + (int64_t)sizeof(cplxf) * (2 * V.oP[nb] + V.oG[nb])
                            : (int64_t)sizeof(cplx) * (3 * V.oP[nb] + 2 * V.oG[nb]);
  }

  if (pending) {
    const int rc = factor_chain(pending);
    if (rc != HBS_OK) return rc;
    pending = 0;
  }
  // ---- root (side stream: it needs level 1's reduced blocks; the skeletons came from the main stream)
  CK(hipEventRecord(ev_act, st));
  CK(hipStreamWaitEvent(sf, ev_act, 0));
  {
    Level& V = h->lv[1];
    const int ka = V.k[0], kc = V.k[1];
    const int n = ka + kc;
    h->nroot = n;
    CK(h->Rfwd.reserve(sizeof(cplx) * n * n));
    CK(h->Rinv.reserve(sizeof(cplx) * n * n));
    cplx* Rf = h->Rfwd.as<cplx>();
    cplx* Ri = h->Rinv.as<cplx>();
    const int* sa = V.skel.as<int>();
    const int* sc = V.skel.as<int>() + V.soff[1];
    std::vector<CopyDesc> cz = {{nullptr, Rf, n, n, n, n}};
    CK(up_sync(arena_f, cz, sf));
    CK(launch_copy(arena_f.as<CopyDesc>(), 1, n * n, sf));
    std::vector<BlockDesc> bd = {{sa, sc, Rf + (int64_t)ka * n, ka, kc, n, 0}, {sc, sa, Rf + ka, kc, ka, n, 0}};
    CK(up_sync(arena_f, bd, sf));
    CK(launch_eval_blocks(h->geo, arena_f.as<BlockDesc>(), 2, std::max(ka * kc, 1), sf));
    std::vector<CopyDesc> cp = {{Rf, Ri, n, n, n, n}};
    CK(up_sync(arena_f, cp, sf));
    CK(launch_copy(arena_f.as<CopyDesc>(), 1, n * n, sf));
    std::vector<CopyDesc> cd = {{V.Dh.as<cplx>() + V.oDh[0], Ri, ka, ka, ka, n},
                                {V.Dh.as<cplx>() + V.oDh[1], Ri + (int64_t)ka * n + ka, kc, kc, kc, n}};
    CK(up_sync(arena_f, cd, sf));
    CK(launch_copy(arena_f.as<CopyDesc>(), 2, std::max(ka * ka, kc * kc), sf));
    if (h->opts.defer_root) {
      h->root_state = 1;  // Ri holds the root matrix until a call needs its inverse
    } else {
      std::vector<InvDesc> iv = {{Ri, n, n}};
      CK(inv_batched_flags(arena_f, work_f, iv, sf, flags_for(1, 0, "root matrix")));
      h->root_state = 0;
    }
    V.Dh.release();
    h->factor_bytes += (int64_t)sizeof(cplx) * 2 * n * n;
  }
  std::vector<int> hflags(foff);
  if (foff > 0) CK(hipMemcpyAsync(hflags.data(), dflags.p, sizeof(int) * foff, hipMemcpyDeviceToHost, sf));
  CK(hipStreamSynchronize(sf));
  CK(hipStreamSynchronize(st));
  for (const auto& fr : franges)
    for (int b = 0; b < fr.cnt; ++b)
      if (hflags[fr.off + b] != 0) {
        set_error(std::string("hbs_build: singular ") + fr.what +
                  (fr.level > 0 ? " at level " + std::to_string(fr.level) + ", box " + std::to_string(b) : ""));
        return HBS_E_SINGULAR;
      }
  h->work.release();
  auto t1 = std::chrono::steady_clock::now();
  h->build_seconds = std::chrono::duration<double>(t1 - t0).count();
  return HBS_OK;
}

#undef CK
#define CK(expr)                                                                                  \
  do {                                                                                            \
    hipError_t _e = (expr);                                                                       \
    if (_e != hipSuccess) {                                                                       \
      set_error(std::string("hbs apply: ") + #expr + ": " + hipGetErrorString(_e));               \
      return _e == hipErrorOutOfMemory ? HBS_E_OOM : HBS_E_DEVICE;                                \
    }                                                                                             \
  } while (0)

// X (N x r) = U Z with U the nested interpolation P^(L) ... P^(1) from the root's active set
// (the level-1 skeletons) to all nodes: the downward pass of the factorization without its
// diagonal terms.
int apply_interp(hbs_handle* h, const cplx* Z, int64_t ldz, cplx* X, int64_t ldx, int64_t r) {
  if (r <= 0) return HBS_OK;
  hipStream_t st = h->stream;
  const int L = h->L;
  auto& lv = h->lv;
  int64_t xmax = 1;
  for (int l = 1; l < L; ++l) xmax = std::max<int64_t>(xmax, lv[l].ntot);
  CK(h->ab_x0.reserve(sizeof(cplx) * xmax * r));
  CK(h->ab_x1.reserve(sizeof(cplx) * xmax * r));
  auto xbuf = [&](int l) { return (l & 1) ? h->ab_x1.as<cplx>() : h->ab_x0.as<cplx>(); };
  std::vector<GemmDesc> all;
  std::vector<LaunchRec> recs;
  for (int l = 1; l <= L; ++l) {
    Level& V = lv[l];
    const cplx* xin = (l == 1) ? Z : xbuf(l - 1);
    const int ldxin = (l == 1) ? (int)ldz : (int)V.ktot;
    cplx* out = (l == L) ? X : xbuf(l);
    const int64_t ldo = (l == L) ? ldx : V.ntot;
    LaunchRec rec{all.size(), 0, GemmPlan{0, 0, 0}, 0.0};
    for (int b = 0; b < V.nb; ++b) {
      all.push_back(gd(V.P.as<cplx>() + V.oP[b], V.n[b], 0, xin + V.soff[b], ldxin, out + V.aoff[b], (int)ldo, V.n[b],
                       (int)r, V.k[b]));
      rec.flops += 8.0 * V.n[b] * (double)r * V.k[b];
    }
    rec.cnt = (int)(all.size() - rec.off);
    rec.plan = gemm_plan(all.data() + rec.off, rec.cnt);
    recs.push_back(rec);
  }
  CK(upload(h->arena, all, st));
  for (auto& rc : recs) {
    ProfScope ps("zgemm", st, rc.flops, 0.0);
    CK(launch_zgemm(h->arena.as<GemmDesc>() + rc.off, rc.cnt, rc.plan, st));
  }
  // stream-ordered: the caller's later work on the handle's stream sees the result
  return HBS_OK;
}

// X (N x r) = E_L ... E_1 Z: the downward pass of the inverse with E only.  Since F^T P = I and
// G P = 0 for every box (Dh = (P^T D^{-1} P)^{-1}), A^{-1} U = E_L ... E_1 R^{-1} and U^T A^{-1} U
// = R^{-1}: this gives V = A^{-1} U from Z = R^{-1} without forming U.  complex128 levels only.
int apply_down_E(hbs_handle* h, const cplx* Z, int64_t ldz, cplx* X, int64_t ldx, int64_t r) {
  if (r <= 0) return HBS_OK;
  if (h->fp64_top < h->L) {
    set_error("hbs apply: E-only downward pass needs complex128 factors on every level");
    return HBS_E_INVALID_ARG;
  }
  hipStream_t st = h->stream;
  const int L = h->L;
  auto& lv = h->lv;
  int64_t xmax = 1;
  for (int l = 1; l < L; ++l) xmax = std::max<int64_t>(xmax, lv[l].ntot);
  CK(h->ab_x0.reserve(sizeof(cplx) * xmax * r));
  CK(h->ab_x1.reserve(sizeof(cplx) * xmax * r));
  auto xbuf = [&](int l) { return (l & 1) ? h->ab_x1.as<cplx>() : h->ab_x0.as<cplx>(); };
  std::vector<GemmDesc> all;
  std::vector<LaunchRec> recs;
  for (int l = 1; l <= L; ++l) {
    Level& V = lv[l];
    const cplx* xin = (l == 1) ? Z : xbuf(l - 1);
    const int ldxin = (l == 1) ? (int)ldz : (int)V.ktot;
    cplx* out = (l == L) ? X : xbuf(l);
    const int64_t ldo = (l == L) ? ldx : V.ntot;
    LaunchRec rec{all.size(), 0, GemmPlan{0, 0, 0}, 0.0};
    for (int b = 0; b < V.nb; ++b) {
      all.push_back(gd(V.E.as<cplx>() + V.oE[b], V.n[b], 0, xin + V.soff[b], ldxin, out + V.aoff[b], (int)ldo, V.n[b],
                       (int)r, V.k[b]));
      rec.flops += 8.0 * V.n[b] * (double)r * V.k[b];
    }
    rec.cnt = (int)(all.size() - rec.off);
    rec.plan = gemm_plan(all.data() + rec.off, rec.cnt);
    recs.push_back(rec);
  }
  CK(upload(h->arena, all, st));
  for (auto& rc : recs) {
    ProfScope ps("zgemm", st, rc.flops, 0.0);
    CK(launch_zgemm(h->arena.as<GemmDesc>() + rc.off, rc.cnt, rc.plan, st));
  }
  // stream-ordered: the caller's later work on the handle's stream sees the result
  return HBS_OK;
}

// Z (nr x r) = U^T X: the transpose of the nested interpolation, i.e. the upward pass with P^T
// from the leaves to the root's active set (outgoing fields of X seen from beyond every proxy circle).
int apply_interp_t(hbs_handle* h, const cplx* X, int64_t ldx, cplx* Z, int64_t ldz, int64_t r) {
  if (r <= 0) return HBS_OK;
  hipStream_t st = h->stream;
  const int L = h->L;
  auto& lv = h->lv;
  int64_t xmax = 1;
  for (int l = 2; l <= L; ++l) xmax = std::max<int64_t>(xmax, lv[l].ktot);
  CK(h->ab_x0.reserve(sizeof(cplx) * xmax * r));
  CK(h->ab_x1.reserve(sizeof(cplx) * xmax * r));
  auto xbuf = [&](int l) { return (l & 1) ? h->ab_x1.as<cplx>() : h->ab_x0.as<cplx>(); };
  std::vector<GemmDesc> all;
  std::vector<LaunchRec> recs;
  for (int l = L; l >= 1; --l) {
    Level& V = lv[l];
    const cplx* src = (l == L) ? X : xbuf(l);
    const int lds = (l == L) ? (int)ldx : (int)V.ntot;
    cplx* dst = (l == 1) ? Z : xbuf(l - 1);
    const int ldd = (l == 1) ? (int)ldz : (int)V.ktot;
    LaunchRec rec{all.size(), 0, GemmPlan{0, 0, 0}, 0.0};
    for (int b = 0; b < V.nb; ++b) {
      all.push_back(gd(V.P.as<cplx>() + V.oP[b], V.n[b], 1, src + V.aoff[b], lds, dst + V.soff[b], ldd, V.k[b], (int)r,
                       V.n[b]));
      rec.flops += 8.0 * V.n[b] * (double)r * V.k[b];
    }
    rec.cnt = (int)(all.size() - rec.off);
    rec.plan = gemm_plan(all.data() + rec.off, rec.cnt);
    recs.push_back(rec);
  }
  CK(upload(h->arena, all, st));
  for (auto& rc : recs) {
    ProfScope ps("zgemm", st, rc.flops, 0.0);
    CK(launch_zgemm(h->arena.as<GemmDesc>() + rc.off, rc.cnt, rc.plan, st));
  }
  // stream-ordered: the caller's later work on the handle's stream sees the result
  return HBS_OK;
}

template <class R>
static GemmDescT<R> gdt(const typename cx<R>::T* A, int lda, int transA, const typename cx<R>::T* B, int ldb,
                        typename cx<R>::T* C, int ldc, int m, int n, int k, double beta) {
  GemmDescT<R> g;
  g.A = A; g.B = B; g.C = C;
  g.m = m; g.n = n; g.k = k;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc;
  g.transA = transA; g.pad = 0;
  g.alpha = cx<R>::make(1, 0);
  g.beta = cx<R>::make(beta, 0);
  return g;
}

// The telescoping factorization applied level by level: upward b^ = Up b (F^T or P^T), the root
// (inverse or coupling), downward x = Dn x^ + Dg b (E, G or P, D_fwd).  The levels > split run in
// complex64 on the complex64 factors (inverse only), levels 1..split and the root in complex128;
// the vectors crossing the split are cast.  split = L: everything in complex128.
namespace {
struct Step {
  int kind;  // 0: FP64 GEMM batch, 1: FP32 GEMM batch, 2: cast to complex64, 3: cast to complex128
  size_t off;
  int cnt;
  GemmPlan plan;
  double flops;
  const void* src;
  void* dst;
  int64_t n;
};
}  // namespace

// phase 0: the whole apply; 1: the upward pass and the root product only; 2: the downward pass
// only, from root_set (nroot x r) when given, else from the root workspace as phase 1 left it (the
// upward results of the same B stay in the handle's workspace between the two calls)
static int apply_mixed(hbs_handle* h, bool inv, int split, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r,
                       bool sync = true, const cplx* root_add = nullptr, cplx* root_up = nullptr, int phase = 0,
                       const cplx* root_set = nullptr, hipEvent_t root_wait = nullptr) {
  if (r <= 0) return HBS_OK;
  // the downward pass alone does not read the root inverse; with root_wait the caller forms it
  if (inv && phase != 2 && !root_wait) {
    const int rc = ensure_root(h);
    if (rc != HBS_OK) return rc;
  }
  if (root_wait && h->opts.graph) {
    set_error("hbs apply: a root wait cannot be captured");
    return HBS_E_INVALID_ARG;
  }
  hipStream_t st = h->stream;
  const int L = h->L;
  auto& lv = h->lv;
  if (!inv) split = L;
  split = std::max(0, std::min(L, split));
  const bool mixed = split < L;  // level L (and maybe more) in complex64
  const int64_t N = h->NU;
  const int rr = (int)r;
  // up[j] (j = 0..L-1) = output of the upward step of level j+1, lv[j+1].ktot rows
  std::vector<int64_t> rows_up(L);
  for (int j = 0; j < L; ++j) rows_up[j] = lv[j + 1].ktot;
  // complex128 up buffers hold j = 0..min(split, L-1); complex64 ones j = split..L-1
  std::vector<int64_t> o64(L + 1, 0), o32(L + 1, 0);
  for (int j = 0; j < L; ++j) {
    o64[j + 1] = o64[j] + (j <= split ? rows_up[j] * r : 0);
    o32[j + 1] = o32[j] + (j >= split ? rows_up[j] * r : 0);
  }
  int64_t x64max = 1, x32max = 1;
  for (int l = 1; l < L; ++l) {
    if (l <= split) x64max = std::max<int64_t>(x64max, lv[l].ntot);
    else x32max = std::max<int64_t>(x32max, lv[l].ntot);
  }
  if (mixed) x32max = std::max<int64_t>(x32max, lv[split + 1].ktot);
  CK(h->ab_up.reserve(sizeof(cplx) * std::max<int64_t>(1, o64[L])));
  CK(h->ab_x0.reserve(sizeof(cplx) * x64max * r));
  CK(h->ab_x1.reserve(sizeof(cplx) * x64max * r));
  CK(h->ab_root.reserve(sizeof(cplx) * h->nroot * r));
  if (mixed) {
    CK(h->ab_in32.reserve(sizeof(cplxf) * N * r * 2));  // input and output of the complex64 leaf level
    CK(h->ab_up32.reserve(sizeof(cplxf) * std::max<int64_t>(1, o32[L])));
    CK(h->ab_x32a.reserve(sizeof(cplxf) * x32max * r));
    CK(h->ab_x32b.reserve(sizeof(cplxf) * x32max * r));
  }
  cplx* up64 = h->ab_up.as<cplx>();
  cplxf* up32 = mixed ? h->ab_up32.as<cplxf>() : nullptr;
  cplx* xr = h->ab_root.as<cplx>();
  cplxf* in32 = mixed ? h->ab_in32.as<cplxf>() : nullptr;
  cplxf* out32 = mixed ? in32 + N * r : nullptr;
  auto u64 = [&](int j) { return up64 + o64[j]; };
  auto u32 = [&](int j) { return up32 + o32[j]; };
  auto x64 = [&](int l) { return (l & 1) ? h->ab_x1.as<cplx>() : h->ab_x0.as<cplx>(); };
  auto x32 = [&](int l) { return (l & 1) ? h->ab_x32b.as<cplxf>() : h->ab_x32a.as<cplxf>(); };

  std::vector<GemmDesc> d64;
  std::vector<GemmDesc32> d32;
  std::vector<Step> prog;
  auto close64 = [&](size_t s0) {
    Step t{0, s0, (int)(d64.size() - s0), gemm_plan(d64.data() + s0, d64.size() - s0), 0.0, nullptr, nullptr, 0};
    for (size_t i = s0; i < d64.size(); ++i) t.flops += 8.0 * d64[i].m * (double)d64[i].n * d64[i].k;
    if (t.cnt > 0) prog.push_back(t);
  };
  auto close32 = [&](size_t s0) {
    Step t{1, s0, (int)(d32.size() - s0), gemm_plan(d32.data() + s0, d32.size() - s0), 0.0, nullptr, nullptr, 0};
    for (size_t i = s0; i < d32.size(); ++i) t.flops += 8.0 * d32[i].m * (double)d32[i].n * d32[i].k;
    if (t.cnt > 0) prog.push_back(t);
  };
  auto cast = [&](int kind, const void* src, void* dst, int64_t n) {
    prog.push_back({kind, 0, 0, GemmPlan{0, 0, 0}, 0.0, src, dst, n});
  };

  // ---- upward
  if (mixed) {
    if (ldb == N) {
      cast(2, B, in32, N * r);
    } else {
      for (int64_t c = 0; c < r; ++c) cast(2, B + c * ldb, in32 + c * N, N);
    }
  }
  for (int l = L; l >= 1; --l) {
    Level& V = lv[l];
    if (l > split) {
      const cplxf* src = (l == L) ? in32 : u32(l);
      const int64_t lds = (l == L) ? N : V.ntot;
      size_t s0 = d32.size();
      for (int b = 0; b < V.nb; ++b)
        d32.push_back(gdt<float>(V.Ft32.as<cplxf>() + V.oFt[b], V.k[b], 0, src + V.aoff[b], (int)lds, u32(l - 1) + V.soff[b],
                                 (int)V.ktot, V.k[b], rr, V.n[b], 0.0));
      close32(s0);
      if (l - 1 == split) cast(3, u32(split), u64(split), rows_up[split] * r);
    } else {
      const cplx* src = (l == L) ? B : u64(l);
      const int64_t lds = (l == L) ? ldb : V.ntot;
      size_t s0 = d64.size();
      for (int b = 0; b < V.nb; ++b) {
        const int n = V.n[b], k = V.k[b];
        if (inv)
          d64.push_back(gdt<double>(V.Ft.as<cplx>() + V.oFt[b], k, 0, src + V.aoff[b], (int)lds, u64(l - 1) + V.soff[b],
                                    (int)V.ktot, k, rr, n, 0.0));
        else
          d64.push_back(gdt<double>(V.P.as<cplx>() + V.oP[b], n, 1, src + V.aoff[b], (int)lds, u64(l - 1) + V.soff[b],
                                    (int)V.ktot, k, rr, n, 0.0));
      }
      close64(s0);
    }
  }
  {
    size_t s0 = d64.size();
    const cplx* Rt = inv ? h->Rinv.as<cplx>() : h->Rfwd.as<cplx>();
    d64.push_back(gdt<double>(Rt, h->nroot, 0, u64(0), h->nroot, xr, h->nroot, h->nroot, rr, h->nroot, root_add ? 1.0 : 0.0));
    close64(s0);
  }
  const size_t down_begin = prog.size();
  // ---- downward
  for (int l = 1; l <= L; ++l) {
    Level& V = lv[l];
    if (l <= split) {
      const cplx* xin = (l == 1) ? xr : x64(l - 1);
      cplx* out = (l == L) ? X : x64(l);
      const int64_t ldo = (l == L) ? ldx : V.ntot;
      const cplx* src = (l == L) ? B : u64(l);
      const int64_t lds = (l == L) ? ldb : V.ntot;
      size_t s0 = d64.size();
      for (int b = 0; b < V.nb; ++b) {
        const int n = V.n[b], k = V.k[b];
        const cplx* Dn = inv ? V.E.as<cplx>() + V.oE[b] : V.P.as<cplx>() + V.oP[b];
        d64.push_back(gdt<double>(Dn, n, 0, xin + V.soff[b], (int)V.ktot, out + V.aoff[b], (int)ldo, n, rr, k, 0.0));
      }
      close64(s0);
      s0 = d64.size();
      for (int b = 0; b < V.nb; ++b) {
        const int n = V.n[b];
        const cplx* Dg = inv ? V.G.as<cplx>() + V.oG[b] : V.Df.as<cplx>() + V.oG[b];
        d64.push_back(gdt<double>(Dg, n, 0, src + V.aoff[b], (int)lds, out + V.aoff[b], (int)ldo, n, rr, n, 1.0));
      }
      close64(s0);
    } else {
      // the complex64 input of level split+1 shares the buffer that level split+2 writes
      if (l == split + 1) cast(2, (l == 1) ? xr : x64(l - 1), x32(l - 1), V.ktot * r);
      const cplxf* xin = x32(l - 1);
      cplxf* out = (l == L) ? out32 : x32(l);
      const int64_t ldo = (l == L) ? N : V.ntot;
      const cplxf* src = (l == L) ? in32 : u32(l);
      const int64_t lds = (l == L) ? N : V.ntot;
      size_t s0 = d32.size();
      for (int b = 0; b < V.nb; ++b)
        d32.push_back(gdt<float>(V.E32.as<cplxf>() + V.oE[b], V.n[b], 0, xin + V.soff[b], (int)V.ktot, out + V.aoff[b],
                                 (int)ldo, V.n[b], rr, V.k[b], 0.0));
      close32(s0);
      s0 = d32.size();
      for (int b = 0; b < V.nb; ++b)
        d32.push_back(gdt<float>(V.G32.as<cplxf>() + V.oG[b], V.n[b], 0, src + V.aoff[b], (int)lds, out + V.aoff[b], (int)ldo,
                                 V.n[b], rr, V.n[b], 1.0));
      close32(s0);
    }
  }
  if (mixed) {
    if (ldx == N) {
      cast(3, out32, X, N * r);
    } else {
      for (int64_t c = 0; c < r; ++c) cast(3, out32 + c * N, X + c * ldx, N);
    }
  }
  double fl = 0;
  for (auto& t : prog) fl += t.flops;
  // issue the program on stream s (profiled per launch unless it is being captured)
  if (phase != 0 && mixed) {
    set_error("hbs apply: a split apply needs complex128 factors on every level");
    return HBS_E_INVALID_ARG;
  }
  const size_t p0 = phase == 2 ? down_begin : 0, p1 = phase == 1 ? down_begin : prog.size();
  auto issue = [&](const GemmDesc* dd64, const GemmDesc32* dd32, hipStream_t s, bool prof) -> hipError_t {
    for (size_t ti = p0; ti < p1; ++ti) {
      const Step& t = prog[ti];
      hipError_t e;
      if (root_wait && ti + 1 == down_begin) {
        // the root product (the last step before the downward pass) reads the root inverse
        e = hipStreamWaitEvent(s, root_wait, 0);
        if (e != hipSuccess) return e;
      }
      if (t.kind == 0) {
        ProfScope ps2(prof ? "zgemm" : nullptr, s, t.flops, 0.0);
        e = launch_gemm<double>(dd64 + t.off, t.cnt, t.plan, s);
      } else if (t.kind == 1) {
        ProfScope ps2(prof ? "cgemm" : nullptr, s, t.flops, 0.0);
        e = launch_gemm<float>(dd32 + t.off, t.cnt, t.plan, s);
      } else if (t.kind == 2) {
        e = launch_cast_d2f(static_cast<const cplx*>(t.src), static_cast<cplxf*>(t.dst), t.n, s);
      } else {
        e = launch_cast_f2d(static_cast<const cplxf*>(t.src), static_cast<cplx*>(t.dst), t.n, s);
      }
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  const int64_t nroot = h->nroot;
  if (root_add) CK(hipMemcpyAsync(xr, root_add, sizeof(cplx) * nroot * r, hipMemcpyDeviceToDevice, st));
  if (phase == 2 && root_set) CK(hipMemcpyAsync(xr, root_set, sizeof(cplx) * nroot * r, hipMemcpyDeviceToDevice, st));
  auto copy_root_up = [&]() -> hipError_t {
    // the upward result at the root (u64(0), nroot x r) is not touched by the downward pass
    if (!root_up) return hipSuccess;
    return hipMemcpyAsync(root_up, u64(0), sizeof(cplx) * nroot * r, hipMemcpyDeviceToDevice, st);
  };
  if (h->opts.graph) {
    // capture once per operand set on a private stream (kernels only: the descriptors live in the
    // graph's own buffers, uploaded before the capture), then replay on the handle's stream
    const void* ws[8] = {h->ab_up.p, h->ab_x0.p, h->ab_x1.p, h->ab_root.p, h->ab_in32.p, h->ab_up32.p, h->ab_x32a.p,
                         h->ab_x32b.p};
    ApplyGraph* g = nullptr;
    for (auto& c : h->graphs)
      if (c->inv == inv && c->root_acc == (root_add != nullptr) && c->phase == phase && c->split == split && c->B == B &&
          c->ldb == ldb &&
          c->X == X && c->ldx == ldx && c->r == r && std::equal(ws, ws + 8, c->ws))
        g = c.get();
    if (!g) {
      if (!h->cap_stream) CK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
      if (h->graphs.size() >= 4) h->graphs.erase(h->graphs.begin());
      h->graphs.emplace_back(new ApplyGraph);
      g = h->graphs.back().get();
      g->inv = inv; g->root_acc = root_add != nullptr; g->phase = phase; g->split = split; g->B = B; g->ldb = ldb; g->X = X;
      g->ldx = ldx;
      g->r = r;
      std::copy(ws, ws + 8, g->ws);
      CK(upload(g->d64, d64, st));
      if (!d32.empty()) CK(upload(g->d32, d32, st));
      CK(hipStreamSynchronize(st));
      hipGraph_t graph = nullptr;
      CK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
      const hipError_t ie = issue(g->d64.as<GemmDesc>(), d32.empty() ? nullptr : g->d32.as<GemmDesc32>(), h->cap_stream, false);
      const hipError_t ce = hipStreamEndCapture(h->cap_stream, &graph);
      if (ie != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        h->graphs.pop_back();
        CK(ie != hipSuccess ? ie : ce);
      }
      const hipError_t xe = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (xe != hipSuccess) {
        h->graphs.pop_back();
        CK(xe);
      }
      ++h->graph_captures;
    } else {
      ++h->graph_replays;
    }
    {
      ProfScope ps("apply", st, fl, 0.0);
      CK(hipGraphLaunch(g->exec, st));
    }
    CK(copy_root_up());
    if (sync) CK(hipStreamSynchronize(st));
    return HBS_OK;
  }
  CK(upload(h->arena, d64, st));
  if (!d32.empty()) CK(upload(h->arena32, d32, st));
  {
    ProfScope ps("apply", st, fl, 0.0);
    CK(issue(h->arena.as<GemmDesc>(), d32.empty() ? nullptr : h->arena32.as<GemmDesc32>(), st, true));
  }
  CK(copy_root_up());
  if (sync) CK(hipStreamSynchronize(st));
  return HBS_OK;
}

int apply_forward_root(hbs_handle* h, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r, const cplx* root_add,
                       cplx* root_up) {
  return apply_mixed(h, false, h->L, B, ldb, X, ldx, r, false, root_add, root_up);
}

int apply_inverse_up(hbs_handle* h, const cplx* B, int64_t ldb, int64_t r, cplx* root, int64_t ldr, hipEvent_t root_wait) {
  int rc = apply_mixed(h, true, h->fp64_top, B, ldb, nullptr, 0, r, false, nullptr, nullptr, 1, nullptr, root_wait);
  if (rc != HBS_OK || r <= 0) return rc;
  const int64_t n = h->nroot;
  CK(hipMemcpy2DAsync(root, sizeof(cplx) * ldr, h->ab_root.p, sizeof(cplx) * n, sizeof(cplx) * n, r, hipMemcpyDeviceToDevice,
                      h->stream));
  return HBS_OK;
}

int apply_inverse_down(hbs_handle* h, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r, const cplx* root_in) {
  return apply_mixed(h, true, h->fp64_top, B, ldb, X, ldx, r, false, nullptr, nullptr, 2, root_in);
}

int apply_factors(hbs_handle* h, bool inv, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r) {
  return apply_mixed(h, inv, inv ? h->fp64_top : h->L, B, ldb, X, ldx, r);
}

int apply_inverse(hbs_handle* h, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r) {
  return apply_mixed(h, true, h->fp64_top, B, ldb, X, ldx, r);
}

int apply_inverse_root(hbs_handle* h, const cplx* B, int64_t ldb, cplx* X, int64_t ldx, int64_t r, cplx* root, int64_t ldr,
                       bool sync) {
  int rc = apply_mixed(h, true, h->fp64_top, B, ldb, X, ldx, r, sync);
  if (rc != HBS_OK || r <= 0) return rc;
  // the root solution of the apply (still in the root workspace) is U^T A^{-1} B
  const int64_t n = h->nroot;
  if (ldr == n) {
    CK(hipMemcpyAsync(root, h->ab_root.p, sizeof(cplx) * n * r, hipMemcpyDeviceToDevice, h->stream));
  } else {
    CK(hipMemcpy2DAsync(root, sizeof(cplx) * ldr, h->ab_root.p, sizeof(cplx) * n, sizeof(cplx) * n, r,
                        hipMemcpyDeviceToDevice, h->stream));
  }
  if (sync) CK(hipStreamSynchronize(h->stream));
  return HBS_OK;
}

int ensure_root(hbs_handle* h) {
  switch (h->root_state) {
    case 0:
      return HBS_OK;
    case 2: {
      // inverted on the side stream by an earlier call that could not read its flag
      int f = 1;
      CK(hipStreamSynchronize(h->side_stream));
      CK(hipMemcpy(&f, h->root_flag, sizeof(int), hipMemcpyDeviceToHost));
      h->root_state = f ? 3 : 0;
      break;
    }
    case 1: {
      std::vector<InvDesc> iv = {{h->Rinv.as<cplx>(), h->nroot, h->nroot}};
      bool sing = false;
      CK(inv_batched(h->arena, h->work, iv, h->stream, &sing));
      h->root_state = sing ? 3 : 0;
      break;
    }
    default:
      break;
  }
  if (h->root_state != 0) {
    set_error("singular root matrix (hbs_opts.defer_root: found at the first use of the root inverse)");
    return HBS_E_SINGULAR;
  }
  return HBS_OK;
}

int side_stream_init(hbs_handle* h) {
  if (h->side_stream) return HBS_OK;
  // default priority, like every other stream of the library
  CK(hipStreamCreateWithFlags(&h->side_stream, hipStreamNonBlocking));
  for (auto& e : h->side_ev) CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return HBS_OK;
}

}  // namespace qps

hbs_handle::~hbs_handle() {
  for (auto& g : graphs)
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  for (auto e : side_ev)
    if (e) (void)hipEventDestroy(e);
  if (side_stream) (void)hipStreamDestroy(side_stream);
}
