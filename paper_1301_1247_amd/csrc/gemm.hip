// Batched complex GEMM on CDNA4 matrix cores: C = alpha op(A) B + beta C, in complex128
// (v_mfma_f64_16x16x4f64) or complex64 (v_mfma_f32_16x16x4f32).
//
// A workgroup of WM x WN wavefronts computes a (32 WM) x (32 WN) tile of one batch entry; each
// wavefront owns a 32 x 32 sub-tile = 2 x 2 blocks of the 16 x 16 x 4 MFMA.  A complex product
// takes four real MFMAs into two accumulators (re += ar br - ai bi, im += ar bi + ai br), issued
// so that two updates of one accumulator are 7 MFMAs apart.  Operands are staged through LDS in
// k-slices of 16 (real and imaginary planes); the next slice is fetched into registers while the
// current one is multiplied.  Batch entries may have different shapes; grid.x covers the largest
// tile count and workgroups past an entry's tile count exit.  Every tile configuration runs the
// same MFMA sequence for a given element of C, so the configurations give bitwise equal results
// and the choice among them (gemm_tune.cpp) affects only the time.  Long-K entries with few
// output tiles are split along K into a workspace and summed in a fixed order by a second kernel.
#include "internal.h"

#include <algorithm>

namespace {

constexpr int BK = 16, PADK = 2;

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 MFMA and its result layout (measured): register r of lane l holds column l % 16
// and row (l / 16) + 4 r in FP64, row 4 (l / 16) + r in FP32.
template <class R> struct mfma_t;
template <> struct mfma_t<double> {
  typedef dbl4 acc;
  __device__ static acc op(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct mfma_t<float> {
  typedef flt4 acc;
  __device__ static acc op(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// load of one complex element through a global-address-space pointer (descriptor pointers are
// generic; flat loads would also count against the LDS wait counter and hold up the LDS reads
// behind the prefetch of the next slice)
template <class R>
__device__ __forceinline__ typename cx<R>::T gload(const typename cx<R>::T* p) {
  typedef R v2 __attribute__((ext_vector_type(2)));
  const v2 v = *(const __attribute__((address_space(1))) v2*)p;
  return cx<R>::make(v.x, v.y);
}

template <class R>
__device__ __forceinline__ void gstore(typename cx<R>::T* p, typename cx<R>::T v) {
  typedef R v2 __attribute__((ext_vector_type(2)));
  v2 w;
  w.x = v.x;
  w.y = v.y;
  *(__attribute__((address_space(1))) v2*)p = w;
}

template <class R, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm(const GemmDescT<R>* __restrict__ descs, int xcd) {
  constexpr int BM = 32 * WM, BN = 32 * WN, NT = 64 * WM * WN;
  constexpr int QA = BM * BK / NT, QB = BK * BN / NT;  // slice elements of op(A) and B per thread
  typedef typename cx<R>::T C_t;
  typedef typename mfma_t<R>::acc acc_t;
  // xcd: XCD-aware order over the (descriptor, tile) items of a batch of independent products (the
  // per-box products of a level): the tiles of one descriptor, which share its operand panels, meet
  // in one L2 instead of each XCD fetching the panels.  The K-parts of a product split along K keep
  // launch order: all XCDs then work on the same K range at once and share it through the
  // last-level cache (one K-part per XCD measured twice as slow on products with K = 1.3e5).
  const int nx = gridDim.x;
  const int L = blockIdx.x + blockIdx.y * nx;
  const int T = xcd ? xcd_item(L, nx * gridDim.y) : L;
  const GemmDescT<R> d = descs[T / nx];
  const int tm = (d.m + BM - 1) / BM, tn = (d.n + BN - 1) / BN;
  const int t = T % nx;
  if (t >= tm * tn || d.k <= 0) {
    // k == 0: C = beta C
    if (t < tm * tn && d.k <= 0) {
      const int i0 = (t % tm) * BM, j0 = (t / tm) * BN;
      for (int e = threadIdx.x; e < BM * BN; e += NT) {
        const int i = i0 + e % BM, j = j0 + e / BM;
        if (i < d.m && j < d.n) {
          C_t* c = d.C + i + (size_t)j * d.ldc;
          gstore<R>(c, (d.beta.x == 0 && d.beta.y == 0) ? cx<R>::make(0, 0) : cmul(d.beta, gload<R>(c)));
        }
      }
    }
    return;
  }
  const int i0 = (t % tm) * BM, j0 = (t / tm) * BN;
  __shared__ R Are[BK][BM + PADK], Aim[BK][BM + PADK];
  __shared__ R Bre[BK][BN + PADK], Bim[BK][BN + PADK];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront-uniform
  const int wm = wv % WM, wn = wv / WM;
  // 16 x 16 blocks wholly outside C and k-steps past K take no MFMAs (ragged boxes of a batch
  // would otherwise pad every product to whole 64 x 64 x 16 tiles)
  const bool rv0 = i0 + wm * 32 < d.m, rv1 = i0 + wm * 32 + 16 < d.m;
  const bool cv0 = j0 + wn * 32 < d.n, cv1 = j0 + wn * 32 + 16 < d.n;
  const bool a00 = rv0 && cv0, a01 = rv0 && cv1, a10 = rv1 && cv0, a11 = rv1 && cv1;
#define QPS_ACT(a, b) ((a) ? ((b) ? a11 : a10) : ((b) ? a01 : a00))
  acc_t accr[2][2], acci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = (acc_t){0, 0, 0, 0};
      acci[a][b] = (acc_t){0, 0, 0, 0};
    }
  const C_t* __restrict__ A = d.A;
  const C_t* __restrict__ B = d.B;
  // register staging of one k-slice: QA elements of op(A) and QB of B per thread
  C_t ra[QA], rb[QB];
  auto load_slice = [&](int k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * NT;
      int ii, kk;
      if (!d.transA) { ii = e % BM; kk = e / BM; } else { kk = e % BK; ii = e / BK; }
      const int gi = i0 + ii, gk = k0 + kk;
      // a value select (a select of addresses with a local zero would make these flat loads)
      const bool in = gi < d.m && gk < d.k;
      const size_t off = d.transA ? gk + (size_t)gi * d.lda : gi + (size_t)gk * d.lda;
      ra[q] = cx<R>::make(0, 0);
      if (in) ra[q] = gload<R>(A + off);
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * NT;
      const int kb = e % BK, jj = e / BK;
      const int gj = j0 + jj, gkb = k0 + kb;
      rb[q] = cx<R>::make(0, 0);
      if (gj < d.n && gkb < d.k) rb[q] = gload<R>(B + gkb + (size_t)gj * d.ldb);
    }
  };
  auto store_slice = [&]() {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * NT;
      int ii, kk;
      if (!d.transA) { ii = e % BM; kk = e / BM; } else { kk = e % BK; ii = e / BK; }
      Are[kk][ii] = ra[q].x;
      Aim[kk][ii] = ra[q].y;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * NT;
      const int kb = e % BK, jj = e / BK;
      Bre[kb][jj] = rb[q].x;
      Bim[kb][jj] = rb[q].y;
    }
  };
  load_slice(0);
  store_slice();
  __syncthreads();
  for (int k0 = 0; k0 < d.k; k0 += BK) {
    const bool more = k0 + BK < d.k;
    if (more) load_slice(k0 + BK);  // in flight during the MFMAs below
    const int kv = d.k - k0;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      if (ks >= kv) break;
      const int kk = ks + (lane >> 4);
      R ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int ii = wm * 32 + a * 16 + (lane & 15);
        ar[a] = Are[kk][ii];
        ai[a] = Aim[kk][ii];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int jj = wn * 32 + b * 16 + (lane & 15);
        br[b] = Bre[kk][jj];
        bi[b] = Bim[kk][jj];
      }
      // issue order keeps 7 independent MFMAs between two updates of one accumulator
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if (QPS_ACT(a, b)) accr[a][b] = mfma_t<R>::op(ar[a], br[b], accr[a][b]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if (QPS_ACT(a, b)) acci[a][b] = mfma_t<R>::op(ar[a], bi[b], acci[a][b]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if (QPS_ACT(a, b)) accr[a][b] = mfma_t<R>::op(-ai[a], bi[b], accr[a][b]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          if (QPS_ACT(a, b)) acci[a][b] = mfma_t<R>::op(ai[a], br[b], acci[a][b]);
    }
    __syncthreads();
    if (more) {
      store_slice();
      __syncthreads();
    }
  }
#undef QPS_ACT
  // epilogue: register r of a lane holds row (lane/16) + 4r, column lane%16 of each 16 x 16 block
  const bool zero_beta = (d.beta.x == 0 && d.beta.y == 0);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = j0 + wn * 32 + b * 16 + (lane & 15);
      if (j >= d.n) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 32 + a * 16 + mfma_t<R>::row(lane, r);
        if (i >= d.m) continue;
        C_t v = cmul(d.alpha, cx<R>::make(accr[a][b][r], acci[a][b][r]));
        C_t* c = d.C + i + (size_t)j * d.ldc;
        if (!zero_beta) v = cadd(v, cmul(d.beta, gload<R>(c)));
        gstore<R>(c, v);
      }
    }
}

// C = alpha * sum_s W_s + beta * C over S partial products (m x n, ld m each)
template <class C_t>
__global__ __launch_bounds__(256) void k_splitk_reduce(C_t* __restrict__ C, int ldc, int m, int n,
                                                       const C_t* __restrict__ W, int S, C_t alpha, C_t beta) {
  const int64_t total = (int64_t)m * n;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    C_t acc = W[e];
    for (int q = 1; q < S; ++q) acc = cadd(acc, W[e + q * total]);
    const int i = (int)(e % m), j = (int)(e / m);
    C_t* c = C + i + (size_t)j * ldc;
    C_t v = cmul(alpha, acc);
    if (!(beta.x == 0 && beta.y == 0)) v = cadd(v, cmul(beta, *c));
    *c = v;
  }
}

// complex128 <-> complex64
__global__ __launch_bounds__(256) void k_cast_d2f(const cplx* __restrict__ s, cplxf* __restrict__ d, int64_t n) {
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) d[e] = mkcf((float)s[e].x, (float)s[e].y);
}
__global__ __launch_bounds__(256) void k_cast_f2d(const cplxf* __restrict__ s, cplx* __restrict__ d, int64_t n) {
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) d[e] = mkc(s[e].x, s[e].y);
}

}  // namespace

namespace qps {

template <class R>
hipError_t launch_gemm(const GemmDescT<R>* d, int nd, const GemmPlan& p, hipStream_t s) {
  if (nd == 0 || p.tiles == 0) return hipSuccess;
  const dim3 grid(p.tiles, nd);
  GemmTuneTimer tt(p, s);
  switch (p.cfg) {
    case 0: hipLaunchKernelGGL((k_gemm<R, 2, 2>), grid, dim3(256), 0, s, d, p.xcd); break;
    case 1: hipLaunchKernelGGL((k_gemm<R, 1, 1>), grid, dim3(64), 0, s, d, p.xcd); break;
    case 2: hipLaunchKernelGGL((k_gemm<R, 2, 1>), grid, dim3(128), 0, s, d, p.xcd); break;
    case 3: hipLaunchKernelGGL((k_gemm<R, 1, 2>), grid, dim3(128), 0, s, d, p.xcd); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_gemm<double>(const GemmDesc*, int, const GemmPlan&, hipStream_t);
template hipError_t launch_gemm<float>(const GemmDesc32*, int, const GemmPlan&, hipStream_t);

hipError_t launch_cast_d2f(const cplx* src, cplxf* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_d2f, dim3((int)std::min<int64_t>(8192, (n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_cast_f2d(const cplxf* src, cplx* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_f2d, dim3((int)std::min<int64_t>(8192, (n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

template <class R>
static int tiles_of(const GemmDescT<R>& g) { return ((g.m + 63) / 64) * ((g.n + 63) / 64); }

// split-K when there are too few output tiles to occupy the chip and the inner dimension is
// long: partial products go to a workspace and a second kernel sums them in a fixed order.  A
// descriptor with few tiles and a long inner dimension is the critical path of its launch (K >=
// 4096: up to ~1024 workgroups per descriptor, parts of >= 1024); a launch whose descriptors
// together have fewer output tiles than the chip has CUs, with 512 <= K < 4096, is split to ~512
// workgroups in parts of >= 128 (at most 8).  The decision depends on the shapes only, never on
// the tile configuration.
template <class R>
static int64_t launch_tiles(const std::vector<GemmDescT<R>>& v) {
  int64_t t = 0;
  for (const auto& g : v) t += tiles_of(g);
  return t;
}
template <class R>
static int split_of(const GemmDescT<R>& g, int64_t lt) {
  const int64_t tg = tiles_of(g);
  int S = 1;
  if (g.k >= 4096) {
    const int64_t target = 1024;
    if (tg >= target / 2) return 1;
    S = (int)std::min<int64_t>(64, (target + tg - 1) / tg);
    S = std::min(S, g.k / 1024);
  } else if (g.k >= 512 && lt < 256) {
    S = (int)std::min<int64_t>(8, (512 + lt - 1) / lt);
    S = std::min(S, g.k / 128);
  }
  return S >= 2 ? S : 1;
}

template <class R>
void gemm_batched_needs(const std::vector<GemmDescT<R>>& v, size_t* arena_bytes, size_t* ws_bytes) {
  size_t nd = 0, w = 0;
  const int64_t lt = launch_tiles(v);
  for (const auto& g : v) {
    const int S = split_of(g, lt);
    nd += S;
    if (S > 1) w += (size_t)S * g.m * g.n;
  }
  *arena_bytes = nd * sizeof(GemmDescT<R>);
  *ws_bytes = w * sizeof(typename cx<R>::T);
}

template <class R>
hipError_t gemm_batched(DevBuf& arena, const std::vector<GemmDescT<R>>& v0, hipStream_t s, DevBuf* ws) {
  typedef typename cx<R>::T C_t;
  typedef GemmDescT<R> GemmDesc;
  if (v0.empty()) return hipSuccess;
  double flops = 0.0, bytes = 0.0;
  for (const auto& g : v0) {
    flops += 8.0 * g.m * (double)g.n * g.k;
    bytes += 2.0 * sizeof(R) * ((double)g.m * g.k + (double)g.k * g.n + 2.0 * g.m * g.n);
  }
  std::vector<int> split(v0.size(), 1);
  int64_t wtot = 0;
  const int64_t lt = launch_tiles(v0);
  for (size_t i = 0; i < v0.size(); ++i) {
    split[i] = ws ? split_of(v0[i], lt) : 1;
    if (split[i] > 1) wtot += (int64_t)split[i] * v0[i].m * v0[i].n;
  }
  if (wtot > 0) {
    hipError_t e = ws->reserve(sizeof(C_t) * wtot);
    if (e != hipSuccess) return e;
  }
  struct Red { C_t* C; int ldc, m, n; const C_t* W; int S; C_t alpha, beta; };
  std::vector<Red> reds;
  std::vector<GemmDesc> v;
  int64_t woff = 0;
  for (size_t i = 0; i < v0.size(); ++i) {
    const GemmDesc& g = v0[i];
    const int S = split[i];
    if (S == 1) {
      v.push_back(g);
      continue;
    }
    C_t* W = ws->as<C_t>() + woff;
    woff += (int64_t)S * g.m * g.n;
    reds.push_back({g.C, g.ldc, g.m, g.n, W, S, g.alpha, g.beta});
    const int kc = (g.k + S - 1) / S;
    for (int q = 0; q < S; ++q) {
      GemmDesc h = g;
      const int k0 = q * kc;
      h.k = std::max(0, std::min(kc, g.k - k0));
      h.A = g.transA ? g.A + k0 : g.A + (size_t)k0 * g.lda;
      h.B = g.B + k0;
      h.C = W + (int64_t)q * g.m * g.n;
      h.ldc = g.m;
      h.alpha = cx<R>::make(1, 0);
      h.beta = cx<R>::make(0, 0);
      v.push_back(h);
    }
  }
  GemmPlan plan = gemm_plan(v.data(), v.size());
  if (!reds.empty()) plan.xcd = 0;  // K-parts share their K range through the last-level cache
  hipError_t e = upload(arena, v, s);
  if (e != hipSuccess) return e;
  {
    ProfScope ps(sizeof(R) == 8 ? "zgemm" : "cgemm", s, flops, bytes);
    e = launch_gemm<R>(arena.as<GemmDesc>(), (int)v.size(), plan, s);
    if (e != hipSuccess) return e;
  }
  for (const auto& r : reds) {
    const int64_t tot = (int64_t)r.m * r.n;
    const int grid = (int)std::min<int64_t>(8192, (tot + 255) / 256);
    hipLaunchKernelGGL(k_splitk_reduce<C_t>, dim3(grid), dim3(256), 0, s, r.C, r.ldc, r.m, r.n, r.W, r.S, r.alpha, r.beta);
  }
  return hipGetLastError();
}
template void gemm_batched_needs<double>(const std::vector<GemmDesc>&, size_t*, size_t*);
template void gemm_batched_needs<float>(const std::vector<GemmDesc32>&, size_t*, size_t*);
template hipError_t gemm_batched<double>(DevBuf&, const std::vector<GemmDesc>&, hipStream_t, DevBuf*);
template hipError_t gemm_batched<float>(DevBuf&, const std::vector<GemmDesc32>&, hipStream_t, DevBuf*);

}  // namespace qps
