// Batched complex FP64 GEMM on CDNA4 matrix cores: C = alpha op(A) B + beta C.
//
// Each workgroup (4 wavefronts, 2 x 2) computes a 64 x 64 tile of one batch entry; each
// wavefront owns a 32 x 32 sub-tile = 2 x 2 blocks of the 16 x 16 x 4 FP64 MFMA.  A complex
// product takes four real MFMAs into two accumulators (re += ar br - ai bi, im += ar bi + ai br).
// Operands are staged through LDS in k-slices of 16, split into real and imaginary planes.
// Batch entries may have different shapes; grid.x covers the largest tile count and
// workgroups past an entry's tile count exit.
#include "internal.h"

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, PADK = 2;

__device__ inline dbl4 mfma(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(256) void k_zgemm(const GemmDesc* __restrict__ descs) {
  const GemmDesc d = descs[blockIdx.y];
  const int tm = (d.m + BM - 1) / BM, tn = (d.n + BN - 1) / BN;
  const int t = blockIdx.x;
  if (t >= tm * tn || d.k <= 0) {
    // k == 0: C = beta C
    if (t < tm * tn && d.k <= 0) {
      const int i0 = (t % tm) * BM, j0 = (t / tm) * BN;
      for (int e = threadIdx.x; e < BM * BN; e += 256) {
        const int i = i0 + e % BM, j = j0 + e / BM;
        if (i < d.m && j < d.n) {
          cplx* c = d.C + i + (size_t)j * d.ldc;
          *c = (d.beta.x == 0.0 && d.beta.y == 0.0) ? mkc(0, 0) : cmul(d.beta, *c);
        }
      }
    }
    return;
  }
  const int i0 = (t % tm) * BM, j0 = (t / tm) * BN;
  __shared__ double Are[BK][BM + PADK], Aim[BK][BM + PADK];
  __shared__ double Bre[BK][BN + PADK], Bim[BK][BN + PADK];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv & 1, wn = wv >> 1;
  dbl4 accr[2][2], acci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = (dbl4){0.0, 0.0, 0.0, 0.0};
      acci[a][b] = (dbl4){0.0, 0.0, 0.0, 0.0};
    }
  const cplx* __restrict__ A = d.A;
  const cplx* __restrict__ B = d.B;
  for (int k0 = 0; k0 < d.k; k0 += BK) {
    // A slice: op(A)(i0 + ii, k0 + kk)
    if (!d.transA) {
#pragma unroll
      for (int q = 0; q < (BM * BK) / 256; ++q) {
        const int e = tid + q * 256;
        const int ii = e % BM, kk = e / BM;
        const int gi = i0 + ii, gk = k0 + kk;
        cplx v = (gi < d.m && gk < d.k) ? A[gi + (size_t)gk * d.lda] : mkc(0, 0);
        Are[kk][ii] = v.x;
        Aim[kk][ii] = v.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < (BM * BK) / 256; ++q) {
        const int e = tid + q * 256;
        const int kk = e % BK, ii = e / BK;
        const int gi = i0 + ii, gk = k0 + kk;
        cplx v = (gi < d.m && gk < d.k) ? A[gk + (size_t)gi * d.lda] : mkc(0, 0);
        Are[kk][ii] = v.x;
        Aim[kk][ii] = v.y;
      }
    }
#pragma unroll
    for (int q = 0; q < (BN * BK) / 256; ++q) {
      const int e = tid + q * 256;
      const int kk = e % BK, jj = e / BK;
      const int gj = j0 + jj, gk = k0 + kk;
      cplx v = (gj < d.n && gk < d.k) ? B[gk + (size_t)gj * d.ldb] : mkc(0, 0);
      Bre[kk][jj] = v.x;
      Bim[kk][jj] = v.y;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + (lane >> 4);
      double ar[2], ai[2], br[2], bi[2];
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
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          accr[a][b] = mfma(ar[a], br[b], accr[a][b]);
          accr[a][b] = mfma(-ai[a], bi[b], accr[a][b]);
          acci[a][b] = mfma(ar[a], bi[b], acci[a][b]);
          acci[a][b] = mfma(ai[a], br[b], acci[a][b]);
        }
    }
    __syncthreads();
  }
  // epilogue: register r of a lane holds row (lane/16) + 4r, column lane%16 of each 16 x 16 block
  const bool zero_beta = (d.beta.x == 0.0 && d.beta.y == 0.0);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = j0 + wn * 32 + b * 16 + (lane & 15);
      if (j >= d.n) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 32 + a * 16 + (lane >> 4) + 4 * r;
        if (i >= d.m) continue;
        cplx v = cmul(d.alpha, mkc(accr[a][b][r], acci[a][b][r]));
        cplx* c = d.C + i + (size_t)j * d.ldc;
        if (!zero_beta) v = cadd(v, cmul(d.beta, *c));
        *c = v;
      }
    }
}

}  // namespace

namespace qps {

hipError_t launch_zgemm(const GemmDesc* d, int nd, int max_tiles, hipStream_t s) {
  if (nd == 0 || max_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zgemm, dim3(max_tiles, nd), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t gemm_batched(DevBuf& arena, const std::vector<GemmDesc>& v, hipStream_t s) {
  if (v.empty()) return hipSuccess;
  int max_tiles = 0;
  double flops = 0.0, bytes = 0.0;
  for (const auto& g : v) {
    int t = ((g.m + BM - 1) / BM) * ((g.n + BN - 1) / BN);
    if (t > max_tiles) max_tiles = t;
    flops += 8.0 * g.m * (double)g.n * g.k;
    bytes += 16.0 * ((double)g.m * g.k + (double)g.k * g.n + 2.0 * g.m * g.n);
  }
  hipError_t e = upload(arena, v, s);
  if (e != hipSuccess) return e;
  ProfScope ps("zgemm", s, flops, bytes);
  return launch_zgemm(arena.as<GemmDesc>(), (int)v.size(), max_tiles, s);
}

}  // namespace qps
