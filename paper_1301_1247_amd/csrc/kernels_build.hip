// Device kernels of the recursive-skeletonization build (Sec. 4): block assembly of the
// Nystrom matrix, proxy-circle compression matrices (Sec. 3.2), sketching, column-pivoted QR
// interpolative decomposition (Def. 3.1), and batched Gauss-Jordan inversion.
#include "geometry.h"

namespace {

constexpr int NT = 256;  // threads per workgroup (4 wavefronts)

// ---------------------------------------------------------------- block evaluation
// TWO: the transmission operator (Sec. 5; plain and transposed blocks only)
template <bool TWO>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_blocks(Geo G, const BlockDesc* __restrict__ descs) {
  const BlockDesc d = descs[blockIdx.y];
  // one entry per thread, no grid-stride loop: inside a loop the compiler hoists the Hankel
  // coefficient tables into scalar registers and spills hundreds of them to vector lanes
  const int total = d.nr * d.nc;
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= total) return;
  {
    const int r = e % d.nr, c = e / d.nr;
    const int gr = d.rows[r], gc = d.cols[c];
    cplx v;
    if (TWO) {
      if (d.sx != 0.0) {
        // neighbour-image near points: the pair (image of gr as source of gc; image as target of gc)
        // through the exterior field only
        d.out[r + (size_t)c * d.ld] = a_ext_tr(G, gc, gr, 0.0, d.sx);
        d.out[d.pair_off + r + (size_t)c * d.ld] = a_ext_tr(G, gr, gc, d.sx, 0.0);
        return;
      }
      d.out[r + (size_t)c * d.ld] = d.trans ? a_entry_tr(G, gc, gr) : a_entry_tr(G, gr, gc);
      return;
    }
    if (d.trans == 2) {
      // the pair A(gc, gr~), A(gr~, gc) (gr~ = gr shifted by sx) from one Hankel evaluation: both
      // share r = |x_gc - x_gr~|; KR6's correction R depends on (gc - gr) mod N symmetrically
      const double dx = G.x[gc] - G.x[gr] - d.sx, dy = G.y[gc] - G.y[gr];
      const double rr = sqrt(dx * dx + dy * dy);
      cplx h0, h1;
      hankel01(G.omega * rr, h0, h1);
      const double q = 0.25 * G.omega;
      const double nd1 = (G.nx[gr] * dx + G.ny[gr] * dy) / rr;     // source gr~, target gc
      const double nd2 = -(G.nx[gc] * dx + G.ny[gc] * dy) / rr;    // source gc, target gr~
      double R = 1.0;
      if (d.sx == 0.0) {
        int m = gc - gr;
        if (m < 0) m += G.N;
        if (m <= 6) R += G.g[m - 1];
        else if (m >= G.N - 6) R += G.g[G.N - m - 1];
      }
      const cplx k1 = mkc(q * (h0.x - h1.y * nd1), q * (h0.y + h1.x * nd1));
      const cplx k2 = mkc(q * (h0.x - h1.y * nd2), q * (h0.y + h1.x * nd2));
      d.out[r + (size_t)c * d.ld] = cscale(k1, R * G.w[gr]);
      d.out[d.pair_off + r + (size_t)c * d.ld] = cscale(k2, R * G.w[gc]);
      return;
    }
    if (d.sx != 0.0) {
      // image point y_gr + (sx, 0): source of the field at x_gc (trans) or target of the field of x_gc
      v = d.trans ? cscale(helm_kernel(G.omega, G.x[gc] - G.x[gr] - d.sx, G.y[gc] - G.y[gr], G.nx[gr], G.ny[gr]), G.w[gr])
                  : cscale(helm_kernel(G.omega, G.x[gr] + d.sx - G.x[gc], G.y[gr] - G.y[gc], G.nx[gc], G.ny[gc]), G.w[gc]);
    } else {
      v = d.trans ? a_entry(G, gc, gr) : a_entry(G, gr, gc);
    }
    d.out[r + (size_t)c * d.ld] = v;
  }
}

// Transmission problem (Sec. 5): proxy rows for the unknown u = 2 i + c of the box, at the d.nk
// wavenumbers kq (q = 0: omega, q = 1: n omega), G_q = (i/4) H0(kq r), r = |x_i - p_l|:
//   row0 + (3q) np + l      incoming single layer: c = 0: G_q(x_i, p_l); c = 1: dG_q/dn_x      (x wp)
//   row0 + (3q + 1) np + l  incoming double layer: the same row functionals of
//                           [dG_q/dnu_l - i kq G_q](x_i, p_l)                                  (x wp)
//   row0 + (3q + 2) np + l  outgoing field on the circle: c = 0: dG_q/dn_y (p_l, x_i);
//                           c = 1: G_q(p_l, x_i)                                      (x w_i sqrt(wp))
// with the operator's normalization: the rows of c = 1 (normal-derivative functionals) divided by
// kbar, and its outgoing single-layer field multiplied by kbar.
// The fields that reach a box from outside its proxy circle solve Helmholtz' equation at k0 or k1
// inside the circle (spanned by the first two groups), and the fields the box sends out are
// radiating solutions at k0 and k1 fixed by their values on the circle (the third group).
__global__ __launch_bounds__(NT) void k_proxy_tr(Geo G, const ProxyDesc* __restrict__ descs) {
  const ProxyDesc d = descs[blockIdx.y];
  const int total = d.np * d.n;
  const double wp = 2.0 * QPS_PI * d.R / d.np;
  const double swp = sqrt(wp);
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= total) return;
  const int l = e % d.np, iu = e / d.np;
  double sn, cs;
  sincos(2.0 * QPS_PI * l / d.np, &sn, &cs);
  const double px = d.cx + d.R * cs, py = d.cy + d.R * sn;
  const int u = d.act[iu], gi = u >> 1, c = u & 1;
  const double dx = G.x[gi] - px, dy = G.y[gi] - py;  // x_i - p_l
  const double r = sqrt(dx * dx + dy * dy);
  const double ni = (G.nx[gi] * dx + G.ny[gi] * dy) / r;  // n_i.(x_i - p)/r
  const double nu = (cs * dx + sn * dy) / r;              // nu_l.(x_i - p)/r
  const double nn = G.nx[gi] * cs + G.ny[gi] * sn;
  cplx* col = d.wt + (size_t)iu * d.m + d.row0;
  // both Hankel pairs first, in straight-line code (evaluated inside the loop, their coefficient
  // tables are hoisted into scalar registers and spilled)
  cplx hh[2][2];
  hankel01(G.omega * r, hh[0][0], hh[0][1]);
  hankel01(G.omega1 * r, hh[1][0], hh[1][1]);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (q >= d.nk) break;
    const double k = q ? G.omega1 : G.omega;
    const cplx h0 = hh[q][0], h1 = hh[q][1];
    const cplx g = mkc(-0.25 * h0.y, 0.25 * h0.x);                      // G
    const cplx gh1 = mkc(-0.25 * k * h1.y, 0.25 * k * h1.x);            // (i/4) k H1
    cplx in1, in2, out;
    if (c == 0) {
      in1 = g;
      // dG/dnu_p = (i/4) k H1 nu.(x - p)/r;  - i k G = (k/4) H0
      in2 = mkc(gh1.x * nu + 0.25 * k * h0.x, gh1.y * nu + 0.25 * k * h0.y);
      // dG/dn_y(p, x_i) with target p, source x_i: (i/4) k H1 n_i.(p - x_i)/r
      out = cscale(gh1, -ni);
    } else {
      // dG/dn_x = -(i/4) k H1 n_i.(x - p)/r
      in1 = cscale(gh1, -ni);
      // d/dn_x [dG/dnu_p - i k G] = T(x, p; n_i, nu) - i k dG/dn_x,
      // T = (i/4) [k^2 H0 a b + (k H1 / r)(nn - 2 a b)], a = n_i.(x - p)/r, b = nu.(x - p)/r
      const double ab = ni * nu, cc = (nn - 2.0 * ab) / r;
      const cplx T = mkc(-0.25 * (k * k * h0.y * ab + k * h1.y * cc), 0.25 * (k * k * h0.x * ab + k * h1.x * cc));
      const cplx dx_ = cscale(gh1, -ni);                                // dG/dn_x
      in2 = mkc(T.x + k * dx_.y, T.y - k * dx_.x);                        // T - i k dG/dn_x
      out = g;
    }
    const double fin = c ? wp / G.kbar : wp, fout = c ? G.w[gi] * swp * G.kbar : G.w[gi] * swp;
    col[(3 * q) * d.np + l] = cscale(in1, fin);
    col[(3 * q + 1) * d.np + l] = cscale(in2, fin);
    col[(3 * q + 2) * d.np + l] = cscale(out, fout);
  }
}

// Proxy rows of W^T for one box.  For proxy p_l = c + R (cos th_l, sin th_l) with outward
// normal nu_l and active point x_i (normal n_i, weight w_i), with wp = 2 pi R / np:
//   row0 + l          G(x_i, p_l) wp                         (incoming fields, single layer)
//   row0 + np + l     [dG/dnu_l - i omega G](x_i, p_l) wp      (incoming fields, double layer)
//   row0 + 2 np + l   K(p_l, x_i, n_i) w_i sqrt(wp)          (outgoing field of x_i on the circle)
__global__ __launch_bounds__(NT) void k_proxy(Geo G, const ProxyDesc* __restrict__ descs) {
  const ProxyDesc d = descs[blockIdx.y];
  const int total = d.np * d.n;
  const double wp = 2.0 * QPS_PI * d.R / d.np;
  const double swp = sqrt(wp);
  const double q = 0.25 * G.omega;
  // one entry per thread (see k_eval_blocks)
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= total) return;
  {
    const int l = e % d.np, i = e / d.np;
    double sn, cs;
    sincos(2.0 * QPS_PI * l / d.np, &sn, &cs);
    const double px = d.cx + d.R * cs, py = d.cy + d.R * sn;
    const int gi = d.act[i];
    const double dx = G.x[gi] - px, dy = G.y[gi] - py;  // x_i - p_l
    const double r = sqrt(dx * dx + dy * dy);
    cplx h0, h1;
    hankel01(G.omega * r, h0, h1);
    // G = (i/4) h0
    const cplx gv = mkc(-0.25 * h0.y, 0.25 * h0.x);
    // K(x_i, p_l, nu_l): n = nu_l, x - y = (dx, dy)
    const double nd1 = (cs * dx + sn * dy) / r;
    const cplx k1 = mkc(q * (h0.x - h1.y * nd1), q * (h0.y + h1.x * nd1));
    // K(p_l, x_i, n_i): x - y = -(dx, dy)
    const double nd2 = -(G.nx[gi] * dx + G.ny[gi] * dy) / r;
    const cplx k2 = mkc(q * (h0.x - h1.y * nd2), q * (h0.y + h1.x * nd2));
    cplx* col = d.wt + (size_t)i * d.m + d.row0;
    col[l] = cscale(gv, wp);
    col[d.np + l] = cscale(k1, wp);
    col[2 * d.np + l] = cscale(k2, G.w[gi] * swp);
  }
}

// Rademacher signs from a counter-based hash (SplitMix64's finalizer)
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Z = Omega * W^T with complex Rademacher entries (+-1 +- i)/sqrt(2), tiles of 32 (sketch rows) x 32
// (columns) per workgroup.  One hash gives the 64 sign bits of a sketch row over a 32-row slice of W.
// (A real sign matrix would halve the multiply-adds, but it embeds the k complex dimensions of W's
// row space as 2k real ones, too many for the 2n + 8 rows of the top levels, where k is close to n.)
__global__ __launch_bounds__(NT) void k_sketch(const SketchDesc* __restrict__ descs, uint64_t seed) {
  // XCD-aware order: the row tiles of one column tile read the same columns of W
  const int gx = gridDim.x, gy = gridDim.y;
  const int T = xcd_item(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
  const SketchDesc d = descs[T / (gx * gy)];
  const int q0 = (T % gx) * 32, i0 = ((T / gx) % gy) * 32;
  if (q0 >= d.s || i0 >= d.n) return;
  __shared__ cplx Ws[32][33];
  __shared__ uint64_t Om[32];
  const int tid = threadIdx.x;
  const int tq = tid % 32, ti = tid / 32;  // each thread: row q0+tq, columns i0+ti+8*c
  cplx acc[4] = {mkc(0, 0), mkc(0, 0), mkc(0, 0), mkc(0, 0)};
  const uint64_t bseed = mix64(seed ^ (0x9E3779B97F4A7C15ull * (uint64_t)(d.box + 1)));
  constexpr double h = 0.70710678118654752440;
  for (int r0 = 0; r0 < d.m; r0 += 32) {
    for (int e = tid; e < 32 * 32; e += NT) {
      const int rr = e % 32, ii = e / 32;
      const int gr = r0 + rr, gi = i0 + ii;
      Ws[rr][ii] = (gr < d.m && gi < d.n) ? d.wt[gr + (size_t)gi * d.m] : mkc(0, 0);
    }
    if (tid < 32)
      Om[tid] = mix64(bseed + 0xD1B54A32D192ED03ull * (uint64_t)(q0 + tid) + 0x8CB92BA72F3D8DD7ull * (uint64_t)(r0 >> 5));
    __syncthreads();
    const uint64_t bits = Om[tq];
#pragma unroll 8
    for (int rr = 0; rr < 32; ++rr) {
      const cplx o = mkc(((bits >> (2 * rr)) & 1) ? h : -h, ((bits >> (2 * rr + 1)) & 1) ? h : -h);
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = cfma(o, Ws[rr][ti + 8 * c], acc[c]);
    }
    __syncthreads();
  }
  const int q = q0 + tq;
  if (q < d.s) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + ti + 8 * c;
      if (i < d.n) d.z[q + (size_t)i * d.s] = acc[c];
    }
  }
}

// ---------------------------------------------------------------- CPQR / ID
// T = R11^{-1} R12 in place in Z[0:k, k:n] (Z: s x n, ld s), by blocks of 64 rows from the bottom:
// the diagonal block is solved by one wavefront per column with the right-hand side in registers
// (the solved entry is broadcast with readlane), then the rows above are updated by all threads.
// With lds (room for BH (BH + 1) + BH complex values), the blocks are BH rows high and each block
// of R11 and the inverses of its diagonal are staged there first, so the serial steps wait on
// LDS instead of on global memory (same arithmetic, same results).  Called by the whole
// workgroup.
template <int BH>
constexpr int cpqr_ts_lds() { return BH * (BH + 1) + BH; }
constexpr int CPQR_TS_LDS = cpqr_ts_lds<64>();
template <int NTQ, int BH = 64>
__device__ void cpqr_tsolve(cplx* Z, int s, int n, int k, cplx* lds) {
  static_assert(BH >= 1 && BH <= 64, "one lane per row of a block");
  constexpr int LD = BH + 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nw = NTQ / 64;
  for (int i1 = k; i1 > 0; i1 -= BH) {
    const int i0 = max(0, i1 - BH);
    const int nbk = i1 - i0;
    if (lds) {
      for (int e = tid; e < nbk * nbk; e += NTQ) {
        const int r = e % nbk, c = e / nbk;
        lds[r * LD + c] = Z[(i0 + r) + (size_t)(i0 + c) * s];
      }
      __syncthreads();
      for (int r = tid; r < nbk; r += NTQ) {
        const cplx zii = lds[r * LD + r];
        lds[BH * LD + r] = cabs2(zii) > 0.0 ? cinv(zii) : mkc(0, 0);
      }
      __syncthreads();
    }
    for (int j = k + wv; j < n; j += nw) {
      cplx* col = Z + (size_t)j * s;
      const int l = i0 + lane;
      cplx t = (l < i1) ? col[l] : mkc(0, 0);
      for (int i = i1 - 1; i >= i0; --i) {
        const int li = i - i0;
        if (lane == li) {
          if (lds) {
            t = cmul(t, lds[BH * LD + li]);
          } else {
            const cplx zii = Z[i + (size_t)i * s];
            t = cabs2(zii) > 0.0 ? cmul(t, cinv(zii)) : mkc(0, 0);
          }
        }
        const long long bx = __double_as_longlong(t.x), by = __double_as_longlong(t.y);
        const int xlo = __builtin_amdgcn_readlane((int)(bx & 0xffffffff), li), xhi = __builtin_amdgcn_readlane((int)(bx >> 32), li);
        const int ylo = __builtin_amdgcn_readlane((int)(by & 0xffffffff), li), yhi = __builtin_amdgcn_readlane((int)(by >> 32), li);
        const cplx ti = mkc(__longlong_as_double(((long long)xhi << 32) | (unsigned)xlo),
                            __longlong_as_double(((long long)yhi << 32) | (unsigned)ylo));
        if (lane < li) {
          const cplx zl = lds ? lds[lane * LD + li] : Z[l + (size_t)i * s];
          t = csub(t, cmul(zl, ti));
        }
      }
      if (l < i1) col[l] = t;
    }
    __syncthreads();
    if (i0 > 0) {
      const int rows = i0, cols = n - k;
      for (int e = tid; e < rows * cols; e += NTQ) {
        const int r = e % rows, j = k + e / rows;
        cplx* col = Z + (size_t)j * s;
        cplx acc = col[r];
#pragma unroll 8
        for (int i = i0; i < i1; ++i) acc = csub(acc, cmul(Z[r + (size_t)i * s], col[i]));
        col[r] = acc;
      }
      __syncthreads();
    }
  }
}

// One workgroup per box.  Householder QR with column pivoting on Z (s x n, in place, global
// memory).  Column norms of the trailing rows are recomputed exactly in every update pass.
// Rank: the first p with |R_pp| <= tol |R_00| (at least 1).
// Two instantiations: 1024 threads with room for s <= 4608, n <= 2048 (few, large boxes), and
// 256 threads with s <= 512, n <= 256 (many small boxes: several workgroups per CU hide the
// memory latency of the column updates).
constexpr int CPQR_MAXN = 2048;
constexpr int CPQR_MAXS = 4608;
// RC > 0: while the trailing rows fit in RC per lane (16 lanes per column), a column's rows are
// loaded into registers in one burst, so its inner product and update wait for memory once.
template <int NTQ, int MAXS, int MAXN, int RC>
__global__ __launch_bounds__(NTQ) void k_cpqr(const CpqrDesc* __restrict__ descs, double tol, int* __restrict__ k_out) {
  const CpqrDesc d = descs[blockIdx.x];
  const int s = d.s, n = d.n;
  cplx* Z = d.z;
  __shared__ double cn[MAXN];
  __shared__ int perm[MAXN];
  __shared__ cplx v[MAXS];
  __shared__ double red_v[NTQ / 64];
  __shared__ int red_i[NTQ / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nw = NTQ / 64;
  for (int j = tid; j < n; j += NTQ) perm[j] = j;
  for (int j = wv; j < n; j += nw) {
    double a = 0.0;
    for (int i = lane; i < s; i += 64) a += cabs2(Z[i + (size_t)j * s]);
    a = wave_sum(a);
    if (lane == 0) cn[j] = a;
  }
  __syncthreads();
  const int pmax = min(s, n);
  int k = pmax;
  double r00 = 0.0;
  for (int p = 0; p < pmax; ++p) {
    // pivot: argmax over j in [p, n), then every thread reduces the wavefronts' candidates
    double bv = -1.0;
    int bi = n;
    for (int j = p + tid; j < n; j += NTQ) {
      const double c = cn[j];
      if (c > bv || (c == bv && j < bi)) { bv = c; bi = j; }
    }
    wave_argmax(bv, bi);
    if (lane == 0) { red_v[wv] = bv; red_i[wv] = bi; }
    __syncthreads();
    double b = red_v[0];
    int jp = red_i[0];
    for (int w = 1; w < nw; ++w)
      if (red_v[w] > b || (red_v[w] == b && red_i[w] < jp)) { b = red_v[w]; jp = red_i[w]; }
    const double nr = sqrt(fmax(b, 0.0));
    if (p == 0) r00 = nr;
    if ((p > 0 && nr <= tol * r00) || (p == 0 && nr == 0.0)) { k = (p == 0) ? 1 : p; break; }
    // swap columns p and jp, and stage the new column p (rows p..s-1) in LDS
    for (int i = tid; i < s; i += NTQ) {
      const cplx zp = Z[i + (size_t)p * s];
      const cplx zj = Z[i + (size_t)jp * s];
      if (jp != p) Z[i + (size_t)jp * s] = zp;
      Z[i + (size_t)p * s] = zj;
      if (i >= p) v[i] = zj;
    }
    if (tid == 0 && jp != p) {
      double t = cn[p]; cn[p] = cn[jp]; cn[jp] = t;
      int ti = perm[p]; perm[p] = perm[jp]; perm[jp] = ti;
    }
    __syncthreads();
    // Householder vector of x = Z[p:s, p] (every wavefront forms the same reduction)
    double a = 0.0;
    for (int i = p + lane; i < s; i += 64) a += cabs2(v[i]);
    a = wave_sum(a);
    const double xn = sqrt(a);
    const cplx x0 = v[p];
    const double ax0 = sqrt(cabs2(x0));
    const cplx alpha = (ax0 > 0.0) ? cscale(x0, -xn / ax0) : mkc(-xn, 0.0);
    const cplx v0 = csub(x0, alpha);
    const double vn2 = a - ax0 * ax0 + cabs2(v0);
    const double tau = (vn2 > 0.0) ? 2.0 / vn2 : 0.0;
    if (tid == 0) Z[p + (size_t)p * s] = alpha;
    // apply H = I - tau v v^* to columns j > p (v[p] replaced by v0 in registers) and recompute
    // the trailing norms.  Each 16-lane row of a wavefront takes one column, so one reduction
    // instruction serves four columns.
    const int sub = lane >> 4, rl = lane & 15;
    if (RC > 0 && s - p <= 16 * RC) {
      for (int j0 = p + 1 + 4 * wv; j0 < n; j0 += 4 * nw) {
        const int j = j0 + sub;
        const bool act = j < n;
        cplx* col = Z + (size_t)(act ? j : p) * s;
        cplx c[RC > 0 ? RC : 1];
#pragma unroll
        for (int t = 0; t < RC; ++t) {
          const int i = p + rl + 16 * t;
          c[t] = (act && i < s) ? col[i] : mkc(0, 0);
        }
        cplx w = mkc(0, 0);
#pragma unroll
        for (int t = 0; t < RC; ++t) {
          const int i = p + rl + 16 * t;
          if (i < s) w = cadd(w, cmul(cconj(i == p ? v0 : v[i]), c[t]));
        }
        w = cscale(row16_csum(w), tau);
        double an = 0.0;
#pragma unroll
        for (int t = 0; t < RC; ++t) {
          const int i = p + rl + 16 * t;
          if (act && i < s) {
            const cplx z = csub(c[t], cmul(w, i == p ? v0 : v[i]));
            col[i] = z;
            if (i > p) an += cabs2(z);
          }
        }
        an = row16_sum(an);
        if (act && rl == 0) cn[j] = an;
      }
    } else {
      for (int j0 = p + 1 + 4 * wv; j0 < n; j0 += 4 * nw) {
        const int j = j0 + sub;
        const bool act = j < n;
        cplx* col = Z + (size_t)(act ? j : p) * s;
        cplx w = mkc(0, 0);
        if (act)
          for (int i = p + rl; i < s; i += 16) w = cadd(w, cmul(cconj(i == p ? v0 : v[i]), col[i]));
        w = cscale(row16_csum(w), tau);
        double an = 0.0;
        if (act)
          for (int i = p + rl; i < s; i += 16) {
            const cplx z = csub(col[i], cmul(w, i == p ? v0 : v[i]));
            col[i] = z;
            if (i > p) an += cabs2(z);
          }
        an = row16_sum(an);
        if (act && rl == 0) cn[j] = an;
      }
    }
    __syncthreads();
  }
  __syncthreads();  // v is reused as the staging area of the triangular solve
  if constexpr (MAXS >= cpqr_ts_lds<64>())
    cpqr_tsolve<NTQ, 64>(Z, s, n, k, v);
  else
    cpqr_tsolve<NTQ, 16>(Z, s, n, k, v);
  static_assert(MAXS >= cpqr_ts_lds<16>(), "pivot vector too small to stage the triangular solve");
  for (int j = tid; j < n; j += NTQ) d.perm[j] = perm[j];
  if (tid == 0) k_out[blockIdx.x] = k;
}

// ---- column-pivoted QR of a few large boxes: one launch per pivot step
// The one-workgroup kernel streams a box's whole trailing matrix through one CU at every pivot;
// at the top levels (a handful of boxes) that leaves most of the chip idle and bounds a step by
// one CU's bandwidth.  Here each pivot step is one launch, and each box's columns are spread over
// workgroups of 16 columns: every workgroup finds the pivot from the column norms the previous
// launch left, forms the same Householder vector from the pivot column (same data, same
// arithmetic, hence the same bits in every workgroup), and applies it to its own 16 columns.
// Columns do not move: a logical-to-physical column map and the norms are double-buffered
// between launches (launch p reads buffer p & 1 and writes the other, for the columns after p),
// and the pivot's physical column and R's diagonal entry are recorded per step.  A gather puts
// the columns in pivot order into a second buffer, T = R11^{-1} R12 is formed there, and the
// result is copied back.  The termination rule and the outputs are those of k_cpqr.
constexpr int CPQRM_MAXS = 1024;
struct CpqrmState {
  int done, k, np, pad;  // np: pivot steps carried out (columns in pivot order)
  double r00, pad2;
};
struct CpqrmWs {
  int *pcA, *pcB, *fin;
  double *cnA, *cnB;
  cplx* alph;
  CpqrmState* st;
  cplx* W2;
  int maxn;
  int64_t zstride;
};

__global__ __launch_bounds__(256) void k_cpqrm_init(const CpqrDesc* __restrict__ descs, CpqrmWs W) {
  const CpqrDesc d = descs[blockIdx.y];
  const int b = blockIdx.y, s = d.s, n = d.n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, sub = lane >> 4, rl = lane & 15;
  const int j = 16 * blockIdx.x + 4 * wv + sub;
  double a = 0.0;
  if (j < n)
    for (int i = rl; i < s; i += 16) a += cabs2(d.z[i + (size_t)j * s]);
  a = row16_sum(a);
  if (j < n && rl == 0) {
    W.cnA[(size_t)b * W.maxn + j] = a;
    W.pcA[(size_t)b * W.maxn + j] = j;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int pmax = min(s, n);
    CpqrmState st0;
    st0.done = 0; st0.k = pmax; st0.np = pmax; st0.pad = 0; st0.r00 = 0.0; st0.pad2 = 0.0;
    W.st[b] = st0;
  }
}

constexpr int CPQRM_RC = 24;  // rows per lane of a column held in registers (16 lanes per column)
__global__ __launch_bounds__(256) void k_cpqrm_step(const CpqrDesc* __restrict__ descs, CpqrmWs W, int p, double tol) {
  const CpqrDesc d = descs[blockIdx.y];
  const int b = blockIdx.y, s = d.s, n = d.n;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (p >= min(s, n)) return;
  const int slot0 = p + 1 + 16 * (int)blockIdx.x;
  if (blockIdx.x != 0 && slot0 >= n) return;
  CpqrmState* S = W.st + b;
  // a box whose rank is found costs its remaining launches nothing but this read
  if (S->done) return;
  const size_t o = (size_t)b * W.maxn;
  const int* pcO = ((p & 1) ? W.pcB : W.pcA) + o;
  const double* cnO = ((p & 1) ? W.cnB : W.cnA) + o;
  int* pcN = ((p & 1) ? W.pcA : W.pcB) + o;
  double* cnN = ((p & 1) ? W.cnA : W.cnB) + o;
  // this workgroup's columns (16 lanes per column, 4 per wavefront): their rows p.. are loaded
  // now, beside the pivot search, unless the column is the one that moves to position jp
  const int sub = lane >> 4, rl = lane & 15;
  const int j = slot0 + 4 * wv + sub;
  const bool act = j < n;
  const bool reg = s - p <= 16 * CPQRM_RC;
  // (clamped: a box that stopped at step 0 never wrote the second map buffer; it returns below,
  // but the prefetch must stay inside Z)
  int phys = act ? min(max(pcO[j], 0), n - 1) : 0;
  cplx c[CPQRM_RC];
  if (reg) {
#pragma unroll
    for (int t = 0; t < CPQRM_RC; ++t) {
      const int i = p + rl + 16 * t;
      c[t] = (act && i < s) ? d.z[i + (size_t)phys * s] : mkc(0, 0);
    }
  }
  __shared__ double rv[4];
  __shared__ int ri[4];
  __shared__ cplx v[CPQRM_MAXS];
  // pivot: the largest remaining norm (ties: the smaller position)
  double bv = -1.0;
  int bi = n;
  for (int j = p + tid; j < n; j += 256) {
    const double c = cnO[j];
    if (c > bv || (c == bv && j < bi)) { bv = c; bi = j; }
  }
  wave_argmax(bv, bi);
  if (lane == 0) { rv[wv] = bv; ri[wv] = bi; }
  __syncthreads();
  double bb = rv[0];
  int jp = ri[0];
  for (int w = 1; w < 4; ++w)
    if (rv[w] > bb || (rv[w] == bb && ri[w] < jp)) { bb = rv[w]; jp = ri[w]; }
  const double nr = sqrt(fmax(bb, 0.0));
  const double r00 = (p == 0) ? nr : S->r00;
  if ((p > 0 && nr <= tol * r00) || (p == 0 && nr == 0.0)) {
    if (blockIdx.x == 0 && tid == 0) {
      S->k = (p == 0) ? 1 : p;
      S->np = p;
      S->done = 1;
    }
    return;
  }
  const int ph = pcO[jp];  // the pivot's physical column (read only in this launch)
  const int pq = pcO[p];   // the column that moves to position jp
  const cplx* zc = d.z + (size_t)ph * s;
  for (int i = p + tid; i < s; i += 256) v[i - p] = zc[i];
  __syncthreads();
  // Householder vector of x = Z[p:s, ph] (every wavefront forms the same reduction)
  double a = 0.0;
  for (int i = lane; i < s - p; i += 64) a += cabs2(v[i]);
  a = wave_sum(a);
  const double xn = sqrt(a);
  const cplx x0 = v[0];
  const double ax0 = sqrt(cabs2(x0));
  const cplx alpha = (ax0 > 0.0) ? cscale(x0, -xn / ax0) : mkc(-xn, 0.0);
  const cplx v0 = csub(x0, alpha);
  const double vn2 = a - ax0 * ax0 + cabs2(v0);
  const double tau = (vn2 > 0.0) ? 2.0 / vn2 : 0.0;
  if (blockIdx.x == 0 && tid == 0) {
    W.fin[o + p] = ph;
    W.alph[o + p] = alpha;
    if (p == 0) S->r00 = nr;
  }
  // the column at position jp is the one that was at position p
  if (act && j == jp) {
    phys = pq;
    if (reg) {
#pragma unroll
      for (int t = 0; t < CPQRM_RC; ++t) {
        const int i = p + rl + 16 * t;
        c[t] = (i < s) ? d.z[i + (size_t)phys * s] : mkc(0, 0);
      }
    }
  }
  cplx* col = d.z + (size_t)(act ? phys : ph) * s;
  cplx w = mkc(0, 0);
  double an = 0.0;
  if (reg) {
#pragma unroll
    for (int t = 0; t < CPQRM_RC; ++t) {
      const int i = p + rl + 16 * t;
      if (act && i < s) w = cadd(w, cmul(cconj(i == p ? v0 : v[i - p]), c[t]));
    }
    w = cscale(row16_csum(w), tau);
#pragma unroll
    for (int t = 0; t < CPQRM_RC; ++t) {
      const int i = p + rl + 16 * t;
      if (act && i < s) {
        const cplx z = csub(c[t], cmul(w, i == p ? v0 : v[i - p]));
        col[i] = z;
        if (i > p) an += cabs2(z);
      }
    }
  } else {
    if (act)
      for (int i = p + rl; i < s; i += 16) w = cadd(w, cmul(cconj(i == p ? v0 : v[i - p]), col[i]));
    w = cscale(row16_csum(w), tau);
    if (act)
      for (int i = p + rl; i < s; i += 16) {
        const cplx z = csub(col[i], cmul(w, i == p ? v0 : v[i - p]));
        col[i] = z;
        if (i > p) an += cabs2(z);
      }
  }
  an = row16_sum(an);
  if (act && rl == 0) {
    cnN[j] = an;
    pcN[j] = phys;
  }
}

// columns in pivot order into W2 (R's diagonal from the recorded steps), the permutation, the rank
__global__ __launch_bounds__(256) void k_cpqrm_gather(const CpqrDesc* __restrict__ descs, CpqrmWs W, int* __restrict__ k_out) {
  const CpqrDesc d = descs[blockIdx.y];
  const int b = blockIdx.y, s = d.s, n = d.n, j = blockIdx.x;
  if (j >= n) return;
  const CpqrmState S = W.st[b];
  const int pmax = min(s, n);
  const int k = S.done ? S.k : pmax, np = S.done ? S.np : pmax;
  const size_t o = (size_t)b * W.maxn;
  const int* pcF = ((np & 1) ? W.pcB : W.pcA) + o;
  const int phys = (j < np) ? W.fin[o + j] : pcF[j];
  const cplx* src = d.z + (size_t)phys * s;
  cplx* dst = W.W2 + (size_t)b * W.zstride + (size_t)j * s;
  const cplx al = (j < np) ? W.alph[o + j] : mkc(0, 0);
  for (int i = threadIdx.x; i < s; i += 256) {
    cplx val = src[i];
    if (j < np && i == j) val = al;
    dst[i] = val;
  }
  if (threadIdx.x == 0) {
    d.perm[j] = phys;
    if (j == 0) k_out[b] = k;
  }
}

// T = R11^{-1} R12 in W2, then W2 back into Z
__global__ __launch_bounds__(1024) void k_cpqrm_tsolve(const CpqrDesc* __restrict__ descs, CpqrmWs W) {
  const CpqrDesc d = descs[blockIdx.x];
  const int b = blockIdx.x, s = d.s, n = d.n;
  const CpqrmState S = W.st[b];
  const int k = S.done ? S.k : min(s, n);
  cplx* Z2 = W.W2 + (size_t)b * W.zstride;
  __shared__ cplx stage[CPQR_TS_LDS];
  cpqr_tsolve<1024>(Z2, s, n, k, stage);
  __syncthreads();
  const int64_t tot = (int64_t)s * n;
  for (int64_t e = threadIdx.x; e < tot; e += 1024) d.z[e] = Z2[e];
}

// P (n x k): P[perm[j], j] = 1 (j < k), P[perm[k + i], j] = T[j, i]
__global__ __launch_bounds__(NT) void k_buildP(const PDesc* __restrict__ descs) {
  const PDesc d = descs[blockIdx.y];
  const int total = d.n * d.k;
  for (int e = blockIdx.x * NT + threadIdx.x; e < total; e += gridDim.x * NT) {
    const int r = e % d.n, j = e / d.n;  // r: position in pivot order
    const int row = d.perm[r];
    cplx v;
    if (r < d.k) v = mkc(r == j ? 1.0 : 0.0, 0.0);
    else v = d.z[j + (size_t)r * d.s];
    d.P[row + (size_t)j * d.n] = v;
  }
}

__global__ __launch_bounds__(NT) void k_copy(const CopyDesc* __restrict__ descs) {
  const CopyDesc d = descs[blockIdx.y];
  const int total = d.nr * d.nc;
  for (int e = blockIdx.x * NT + threadIdx.x; e < total; e += gridDim.x * NT) {
    const int r = e % d.nr, c = e / d.nr;
    d.dst[r + (size_t)c * d.ldd] = d.src ? d.src[r + (size_t)c * d.lds] : mkc(0, 0);
  }
}

// Bounding circle of the nodes lo[b] <= i < hi[b] of every box b: centre = middle of the
// Per box [lo, hi) of the original nodes (one workgroup per box, every level in one launch):
// bounding box, radius = largest distance from its centre, and the features of the rank
// predictor: max and mean |curvature| over the nodes (|kappa_i| when the curvature is given,
// else the turning angle of the normals between the neighbours i-1, i+1 over the arc length
// between them) and the box's arc length (sum of the weights).
// out = cx, cy, r, x0, x1, y0, y1, max|kappa|, mean|kappa|, arc length (BOX_OUT per box).
constexpr int BOX_OUT = 10;
__global__ __launch_bounds__(NT) void k_box_circles(Geo G, const int* __restrict__ lo, const int* __restrict__ hi,
                                                    double* __restrict__ out) {
  const int b = blockIdx.x;
  const int i0 = lo[b], i1 = hi[b], N = G.N;
  const double* __restrict__ x = G.x;
  const double* __restrict__ y = G.y;
  __shared__ double red[7][NT / 64];
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300, km = 0.0, ks = 0.0, al = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += NT) {
    x0 = fmin(x0, x[i]); x1 = fmax(x1, x[i]);
    y0 = fmin(y0, y[i]); y1 = fmax(y1, y[i]);
    double k;
    if (G.kap) {
      k = fabs(G.kap[i]);
    } else {
      const int a = (i + N - 1) % N, c = (i + 1) % N;
      const double cr = G.nx[a] * G.ny[c] - G.ny[a] * G.nx[c];
      const double dt = G.nx[a] * G.nx[c] + G.ny[a] * G.ny[c];
      k = fabs(atan2(cr, dt)) / (0.5 * G.w[a] + G.w[i] + 0.5 * G.w[c]);
    }
    km = fmax(km, k);
    ks += k;
    al += G.w[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    x0 = fmin(x0, __shfl_xor(x0, o, 64)); x1 = fmax(x1, __shfl_xor(x1, o, 64));
    y0 = fmin(y0, __shfl_xor(y0, o, 64)); y1 = fmax(y1, __shfl_xor(y1, o, 64));
    km = fmax(km, __shfl_xor(km, o, 64));
    ks += __shfl_xor(ks, o, 64);
    al += __shfl_xor(al, o, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = x0; red[1][wv] = x1; red[2][wv] = y0; red[3][wv] = y1;
    red[4][wv] = km; red[5][wv] = ks; red[6][wv] = al;
  }
  __syncthreads();
  x0 = red[0][0]; x1 = red[1][0]; y0 = red[2][0]; y1 = red[3][0];
  km = red[4][0]; ks = red[5][0]; al = red[6][0];
  for (int q = 1; q < NT / 64; ++q) {
    x0 = fmin(x0, red[0][q]); x1 = fmax(x1, red[1][q]);
    y0 = fmin(y0, red[2][q]); y1 = fmax(y1, red[3][q]);
    km = fmax(km, red[4][q]); ks += red[5][q]; al += red[6][q];
  }
  const double cx = 0.5 * (x0 + x1), cy = 0.5 * (y0 + y1);
  double r = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += NT) r = fmax(r, sqrt((x[i] - cx) * (x[i] - cx) + (y[i] - cy) * (y[i] - cy)));
  for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[0][wv] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < NT / 64; ++q) r = fmax(r, red[0][q]);
    double* o = out + (size_t)BOX_OUT * b;
    o[0] = cx; o[1] = cy; o[2] = r;
    o[3] = x0; o[4] = x1; o[5] = y0; o[6] = y1;
    o[7] = km;
    o[8] = ks / (double)max(1, i1 - i0);
    o[9] = al;
  }
}

// identity blocks: dst[r + c ldd] = (r == c) for r < nr, c < nc
__global__ __launch_bounds__(NT) void k_eye(const CopyDesc* __restrict__ descs) {
  const CopyDesc d = descs[blockIdx.y];
  const int total = d.nr * d.nc;
  for (int e = blockIdx.x * NT + threadIdx.x; e < total; e += gridDim.x * NT) {
    const int r = e % d.nr, c = e / d.nr;
    d.dst[r + (size_t)c * d.ldd] = mkc(r == c ? 1.0 : 0.0, 0.0);
  }
}

__global__ void k_gather_idx(const int* __restrict__ src, const int* __restrict__ idx, int* __restrict__ dst, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) dst[e] = src[idx[e]];
}

// ---------------------------------------------------------------- blocked Gauss-Jordan
constexpr int GJ_NB = 32;

// Sweep the pivots of panel columns [c0, c0+nb) within the panel (one workgroup of 1024 threads
// per matrix).  Per pivot: arg-max search, then the pivot-row swap and scaling (one thread per
// panel column), then the elimination with one thread per row (each thread reads its own
// multiplier before overwriting column p, so no barrier is needed between the two).
constexpr int NTP = 1024;
template <class R>
__global__ __launch_bounds__(NTP) void k_gj_panel(const InvDescT<R>* __restrict__ descs, int c0, int* __restrict__ ipiv_all,
                                                  int maxn, int* __restrict__ info) {
  typedef typename cx<R>::T C_t;
  const InvDescT<R> d = descs[blockIdx.x];
  const int n = d.n;
  if (c0 >= n) return;
  const int c1 = min(c0 + GJ_NB, n);
  const int ld = d.ld;
  C_t* A = d.a;
  int* ipiv = ipiv_all + (size_t)blockIdx.x * maxn;
  __shared__ double red_v[NTP / 64];
  __shared__ int red_i[NTP / 64];
  __shared__ C_t rowp[GJ_NB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int p = c0; p < c1; ++p) {
    double bv = -1.0;
    int bi = n;
    for (int i = p + tid; i < n; i += NTP) {
      const double a = (double)cabs2(A[i + (size_t)p * ld]);
      if (a > bv || (a == bv && i < bi)) { bv = a; bi = i; }
    }
    wave_argmax(bv, bi);
    if (lane == 0) { red_v[wv] = bv; red_i[wv] = bi; }
    __syncthreads();
    double b = red_v[0];
    int r = red_i[0];
    for (int q = 1; q < NTP / 64; ++q)
      if (red_v[q] > b || (red_v[q] == b && red_i[q] < r)) { b = red_v[q]; r = red_i[q]; }
    if (!(b > 0.0)) r = p;
    const C_t piv = A[r + (size_t)p * ld];
    const C_t dd = (cabs2(piv) > 0) ? cinv(piv) : cx<R>::make(0.0, 0.0);
    __syncthreads();  // every thread has read the pivot before rows p, r change
    if (tid == 0) {
      ipiv[p] = r;
      if (!(b > 0.0)) info[blockIdx.x] = p + 1;
    }
    // swap rows p, r in the panel and scale the new pivot row
    for (int j = c0 + tid; j < c1; j += NTP) {
      const C_t vr = A[r + (size_t)j * ld];
      const C_t vp = A[p + (size_t)j * ld];
      const C_t sc = (j == p) ? dd : cmul(vr, dd);
      rowp[j - c0] = sc;
      A[p + (size_t)j * ld] = sc;
      if (r != p) A[r + (size_t)j * ld] = vp;
    }
    __syncthreads();
    // eliminate column p from every other row; column p becomes the inverse's column
    for (int i = tid; i < n; i += NTP) {
      if (i == p) continue;
      const C_t f = A[i + (size_t)p * ld];
      for (int j = c0; j < c1; ++j) {
        if (j == p) continue;
        A[i + (size_t)j * ld] = csub(A[i + (size_t)j * ld], cmul(f, rowp[j - c0]));
      }
      A[i + (size_t)p * ld] = cmul(cx<R>::make(-f.x, -f.y), dd);
    }
    __syncthreads();
  }
}

// Register-resident variant for n <= 1024: thread i holds row i of the NBR-column panel, and a
// pivot step costs one barrier and two LDS reads per wavefront.  Before it, every wavefront publishes its best candidate (a key
// holding |a|^2 with the row index in its low 11 bits, so one 64-bit max finds the pivot, ties
// going to the smaller row) together with that candidate's whole row, and the thread of row p
// publishes row p; after it, every thread picks the winning wavefront and reads the pivot row
// from LDS.  The LDS slots alternate between two buffers from step to step: a wavefront can be
// at most one step ahead of another.  Dropping the 11 low mantissa bits of |a|^2 only lets
// candidates within a relative 2^-41 of each other count as equal.
// The workgroup has as many whole wavefronts as the largest matrix of the batch has rows.
// The pivot steps are instantiated per column (template recursion) so that every access to
// the row array has a constant index and the row stays in registers.
constexpr int GJ_NBR = 16;
constexpr int NTP_REG = 1024;

template <class R>
struct GjShared {
  unsigned long long key[2][NTP_REG / 64];
  typename cx<R>::T cand[2][NTP_REG / 64][GJ_NBR];  // each wavefront's candidate pivot row
  typename cx<R>::T rowo[2][GJ_NBR];                 // row p before the step
};

// 1/x from the hardware reciprocal refined by Newton steps (r <- r + r (1 - x r)); x normal
__device__ __forceinline__ double gj_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float gj_rcp(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// 1/a for the pivot, scaled against overflow as in cinv (the inverse is on the dependent chain of
// every pivot step, so it takes reciprocals refined by Newton steps instead of divisions; the
// scaled modulus lies in [1, 2]); 0 for a = 0.  Pivots of extreme scale take the divisions.
template <class R>
__device__ __forceinline__ typename cx<R>::T gj_recip(typename cx<R>::T a) {
  const R sc = fmax(fabs(a.x), fabs(a.y));
  if (!(sc > 0)) return cx<R>::make(0.0, 0.0);
  constexpr R lo = sizeof(R) == 8 ? R(1e-300) : R(1e-35), hi = sizeof(R) == 8 ? R(1e300) : R(1e35);
  if (sc < lo || sc > hi) {
    const R is = R(1) / sc;
    const R ar = a.x * is, ai = a.y * is;
    const R q = is / (ar * ar + ai * ai);
    return cx<R>::make(ar * q, -ai * q);
  }
  const R is = gj_rcp(sc);
  const R ar = a.x * is, ai = a.y * is;
  const R q = is * gj_rcp(ar * ar + ai * ai);
  return cx<R>::make(ar * q, -ai * q);
}

template <class R, int JJ>
__device__ __forceinline__ void gj_pivot_steps(typename cx<R>::T (&a)[GJ_NBR], GjShared<R>& sh, int c0, int w, int n,
                                               int* __restrict__ ipiv, int* __restrict__ info_m) {
  typedef typename cx<R>::T C_t;
  if (JJ < w) {
    constexpr int buf = JJ & 1;
    const int i = threadIdx.x, lane = i & 63, wv = i >> 6;
    const C_t zero = cx<R>::make(0.0, 0.0);
    const int p = c0 + JJ;
    unsigned long long key = 0;
    if (i >= p && i < n) {
      const double v = (double)cabs2(a[JJ]);
      key = ((unsigned long long)__double_as_longlong(v) & ~0x7FFull) | (unsigned long long)(0x7FF - i);
    }
    const unsigned long long wk = wave_umax64(key);
    if (wk != 0 && key == wk) {
#pragma unroll
      for (int j = 0; j < GJ_NBR; ++j) sh.cand[buf][wv][j] = a[j];
    }
    if (lane == 0) sh.key[buf][wv] = wk;
    if (i == p) {
#pragma unroll
      for (int j = 0; j < GJ_NBR; ++j) sh.rowo[buf][j] = a[j];
    }
    __syncthreads();
    // the wavefronts' keys: one LDS read per lane and a wavefront max; the pivot row: one LDS read
    // by lanes 0..15 and lane broadcasts (wavefront-uniform values, no per-lane LDS traffic)
    const int nwv = blockDim.x >> 6;
    const unsigned long long best = wave_umax64(lane < nwv ? sh.key[buf][lane] : 0ull);
    const bool ok = (best >> 11) != 0;  // a nonzero pivot exists
    const int r = ok ? 0x7FF - (int)(best & 0x7FF) : p;
    const C_t* prow = ok ? sh.cand[buf][r >> 6] : sh.rowo[buf];
    if (i == 0) {
      ipiv[p] = r;
      if (!ok) *info_m = p + 1;
    }
    const C_t pl = lane < GJ_NBR ? prow[lane] : zero;
    C_t pr[GJ_NBR];
#pragma unroll
    for (int j = 0; j < GJ_NBR; ++j) pr[j] = lane_bcast(pl, j);
    const C_t dd = gj_recip<R>(pr[JJ]);
    if (i == p) {
#pragma unroll
      for (int j = 0; j < GJ_NBR; ++j) a[j] = (j == JJ) ? dd : cmul(pr[j], dd);
    } else if (i < n) {
      if (i == r) {
#pragma unroll
        for (int j = 0; j < GJ_NBR; ++j) a[j] = sh.rowo[buf][j];
      }
      const C_t fd = cmul(a[JJ], dd);
      const C_t nfd = cx<R>::make(-fd.x, -fd.y);
#pragma unroll
      for (int j = 0; j < GJ_NBR; ++j)
        if (j != JJ) a[j] = cfma(nfd, pr[j], a[j]);  // four FMAs per entry
      a[JJ] = nfd;
    }
    if constexpr (JJ + 1 < GJ_NBR) gj_pivot_steps<R, JJ + 1>(a, sh, c0, w, n, ipiv, info_m);
  }
}

// Applies panel [cp, cp + wp) of the register Gauss-Jordan inversion to the 16-column strip at cs,
// for the calling thread's row i, into a[]: the panel's row interchanges as one gather
// (sigma(i) = s_1(s_2(... s_wp(i))) for the interchanges s_t in the order they were made), then
// strip = mask(strip) + A[:, panel] T with T the interchanged strip's pivot rows cp.. and mask
// zeroing those rows.  The whole workgroup calls it (two barriers); one workgroup owns the strip.
template <class R>
__device__ __forceinline__ void gj_strip_update(const InvDescT<R>& d, int n, int cp, int cs, int ws, const int* __restrict__ ipiv,
                                                typename cx<R>::T (&a)[GJ_NBR], typename cx<R>::T (*T)[GJ_NBR], int* sp) {
  typedef typename cx<R>::T C_t;
  const int i = threadIdx.x;
  const int wp = min(GJ_NBR, n - cp);
  const int ld = d.ld;
  if (i < wp) sp[i] = ipiv[cp + i];
  __syncthreads();
  int src = i;
  for (int t = wp - 1; t >= 0; --t) {
    const int p = cp + t, r = sp[t];
    src = (src == p) ? r : (src == r ? p : src);
  }
#pragma unroll
  for (int j = 0; j < GJ_NBR; ++j) a[j] = (i < n && j < ws) ? d.a[src + (size_t)(cs + j) * ld] : cx<R>::make(0.0, 0.0);
  if (i >= cp && i < cp + wp) {
#pragma unroll
    for (int j = 0; j < GJ_NBR; ++j) {
      T[i - cp][j] = a[j];
      a[j] = cx<R>::make(0.0, 0.0);
    }
  }
  // the strip is permuted in place: every gather load has landed before any row is stored
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (i < n) {
    for (int q = 0; q < wp; ++q) {
      const C_t f = d.a[i + (size_t)(cp + q) * ld];
#pragma unroll
      for (int j = 0; j < GJ_NBR; ++j) a[j] = cfma(f, T[q][j], a[j]);
    }
  }
}

// One step of the register Gauss-Jordan inversion with look-ahead: workgroup x = 0 brings the
// strip of panel c0 up to date with panel cp and factors it in registers; workgroups x >= 1 each
// apply panel cp to one other 16-column strip (all of its rows).  Launched for c0 = 0, 16, ...
// up to and including the first c0 >= n (then only the updates run); cp = c0 - 16.
template <class R>
__global__ __launch_bounds__(NTP_REG) void k_gj_step(const InvDescT<R>* __restrict__ descs, int cp, int c0, int* __restrict__ ipiv_all,
                                                     int maxn, int* __restrict__ info) {
  typedef typename cx<R>::T C_t;
  const InvDescT<R> d = descs[blockIdx.y];
  const int n = d.n;
  const bool panel = blockIdx.x == 0;
  const int cs = panel ? c0 : GJ_NBR * (int)(blockIdx.x - 1);
  if (cs >= n) return;
  if (!panel && (cp < 0 || cp >= n || cs == cp || cs == c0)) return;
  int* ipiv = ipiv_all + (size_t)blockIdx.y * maxn;
  __shared__ GjShared<R> sh;
  __shared__ C_t T[GJ_NBR][GJ_NBR];
  __shared__ int sp[GJ_NBR];
  const int i = threadIdx.x;
  const int ld = d.ld;
  const int ws = min(GJ_NBR, n - cs);
  C_t a[GJ_NBR];
  if (cp >= 0) {
    gj_strip_update<R>(d, n, cp, cs, ws, ipiv, a, T, sp);
  } else {
#pragma unroll
    for (int j = 0; j < GJ_NBR; ++j) a[j] = (i < n && j < ws) ? d.a[i + (size_t)(cs + j) * ld] : cx<R>::make(0.0, 0.0);
  }
  if (panel) gj_pivot_steps<R, 0>(a, sh, c0, ws, n, ipiv, info + blockIdx.y);
  if (i < n) {
#pragma unroll
    for (int j = 0; j < GJ_NBR; ++j)
      if (j < ws) d.a[i + (size_t)(cs + j) * ld] = a[j];
  }
}

// For columns outside the panel: apply the panel's row swaps, save the pivot rows to T.
template <class R, int NB>
__global__ __launch_bounds__(NT) void k_gj_swapsave(const InvDescT<R>* __restrict__ descs, int c0, const int* __restrict__ ipiv_all,
                                                    int maxn, typename cx<R>::T* __restrict__ tbuf) {
  typedef typename cx<R>::T C_t;
  const InvDescT<R> d = descs[blockIdx.y];
  const int n = d.n;
  if (c0 >= n) return;
  const int c1 = min(c0 + NB, n);
  const int ld = d.ld;
  const int* ipiv = ipiv_all + (size_t)blockIdx.y * maxn;
  C_t* T = tbuf + (size_t)blockIdx.y * NB * maxn;
  for (int j = blockIdx.x * NT + threadIdx.x; j < n; j += gridDim.x * NT) {
    if (j >= c0 && j < c1) continue;
    C_t* col = d.a + (size_t)j * ld;
    for (int p = c0; p < c1; ++p) {
      const int r = ipiv[p];
      if (r != p) { C_t t = col[p]; col[p] = col[r]; col[r] = t; }
    }
    for (int p = c0; p < c1; ++p) T[(p - c0) + (size_t)j * NB] = col[p];
  }
}

// A[:, j] = mask(A[:, j]) + A[:, c0:c1] T[:, j]  for j outside the panel (mask zeroes rows c0:c1).
template <class R, int NB>
__global__ __launch_bounds__(NT) void k_gj_update(const InvDescT<R>* __restrict__ descs, int c0, int maxn,
                                                  const typename cx<R>::T* __restrict__ tbuf) {
  typedef typename cx<R>::T C_t;
  const InvDescT<R> d = descs[blockIdx.z];
  const int n = d.n;
  if (c0 >= n) return;
  const int c1 = min(c0 + NB, n);
  const int w = c1 - c0;
  const int ld = d.ld;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 16;
  if (i0 >= n || j0 >= n) return;
  const C_t* T = tbuf + (size_t)blockIdx.z * NB * maxn;
  __shared__ C_t Ap[NB][65];
  __shared__ C_t Ts[NB][17];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * NB; e += NT) {
    const int ii = e % 64, pp = e / 64;
    const int i = i0 + ii;
    Ap[pp][ii] = (i < n && pp < w) ? d.a[i + (size_t)(c0 + pp) * ld] : cx<R>::make(0, 0);
  }
  for (int e = tid; e < 16 * NB; e += NT) {
    const int pp = e % NB, jj = e / NB;
    const int j = j0 + jj;
    Ts[pp][jj] = (j < n && pp < w) ? T[pp + (size_t)j * NB] : cx<R>::make(0, 0);
  }
  __syncthreads();
  const int ii = tid % 64, jb = tid / 64;  // 4 column groups of 4
  const int i = i0 + ii;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int jj = jb * 4 + c;
    const int j = j0 + jj;
    if (j >= n || (j >= c0 && j < c1)) continue;
    C_t acc = (i >= c0 && i < c1) ? cx<R>::make(0, 0) : d.a[i + (size_t)j * ld];
    for (int pp = 0; pp < w; ++pp) acc = cfma(Ap[pp][ii], Ts[pp][jj], acc);
    d.a[i + (size_t)j * ld] = acc;
  }
}

// undo the row interchanges on the columns of the inverse: for p = n-1..0 swap columns p, ipiv[p]
template <class R>
__global__ __launch_bounds__(NT) void k_gj_colperm(const InvDescT<R>* __restrict__ descs, const int* __restrict__ ipiv_all, int maxn) {
  typedef typename cx<R>::T C_t;
  const InvDescT<R> d = descs[blockIdx.y];
  const int n = d.n;
  const int* ipiv = ipiv_all + (size_t)blockIdx.y * maxn;
  for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
    for (int p = n - 1; p >= 0; --p) {
      const int r = ipiv[p];
      if (r != p) {
        C_t t = d.a[i + (size_t)p * d.ld];
        d.a[i + (size_t)p * d.ld] = d.a[i + (size_t)r * d.ld];
        d.a[i + (size_t)r * d.ld] = t;
      }
    }
  }
}

// out[r + c*ld] = K(y_rows[r], y_c + shift e_1, n_c) w_c for every node c: rows of the plain
// trapezoid discretization of D - i omega S from a translated copy of the curve (Sec. 2.4, A_j).
// Transmission problem: rows and columns are unknowns (2N columns) and the entries those of the
// exterior field alone.
__global__ __launch_bounds__(NT) void k_eval_shift(Geo G, const int* __restrict__ rows, int nr, double shift,
                                                   cplx* __restrict__ out, int ld) {
  const int64_t total = (int64_t)nr * G.N * (G.two ? 2 : 1);
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int r = (int)(e % nr);
    const int c = (int)(e / nr);
    const int gr = rows[r];
    if (G.two) {
      out[r + (size_t)c * ld] = a_ext_tr(G, gr, c, 0.0, shift);
      continue;
    }
    const cplx K = helm_kernel(G.omega, G.x[gr] - (G.x[c] + shift), G.y[gr] - G.y[c], G.nx[c], G.ny[c]);
    out[r + (size_t)c * ld] = cscale(K, G.w[c]);
  }
}

__global__ void k_hankel(const double* __restrict__ x, int64_t n, cplx* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    cplx h0, h1;
    hankel01(x[e], h0, h1);
    out[e] = h0;
    out[n + e] = h1;
  }
}

// Kernel table of the Alpert correction, one thread per (node i, off-grid node q): the position at
// t_i + u_q h is the Lagrange interpolant of the node positions (weights G.alpL, offsets G.alpo[q] ..),
// its parameter derivative that of the interpolant (weights D, divided by h), whence the speed |z'|,
// the outward normal (z2', -z1') / |z'| and the quadrature weight h |z'|:
//   alpT[i + q N] = wq[q] K(y_i, z, n) h |z'|.
__global__ __launch_bounds__(NT) void k_alpert_table(Geo G, const double* __restrict__ D, const double* __restrict__ wq,
                                                     cplx* __restrict__ T) {
  const int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x;
  const int N = G.N;
  if (e >= (int64_t)N * G.alpn) return;
  const int i = (int)(e % N);
  const int q = (int)(e / N);
  const double h = 2.0 * QPS_PI / N;
  double zx = 0, zy = 0, dx = 0, dy = 0;
  for (int r = 0; r < G.alpnl; ++r) {
    int k = i + G.alpo[q] + r;
    k = ((k % N) + N) % N;
    const double L = G.alpL[q * G.alpnl + r], Dr = D[q * G.alpnl + r];
    zx += L * G.x[k];
    zy += L * G.y[k];
    dx += Dr * G.x[k];
    dy += Dr * G.y[k];
  }
  dx /= h;
  dy /= h;
  const double sp = sqrt(dx * dx + dy * dy);
  const cplx K = helm_kernel(G.omega, G.x[i] - zx, G.y[i] - zy, dy / sp, -dx / sp);
  T[i + (size_t)q * N] = cscale(K, wq[q] * h * sp);
}

__global__ void k_entries(Geo G, const int* __restrict__ rows, const int* __restrict__ cols, int64_t n, cplx* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT)
    out[e] = a_entry_any(G, rows[e], cols[e]);
}

inline int grid_for(int64_t elems, int cap = 4096) {
  int64_t g = (elems + NT - 1) / NT;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

namespace qps {

hipError_t launch_eval_blocks(const Geo& g, const BlockDesc* d, int nd, int max_elems, hipStream_t s) {
  if (nd == 0 || max_elems == 0) return hipSuccess;
  dim3 grid(grid_for(max_elems, 1 << 30), nd);  // every entry its own thread
  if (g.two)
    hipLaunchKernelGGL(k_eval_blocks<true>, grid, dim3(NT), 0, s, g, d);
  else
    hipLaunchKernelGGL(k_eval_blocks<false>, grid, dim3(NT), 0, s, g, d);
  return hipGetLastError();
}
hipError_t launch_proxy(const Geo& g, const ProxyDesc* d, int nd, int max_elems, hipStream_t s) {
  if (nd == 0 || max_elems == 0) return hipSuccess;
  dim3 grid(grid_for(max_elems, 1 << 30), nd);  // every entry its own thread
  if (g.two)
    hipLaunchKernelGGL(k_proxy_tr, grid, dim3(NT), 0, s, g, d);
  else
    hipLaunchKernelGGL(k_proxy, grid, dim3(NT), 0, s, g, d);
  return hipGetLastError();
}
hipError_t launch_sketch(const SketchDesc* d, int nd, int max_s, int max_n, uint64_t seed, hipStream_t s) {
  if (nd == 0) return hipSuccess;
  dim3 grid((max_s + 31) / 32, (max_n + 31) / 32, nd);
  hipLaunchKernelGGL(k_sketch, grid, dim3(NT), 0, s, d, seed);
  return hipGetLastError();
}
hipError_t launch_cpqr(const CpqrDesc* d, int nd, int max_s, int max_n, double tol, int* k_out, hipStream_t s, DevBuf* ws, int* launches) {
  if (nd == 0) return hipSuccess;
  // a few large boxes: one launch per pivot step over workgroups of 16 columns.  A launch costs
  // about as much as a pivot step of the one-workgroup kernel on a 200 x 200 sketch, whose steps
  // grow with s n (the trailing matrix through one CU): the launches pay from there on.
  if (ws && nd <= 16 && max_s <= CPQRM_MAXS && max_n <= CPQR_MAXN && max_s >= 1 && max_n >= 2 &&
      (int64_t)max_s * max_n >= 40000) {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t ni = (size_t)nd * max_n;
    const int64_t zs = (int64_t)max_s * max_n;
    const size_t bst = al(sizeof(CpqrmState) * nd), bi = al(sizeof(int) * ni), bd = al(sizeof(double) * ni),
                 bc = al(sizeof(cplx) * ni), bw = al(sizeof(cplx) * (size_t)nd * zs);
    hipError_t e = ws->reserve(bst + 3 * bi + 2 * bd + bc + bw);
    if (e != hipSuccess) return e;
    char* base = ws->as<char>();
    CpqrmWs W;
    W.st = (CpqrmState*)base;
    W.pcA = (int*)(base + bst);
    W.pcB = (int*)(base + bst + bi);
    W.fin = (int*)(base + bst + 2 * bi);
    W.cnA = (double*)(base + bst + 3 * bi);
    W.cnB = (double*)(base + bst + 3 * bi + bd);
    W.alph = (cplx*)(base + bst + 3 * bi + 2 * bd);
    W.W2 = (cplx*)(base + bst + 3 * bi + 2 * bd + bc);
    W.maxn = max_n;
    W.zstride = zs;
    const int ncg = (max_n + 15) / 16;
    hipLaunchKernelGGL(k_cpqrm_init, dim3(ncg, nd), dim3(256), 0, s, d, W);
    const int pmax = std::min(max_s, max_n);
    const int nwg = (max_n - 1 + 15) / 16;
    for (int p = 0; p < pmax; ++p) hipLaunchKernelGGL(k_cpqrm_step, dim3(nwg, nd), dim3(256), 0, s, d, W, p, tol);
    hipLaunchKernelGGL(k_cpqrm_gather, dim3(max_n, nd), dim3(256), 0, s, d, W, k_out);
    hipLaunchKernelGGL(k_cpqrm_tsolve, dim3(nd), dim3(1024), 0, s, d, W);
    if (launches) *launches = pmax + 3;
    return hipGetLastError();
  }
  if (launches) *launches = 1;
  if (nd >= 256 && max_s <= 512 && max_n <= 256)
    hipLaunchKernelGGL((k_cpqr<256, 512, 256, 8>), dim3(nd), dim3(256), 0, s, d, tol, k_out);
  else
    hipLaunchKernelGGL((k_cpqr<1024, CPQR_MAXS, CPQR_MAXN, 12>), dim3(nd), dim3(1024), 0, s, d, tol, k_out);
  return hipGetLastError();
}
hipError_t launch_buildP(const PDesc* d, int nd, int max_elems, hipStream_t s) {
  if (nd == 0 || max_elems == 0) return hipSuccess;
  dim3 grid(grid_for(max_elems, 256), nd);
  hipLaunchKernelGGL(k_buildP, grid, dim3(NT), 0, s, d);
  return hipGetLastError();
}
hipError_t launch_copy(const CopyDesc* d, int nd, int max_elems, hipStream_t s) {
  if (nd == 0 || max_elems == 0) return hipSuccess;
  dim3 grid(grid_for(max_elems, 256), nd);
  hipLaunchKernelGGL(k_copy, grid, dim3(NT), 0, s, d);
  return hipGetLastError();
}
hipError_t launch_eye(const CopyDesc* d, int nd, int max_elems, hipStream_t s) {
  if (nd == 0 || max_elems == 0) return hipSuccess;
  hipLaunchKernelGGL(k_eye, dim3(grid_for(max_elems, 256), nd), dim3(NT), 0, s, d);
  return hipGetLastError();
}
hipError_t launch_box_circles(const Geo& g, const int* lo, const int* hi, int nbox, double* out, hipStream_t s) {
  if (nbox == 0) return hipSuccess;
  hipLaunchKernelGGL(k_box_circles, dim3(nbox), dim3(NT), 0, s, g, lo, hi, out);
  return hipGetLastError();
}
hipError_t launch_gather_idx(const int* src, const int* idx, int* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_idx, dim3(grid_for(n)), dim3(NT), 0, s, src, idx, dst, n);
  return hipGetLastError();
}
template <class R>
hipError_t launch_inv(const InvDescT<R>* d, int nd, int max_n, typename cx<R>::T* tbuf, int* ipiv, int* info, hipStream_t s) {
  if (nd == 0 || max_n == 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(info, 0, sizeof(int) * nd, s);
  if (e != hipSuccess) return e;
  if (max_n <= NTP_REG) {
    // one thread per row, in whole wavefronts: small matrices get small workgroups; one launch per
    // panel (the previous panel's update runs beside the factorization)
    const int nthr = std::min(NTP_REG, (max_n + 63) / 64 * 64);
    const int np = (max_n + GJ_NBR - 1) / GJ_NBR;
    for (int k = 0; k <= np; ++k)
      hipLaunchKernelGGL(k_gj_step<R>, dim3(1 + np, nd), dim3(nthr), 0, s, d, GJ_NBR * (k - 1), GJ_NBR * k, ipiv, max_n, info);
  } else {
    for (int c0 = 0; c0 < max_n; c0 += GJ_NB) {
      hipLaunchKernelGGL(k_gj_panel<R>, dim3(nd), dim3(NTP), 0, s, d, c0, ipiv, max_n, info);
      hipLaunchKernelGGL((k_gj_swapsave<R, GJ_NB>), dim3(grid_for(max_n, 64), nd), dim3(NT), 0, s, d, c0, ipiv, max_n, tbuf);
      hipLaunchKernelGGL((k_gj_update<R, GJ_NB>), dim3((max_n + 63) / 64, (max_n + 15) / 16, nd), dim3(NT), 0, s, d, c0, max_n,
                         (const typename cx<R>::T*)tbuf);
    }
  }
  hipLaunchKernelGGL(k_gj_colperm<R>, dim3(grid_for(max_n, 64), nd), dim3(NT), 0, s, d, ipiv, max_n);
  return hipGetLastError();
}
template hipError_t launch_inv<double>(const InvDesc*, int, int, cplx*, int*, int*, hipStream_t);
template hipError_t launch_inv<float>(const InvDesc32*, int, int, cplxf*, int*, int*, hipStream_t);
hipError_t launch_eval_shift(const Geo& g, const int* rows, int nr, double shift, cplx* out, int ld, hipStream_t s) {
  if (nr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval_shift, dim3(grid_for((int64_t)nr * g.N * (g.two ? 2 : 1), 8192)), dim3(NT), 0, s, g, rows, nr,
                     shift, out, ld);
  return hipGetLastError();
}
hipError_t launch_hankel(const double* x, int64_t n, cplx* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hankel, dim3(grid_for(n)), dim3(NT), 0, s, x, n, out);
  return hipGetLastError();
}
hipError_t launch_alpert_table(const Geo& g, const double* D, const double* wq, cplx* T, hipStream_t s) {
  const int64_t n = (int64_t)g.N * g.alpn;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_alpert_table, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, g, D, wq, T);
  return hipGetLastError();
}
hipError_t launch_entries(const Geo& g, const int* rows, const int* cols, int64_t n, cplx* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_entries, dim3(grid_for(n)), dim3(NT), 0, s, g, rows, cols, n, out);
  return hipGetLastError();
}

}  // namespace qps
