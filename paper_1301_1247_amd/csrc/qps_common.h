// Shared device/host helpers of the HIP library: complex arithmetic on double2,
// error plumbing, wavefront reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

typedef double2 cplx;

__host__ __device__ inline cplx mkc(double re, double im) { cplx c; c.x = re; c.y = im; return c; }
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return mkc(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return mkc(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplx cmul(cplx a, cplx b) { return mkc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline cplx cscale(cplx a, double s) { return mkc(a.x * s, a.y * s); }
__host__ __device__ inline cplx cconj(cplx a) { return mkc(a.x, -a.y); }
__host__ __device__ inline double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }
// a * conj(b)
__host__ __device__ inline cplx cmulc(cplx a, cplx b) { return mkc(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }
// acc + a*b
__host__ __device__ inline cplx cfma(cplx a, cplx b, cplx acc) {
  return mkc(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
__host__ __device__ inline cplx cinv(cplx a) {
  // 1/a with scaling to avoid overflow for |a| large or small
  double s = fmax(fabs(a.x), fabs(a.y));
  double ar = a.x / s, ai = a.y / s;
  double d = ar * ar + ai * ai;
  return mkc(ar / (d * s), -ai / (d * s));
}
// XCD-aware work order: the dispatcher hands the workgroups of a launch to the 8 XCDs of an MI355X
// round-robin in launch order, and each XCD has its own L2.  Workgroup L (linear, x fastest) of a
// launch of `total` takes item T of an order in which every XCD owns one contiguous range of items,
// so neighbouring items (tiles of one matrix, which share its operand panels) meet in one L2.
constexpr int QPS_NXCD = 8;
__device__ inline int xcd_item(int L, int total) {
  if (total < 2 * QPS_NXCD) return L;
  const int xcd = L % QPS_NXCD, slot = L / QPS_NXCD;
  const int q = total / QPS_NXCD, r = total % QPS_NXCD;
  return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

__device__ inline cplx cexpi(double t) {
  double s, c;
  sincos(t, &s, &c);
  return mkc(c, s);
}
// exp(z) for complex z
__device__ inline cplx cexp(cplx z) {
  double e = exp(z.x);
  double s, c;
  sincos(z.y, &s, &c);
  return mkc(e * c, e * s);
}

// single-precision complex (complex64) helpers
typedef float2 cplxf;
__host__ __device__ inline cplxf mkcf(float re, float im) { cplxf c; c.x = re; c.y = im; return c; }
__host__ __device__ inline cplxf cadd(cplxf a, cplxf b) { return mkcf(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplxf csub(cplxf a, cplxf b) { return mkcf(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplxf cmul(cplxf a, cplxf b) { return mkcf(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline float cabs2(cplxf a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline cplxf cinv(cplxf a) {
  float s = fmaxf(fabsf(a.x), fabsf(a.y));
  float ar = a.x / s, ai = a.y / s;
  float d = ar * ar + ai * ai;
  return mkcf(ar / (d * s), -ai / (d * s));
}
__host__ __device__ inline cplxf cfma(cplxf a, cplxf b, cplxf acc) {
  return mkcf(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}

// precision traits: complex type and constructor for double / float
template <class R> struct cx;
template <> struct cx<double> {
  typedef double2 T;
  __host__ __device__ static T make(double re, double im) { return mkc(re, im); }
};
template <> struct cx<float> {
  typedef float2 T;
  __host__ __device__ static T make(double re, double im) { return mkcf((float)re, (float)im); }
};

// wavefront (64 lanes) reductions with DPP moves; every lane must be active, every lane gets the
// result.  A DPP move of a double moves its two 32-bit halves; lanes a row mask leaves out take
// the move's old value 0, so the partial sums of rows 0 and 2 are not counted twice.
template <int CTRL, int ROWS>
__device__ inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double wave_sum(double v) {
  v += dpp_d<0xB1, 0xF>(v);   // quad_perm 1,0,3,2
  v += dpp_d<0x4E, 0xF>(v);   // quad_perm 2,3,0,1
  v += dpp_d<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_d<0x140, 0xF>(v);  // row_mirror
  v += dpp_d<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_d<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline cplx wave_csum(cplx v) { return mkc(wave_sum(v.x), wave_sum(v.y)); }
// sum over each 16-lane row of the wavefront (every lane of the row gets its row's sum)
__device__ inline double row16_sum(double v) {
  v += dpp_d<0xB1, 0xF>(v);
  v += dpp_d<0x4E, 0xF>(v);
  v += dpp_d<0x141, 0xF>(v);
  v += dpp_d<0x140, 0xF>(v);
  return v;
}
__device__ inline cplx row16_csum(cplx v) { return mkc(row16_sum(v.x), row16_sum(v.y)); }
// Wavefront max / min of an unsigned value with DPP moves (quad swaps, half-row and row
// mirrors, row broadcasts 15 and 31), result read from lane 63: no LDS round trips.
__device__ inline unsigned wave_umax(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ inline unsigned wave_umin(unsigned v) {
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false));
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false));
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));
  v = min(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Wavefront max of a 64-bit unsigned key: each DPP stage moves both halves, lanes outside the row
// mask keep their own key.  Every lane receives the result (from lane 63).
template <int CTRL, int ROWS>
__device__ inline unsigned long long dpp_keep_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)v, (int)(unsigned)v, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(v >> 32), (int)(unsigned)(v >> 32), CTRL, ROWS, 0xF, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ inline unsigned long long wave_umax64(unsigned long long v) {
  unsigned long long o;
  o = dpp_keep_u64<0xB1, 0xF>(v);  v = o > v ? o : v;  // quad_perm 1,0,3,2
  o = dpp_keep_u64<0x4E, 0xF>(v);  v = o > v ? o : v;  // quad_perm 2,3,0,1
  o = dpp_keep_u64<0x141, 0xF>(v); v = o > v ? o : v;  // row_half_mirror
  o = dpp_keep_u64<0x140, 0xF>(v); v = o > v ? o : v;  // row_mirror
  o = dpp_keep_u64<0x142, 0xA>(v); v = o > v ? o : v;  // row_bcast:15
  o = dpp_keep_u64<0x143, 0xC>(v); v = o > v ? o : v;  // row_bcast:31
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// the value of lane j of a wavefront, for every lane (the result is wavefront-uniform)
__device__ __forceinline__ cplx lane_bcast(cplx v, int j) {
  const long long bx = __double_as_longlong(v.x), by = __double_as_longlong(v.y);
  const int xl = __builtin_amdgcn_readlane((int)bx, j), xh = __builtin_amdgcn_readlane((int)(bx >> 32), j);
  const int yl = __builtin_amdgcn_readlane((int)by, j), yh = __builtin_amdgcn_readlane((int)(by >> 32), j);
  return mkc(__longlong_as_double(((long long)xh << 32) | (unsigned)xl),
             __longlong_as_double(((long long)yh << 32) | (unsigned)yl));
}
__device__ __forceinline__ cplxf lane_bcast(cplxf v, int j) {
  return mkcf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), j)),
              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), j)));
}

// arg-max of (val, idx) over a wavefront, ties resolved to the smaller index; values <= 0
// (including the -1 of lanes without a candidate) compare as 0.  The bit pattern of a
// non-negative double orders like the value, so the max is taken on its high then low word.
// Every lane receives the result.
__device__ inline void wave_argmax(double& val, int& idx) {
  const unsigned long long bits = val > 0.0 ? (unsigned long long)__double_as_longlong(val) : 0ull;
  const unsigned hi = (unsigned)(bits >> 32), lo = (unsigned)bits;
  const unsigned mh = wave_umax(hi);
  const unsigned ml = wave_umax(hi == mh ? lo : 0u);
  const unsigned mi = wave_umin((hi == mh && lo == ml) ? (unsigned)idx : 0xFFFFFFFFu);
  val = __longlong_as_double((long long)(((unsigned long long)mh << 32) | ml));
  idx = (int)mi;
}

// host-side status plumbing
namespace qps {
void set_error(const std::string& msg);
}

#define QPS_HIP_CHECK(expr)                                                              \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) {                                                              \
      qps::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));                 \
      return HBS_E_DEVICE;                                                               \
    }                                                                                    \
  } while (0)
