// Device helpers shared by the HIP kernels of libgmps: complex arithmetic, stochastic
// rounding, lane-group butterfly sums, refined reciprocals, LDS ordering and the
// reflection's site blocks.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/gmps.h"
#include "gmps_internal.h"

namespace gmps {

// ----------------------------------------------------------------------------- complex
template <class T>
struct cx {
  T re, im;
};
using cd = cx<double>;

template <class T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <class T>
__device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
// acc + a * b
template <class T>
__device__ __forceinline__ cx<T> cfma(cx<T> acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// conj(a) * b
template <class T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// a / b (b not near the underflow threshold: |b|^2 is formed directly)
template <class T>
__device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  const T d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
template <class S>
__device__ __forceinline__ cx<S> down(cd a) { return {(S)a.re, (S)a.im}; }
template <class S>
__device__ __forceinline__ cd up(cx<S> a) { return {(double)a.re, (double)a.im}; }
template <class S>
__device__ __forceinline__ cx<S> czero() { return {(S)0, (S)0}; }
// conversion between complex types (the identity when T == U)
template <class T, class U>
__device__ __forceinline__ cx<T> cvt(cx<U> a) { return {(T)a.re, (T)a.im}; }

// ---------------------------------------------------------------------- stochastic rounding
// Unbiased (stochastic) rounding of a double to float: 29 random bits are added to the low
// 29 bits of the magnitude, which a float does not keep, and those bits are then cut, so x
// rounds up with probability equal to its distance from the lower neighbour over the gap
// (E[round(x)] = x). The float conversion of the truncated value is exact. Random bits come
// from the high bits of a 64-bit linear congruential stream (Knuth's MMIX constants).
__device__ __forceinline__ uint32_t rng29(uint64_t& st) {
  st = st * 6364136223846793005ull + 1442695040888963407ull;
  return (uint32_t)(st >> 35);
}
__device__ __forceinline__ float sround_f32(double x, uint32_t r29) {
  uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint64_t sign = b & 0x8000000000000000ull;
  uint64_t mag = (b & 0x7FFFFFFFFFFFFFFFull) + (uint64_t)r29;
  mag &= ~((1ull << 29) - 1ull);
  return (float)__longlong_as_double((long long)(sign | mag));
}
// An FP32 result (all-FP32 path) is stored as it is.
template <class S>
__device__ __forceinline__ cx<S> store_cast(cx<float> a, uint64_t&, bool) { return {(S)a.re, (S)a.im}; }
// Conversion of an FP64 result to the storage type S.
template <class S>
__device__ __forceinline__ cx<S> store_cast(cd a, uint64_t& st, bool sr) {
  if constexpr (sizeof(S) == sizeof(double)) {
    return {(S)a.re, (S)a.im};
  } else {
    if (!sr) return {(S)a.re, (S)a.im};
    const float re = sround_f32(a.re, rng29(st));
    const float im = sround_f32(a.im, rng29(st));
    return {re, im};
  }
}
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ------------------------------------------------------------------------ group collectives
// Butterfly sums inside a lane group of G = 2, 4, 8, 16 or 32 lanes. Steps 1 and 2 swap
// neighbours inside a quad (DPP quad_perm); once values are quad-uniform the half-row
// mirror pairs the two quads of an 8-lane half, once they are half-row uniform the row
// mirror pairs the two halves of a 16-lane row, and a swizzle swaps 16-lane halves of a
// 32-lane group. Each step adds a value to its partner's, so every lane of the group ends
// with the same bits (addition is commutative), and branches on the sums are uniform.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double swap16_f64(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_ds_swizzle(lo, 0x401F);  // bit-mask mode: xor lane id with 16
  hi = __builtin_amdgcn_ds_swizzle(hi, 0x401F);
  return __hiloint2double(hi, lo);
}
template <int G>
__device__ __forceinline__ double gsum(double v) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16 || G == 32, "group size");
  v += dpp_f64<0xB1>(v);                   // quad_perm [1,0,3,2]
  if (G > 2) v += dpp_f64<0x4E>(v);        // quad_perm [2,3,0,1]
  if (G > 4) v += dpp_f64<0x141>(v);       // row_half_mirror
  if (G > 8) v += dpp_f64<0x140>(v);       // row_mirror
  if (G > 16) v += swap16_f64(v);
  return v;
}
template <int G>
__device__ __forceinline__ cd gsum(cd v) { return {gsum<G>(v.re), gsum<G>(v.im)}; }
// the same butterfly on FP32 values (all-FP32 path)
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int G>
__device__ __forceinline__ float gsum(float v) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16 || G == 32, "group size");
  v += dpp_f32<0xB1>(v);
  if (G > 2) v += dpp_f32<0x4E>(v);
  if (G > 4) v += dpp_f32<0x141>(v);
  if (G > 8) v += dpp_f32<0x140>(v);
  if (G > 16) v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
  return v;
}
template <int G>
__device__ __forceinline__ cx<float> gsum(cx<float> v) { return {gsum<G>(v.re), gsum<G>(v.im)}; }
// value held by group lane src, delivered to every lane of the group
template <int G>
__device__ __forceinline__ cd gbcast(cd v, int gl, int src) {
  return gsum<G>(gl == src ? v : cd{0.0, 0.0});
}
template <int G>
__device__ __forceinline__ cx<float> gbcast(cx<float> v, int gl, int src) {
  return gsum<G>(gl == src ? v : cx<float>{0.0f, 0.0f});
}

// Raw v_rsq_f64 / v_rcp_f64 are accurate to about 2^-23; two Newton steps bring them to
// working precision, which keeps Householder reflectors and Jacobi rotations unitary.
__device__ __forceinline__ double rsqrt_acc(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double r = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, r, y);
  r = fma(-x * y, y, 1.0);
  return fma(0.5 * y, r, y);
}
__device__ __forceinline__ double rcp_acc(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double r = fma(-x, y, 1.0);
  y = fma(y, r, y);
  r = fma(-x, y, 1.0);
  return fma(y, r, y);
}
// FP32 (all-FP32 path): v_rsq_f32 / v_rcp_f32 are within about 1 ulp; one Newton step
// each brings them to rounding of the working precision.
__device__ __forceinline__ float rsqrt_acc(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  return fmaf(0.5f * y, fmaf(-x * y, y, 1.0f), y);
}
__device__ __forceinline__ float rcp_acc(float x) {
  const float y = __builtin_amdgcn_rcpf(x);
  return fmaf(y, fmaf(-x, y, 1.0f), y);
}
// raw hardware estimates, for quantities that need only angle accuracy
__device__ __forceinline__ double rsq_raw(double x) { return __builtin_amdgcn_rsq(x); }
__device__ __forceinline__ float rsq_raw(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rcp_raw(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ float rcp_raw(float x) { return __builtin_amdgcn_rcpf(x); }

// Orders LDS traffic between the lanes of the (single-wave) workgroup without waiting
// for outstanding global memory operations.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Orders LDS traffic between the lanes of one wave (no barrier: for code that a wave runs
// while another wave of its workgroup runs different code).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Round-robin (circle method) pairing of NC columns: round r pairs NC-1 with r and
// (r+p) with (r-p) mod (NC-1); after NC-1 rounds every pair has met once.
__host__ __device__ constexpr int circ_a(int NC, int r, int p) { return p == 0 ? NC - 1 : (r + p) % (NC - 1); }
__host__ __device__ constexpr int circ_b(int NC, int r, int p) {
  return p == 0 ? r : (r - p + (NC - 1)) % (NC - 1);
}
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int cmax(int a, int b) { return a < b ? b : a; }

// (x, y) <- (c x - conj(se) y, se x + c y) for real c and complex se = s e^{i phi}.
template <class T>
__device__ __forceinline__ void rot2(cx<T>& x, cx<T>& y, T c, cx<T> se) {
  const cx<T> x0 = x, y0 = y;
  x.re = fma(c, x0.re, fma(-se.re, y0.re, -se.im * y0.im));
  x.im = fma(c, x0.im, fma(-se.re, y0.im, se.im * y0.re));
  y.re = fma(c, y0.re, fma(se.re, x0.re, -se.im * x0.im));
  y.im = fma(c, y0.im, fma(se.re, x0.im, se.im * x0.re));
}

template <class S>
__device__ __forceinline__ cx<S> sel(cx<S> a0, cx<S> a1, int s) {
  return {s ? a1.re : a0.re, s ? a1.im : a0.im};
}

// (P A)[s] for P = |xb><xb| (oracle) or |+><+| (diffusion), given A[0] = a0, A[1] = a1.
template <class S>
__device__ __forceinline__ cx<S> proj_apply(cx<S> a0, cx<S> a1, int s, bool diff, int xb) {
  if (diff) {
    const S h = (S)0.5;
    return {h * (a0.re + a1.re), h * (a0.im + a1.im)};
  }
  return s == xb ? sel(a0, a1, xb) : czero<S>();
}

constexpr double kInvSqrt2 = 0.70710678118654752440;  // |+> = (|0> + |1>) / sqrt(2)
constexpr double kJacobiTol2 = 1e-30;  // (relative off-diagonal 1e-15)^2


// The (CM, 2, CM) box of a site slot loaded by G cooperating lanes (element e = lane + t*G of
// the box, row-major; entries outside (chl, 2, chr) read as zero), then written to LDS.
template <class S, int CM, int G>
struct APrefetch {
  static constexpr int NE = (CM * 2 * CM + G - 1) / G;
  cx<S> v[NE];
  int chl_, chr_;
  // The loads are unconditional (element indices are clamped into the box, which lies
  // inside the slot) and the unused elements are masked only when the tile is staged: a
  // load under a branch, or a use of its value right away, would make the compiler wait
  // for the load there instead of one site later.
  __device__ __forceinline__ void load(const cx<S>* slot, int gl, int chl, int chr) {
    constexpr int D = 2 * CM;
    chl_ = chl;
    chr_ = chr;
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = gl + t * G;
      const int ec = e < CM * 2 * CM ? e : CM * 2 * CM - 1;
      const int a = ec / (2 * CM), s = (ec / CM) & 1, b = ec % CM;
      v[t] = slot[a * 2 * D + s * D + b];
    }
  }
  __device__ __forceinline__ void stage(cx<S>* lds_a, int gl) const {
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = gl + t * G;
      const int a = e / (2 * CM), b = e % CM;
      if (e < CM * 2 * CM) lds_a[e] = (a < chl_ && b < chr_) ? v[t] : czero<S>();
    }
  }
};

}  // namespace gmps
