// Host emulation of the HIP device environment used by the iterate kernels: every lane of a
// workgroup is an OS thread; cross-lane operations and barriers synchronise the lanes that
// take part in them (a quad, a half row, a row, 32 lanes, a wave or the workgroup). A lane
// group that does not arrive complete within the timeout is reported as divergent.
#pragma once
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <thread>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
// a block-scope __shared__ variable is one object for all lanes of the (single) workgroup; the
// build compiles copies of the kernel headers whose `extern __shared__` reads `extern`
#define __shared__ static
#define __align__(n) alignas(n)

struct emu_dim3 {
  unsigned x = 0, y = 0, z = 0;
};
extern thread_local emu_dim3 threadIdx;
extern thread_local emu_dim3 blockIdx;
extern emu_dim3 blockDim, gridDim;

typedef int hipError_t;
typedef void* hipStream_t;
constexpr int hipSuccess = 0;
constexpr int hipErrorInvalidValue = 1;
inline hipError_t hipGetLastError() { return 0; }

using std::fma;
using std::fmaf;
using std::fmin;
using std::fmax;
using std::fabs;
using std::sqrt;
using std::isfinite;
using std::min;
using std::max;

inline long long __double_as_longlong(double x) { long long r; std::memcpy(&r, &x, 8); return r; }
inline double __longlong_as_double(long long x) { double r; std::memcpy(&r, &x, 8); return r; }
inline int __double2loint(double x) { return (int)(uint32_t)((uint64_t)__double_as_longlong(x) & 0xFFFFFFFFull); }
inline int __double2hiint(double x) { return (int)(uint32_t)((uint64_t)__double_as_longlong(x) >> 32); }
inline double __hiloint2double(int hi, int lo) {
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo));
}
inline int __float_as_int(float x) { int r; std::memcpy(&r, &x, 4); return r; }
inline float __int_as_float(int x) { float r; std::memcpy(&r, &x, 4); return r; }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline unsigned __lane_id() { return threadIdx.x & 63u; }

namespace emu {
constexpr int kMaxThreads = 256;
// group barrier over the lanes [base, base + size) of the workgroup
void gsync(int base, int size, const char* what);
extern int32_t xch[kMaxThreads];
extern uint64_t bal[kMaxThreads / 64];
}  // namespace emu

inline double __builtin_amdgcn_rsq(double x) { return 1.0 / std::sqrt(x); }
inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }
inline float __builtin_amdgcn_rsqf(float x) { return 1.0f / std::sqrt(x); }
inline float __builtin_amdgcn_rcpf(float x) { return 1.0f / x; }
inline void __builtin_amdgcn_fence(int, const char*, const char* = nullptr) { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __builtin_amdgcn_s_barrier() { emu::gsync(0, (int)blockDim.x, "s_barrier"); }
inline void __builtin_amdgcn_wave_barrier() { emu::gsync((int)(threadIdx.x & ~63u), 64, "wave_barrier"); }

// DPP: quad_perm (ctrl < 0x100), row_mirror (0x140) and row_half_mirror (0x141) only
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int, int, bool) {
  const int t = (int)threadIdx.x;
  int size, from;
  if (ctrl < 0x100) {
    size = 4;
    from = (t & ~3) + ((ctrl >> (2 * (t & 3))) & 3);
  } else if (ctrl == 0x140) {
    size = 16;
    from = (t & ~15) + (15 - (t & 15));
  } else if (ctrl == 0x141) {
    size = 8;
    from = (t & ~7) + (7 - (t & 7));
  } else {
    std::fprintf(stderr, "emu: unsupported dpp ctrl 0x%x\n", ctrl);
    std::abort();
  }
  (void)old;
  const int base = t & ~(size - 1);
  emu::xch[t] = src;
  emu::gsync(base, size, "dpp");
  const int v = emu::xch[from];
  emu::gsync(base, size, "dpp");
  return v;
}
// ds_swizzle in bit-mask mode 0x401F: lane xor 16 inside 32-lane groups
inline int __builtin_amdgcn_ds_swizzle(int src, int pattern) {
  if (pattern != 0x401F) {
    std::fprintf(stderr, "emu: unsupported swizzle 0x%x\n", pattern);
    std::abort();
  }
  const int t = (int)threadIdx.x;
  const int base = t & ~31;
  emu::xch[t] = src;
  emu::gsync(base, 32, "swizzle");
  const int v = emu::xch[t ^ 16];
  emu::gsync(base, 32, "swizzle");
  return v;
}
// ds_bpermute: every lane of the wave takes part; byte address / 4 names the source lane
inline int __builtin_amdgcn_ds_bpermute(int addr, int src) {
  const int t = (int)threadIdx.x;
  const int base = t & ~63;
  emu::xch[t] = src;
  emu::gsync(base, 64, "bpermute");
  const int from = base + ((addr >> 2) & 63);
  const int v = emu::xch[from];
  emu::gsync(base, 64, "bpermute");
  return v;
}
inline uint64_t __ballot(int pred) {
  const int t = (int)threadIdx.x;
  const int base = t & ~63;
  emu::xch[t] = pred ? 1 : 0;
  emu::gsync(base, 64, "ballot");
  uint64_t m = 0;
  for (int l = 0; l < 64; ++l)
    if (emu::xch[base + l]) m |= 1ull << l;
  emu::gsync(base, 64, "ballot");
  return m;
}
template <class T>
inline T atomicAdd(T* p, T v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
