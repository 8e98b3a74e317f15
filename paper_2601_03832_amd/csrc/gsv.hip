// Dense-statevector iterative Grover backend of libgmps (gfx950): the comparison path of the
// paper's Section III-A / Fig. 2. The real state vector psi' (the state with the oracle of
// the coming iteration already applied) lives in HBM; one iteration is
//   pass:  y = 2 mu - psi'       (the diffusion D = 2|s><s| - I of Eq. (4); mu = mean of psi')
//          and per-block sums of y, written to a partial-sum array (no atomics)
//   fix:   one block adds the partials in a fixed order, flips the M marked entries of y
//          (the oracle O of Eq. (3) for the next iteration) and corrects the sum, giving
//          2 mu for the next pass.
// The pass streams N values in and N out: it is HBM-bound (8 TB/s: 2^28 FP64 values in
// 0.54 ms). Sums are FP64 in both precisions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_set>
#include <vector>

#include "../../include/gsv.h"

namespace {

constexpr int kThreads = 256;
constexpr int kPairsPerThread = 8;  // 16 amplitudes per thread and loop trip
constexpr int kMaxBlocks = 4096;
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

template <class T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};

// 256-thread block sum, same result in every run (fixed order); returns it to thread 0.
__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// y = two_mu - x over all pairs (two_mu == nullptr: y = fill, the uniform state); block sums.
template <class T>
__global__ __launch_bounds__(kThreads) void sv_pass_kernel(T* psi, int64_t npairs, const double* two_mu,
                                                           double fill, double* partial) {
  __shared__ double red[kThreads / 64];
  using V = typename Vec2<T>::type;
  V* p = reinterpret_cast<V*>(psi);
  const double tm = two_mu ? *two_mu : 0.0;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads * kPairsPerThread;
  for (int64_t base = ((int64_t)blockIdx.x * kThreads) * kPairsPerThread + threadIdx.x; base < npairs;
       base += stride) {
    // The vector is read and written once per pass and is far larger than the caches:
    // non-temporal loads and stores keep it from evicting other lines (about 9% faster in
    // FP64 and, with 8 pairs per thread, 18% in FP32 at n = 28).
    V v[kPairsPerThread];
#pragma unroll
    for (int u = 0; u < kPairsPerThread; ++u) {
      const int64_t i = base + (int64_t)u * kThreads;
      if (i < npairs) {
        v[u].x = __builtin_nontemporal_load(&p[i].x);
        v[u].y = __builtin_nontemporal_load(&p[i].y);
      }
    }
#pragma unroll
    for (int u = 0; u < kPairsPerThread; ++u) {
      const int64_t i = base + (int64_t)u * kThreads;
      if (i < npairs) {
        const double y0 = two_mu ? tm - (double)v[u].x : fill;
        const double y1 = two_mu ? tm - (double)v[u].y : fill;
        V o;
        o.x = (T)y0;
        o.y = (T)y1;
        __builtin_nontemporal_store(o.x, &p[i].x);
        __builtin_nontemporal_store(o.y, &p[i].y);
        acc += (double)o.x + (double)o.y;
      }
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Sum of the partials, oracle flip of the marked entries, 2 mu of the flipped state.
template <class T>
__global__ __launch_bounds__(kThreads) void sv_fix_kernel(T* psi, const uint64_t* marked, int64_t M,
                                                          const double* partial, int nblocks, double inv_n,
                                                          double* two_mu) {
  __shared__ double red[kThreads / 64];
  double a = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kThreads) a += partial[b];
  double f = 0.0;
  for (int64_t j = threadIdx.x; j < M; j += kThreads) {
    const uint64_t x = marked[j];
    const T v = psi[x];
    psi[x] = -v;
    f += (double)v;
  }
  const double sum = block_sum(a, red);
  const double flipped = block_sum(f, red);
  if (threadIdx.x == 0) *two_mu = 2.0 * (sum - 2.0 * flipped) * inv_n;
}

// sum of psi^2 over all entries (per-block partials) for the norm
template <class T>
__global__ __launch_bounds__(kThreads) void sv_norm_kernel(const T* psi, int64_t npairs, double* partial) {
  __shared__ double red[kThreads / 64];
  using V = typename Vec2<T>::type;
  const V* p = reinterpret_cast<const V*>(psi);
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < npairs; i += (int64_t)gridDim.x * kThreads) {
    const V v = p[i];
    acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <class T>
__global__ void sv_gather_kernel(const T* psi, const uint64_t* xs, int64_t cnt, double* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) out[t] = (double)psi[xs[t]];
}

}  // namespace

struct gsv_state {
  int n = 0;
  int64_t N = 0, M = 0;
  bool f32 = false;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  void* psi = nullptr;
  uint64_t* marked = nullptr;
  double* partial = nullptr;
  double* two_mu = nullptr;
  double* out = nullptr;  // read-out staging: [2 + 2*kMaxBlocks]
  std::vector<uint64_t> marked_h;
  int blocks = 1;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
};

namespace {

int hipfail(hipError_t e) { return e == hipSuccess ? GMPS_OK : GMPS_E_HIP; }
#define GSV_HIP(call)                        \
  do {                                       \
    if ((call) != hipSuccess) return GMPS_E_HIP; \
  } while (0)

struct SvLayout {
  size_t psi, marked, partial, two_mu, out, total;
};
bool sv_layout(int32_t n, int32_t M, gmps_prec prec, SvLayout* L) {
  if (n < 1 || n > 34 || M < 1 || (prec != GMPS_FP64 && prec != GMPS_MIXED)) return false;
  const int64_t N = int64_t(1) << n;
  if (M >= N) return false;
  size_t off = 0;
  L->psi = off;     off = align_up(off + (size_t)N * (prec == GMPS_FP64 ? 8 : 4));
  L->marked = off;  off = align_up(off + sizeof(uint64_t) * (size_t)M);
  L->partial = off; off = align_up(off + sizeof(double) * kMaxBlocks);
  L->two_mu = off;  off = align_up(off + sizeof(double));
  L->out = off;     off = align_up(off + sizeof(double) * (2 + 2 * kMaxBlocks));
  L->total = off;
  return true;
}

template <class T>
hipError_t pass(gsv_state* s, bool init) {
  const double fill = 1.0 / std::sqrt((double)s->N);
  sv_pass_kernel<T><<<s->blocks, kThreads, 0, s->stream>>>(reinterpret_cast<T*>(s->psi), s->N / 2,
                                                           init ? nullptr : s->two_mu, fill, s->partial);
  sv_fix_kernel<T><<<1, kThreads, 0, s->stream>>>(reinterpret_cast<T*>(s->psi), s->marked, s->M, s->partial,
                                                  s->blocks, 1.0 / (double)s->N, s->two_mu);
  return hipGetLastError();
}

}  // namespace

extern "C" {

size_t gsv_workspace_bytes(int32_t n, int32_t M, gmps_prec prec) {
  SvLayout L;
  return sv_layout(n, M, prec, &L) ? L.total : 0;
}

int gsv_create(gsv_state** out, int32_t n, const uint64_t* marked, int32_t M, gmps_prec prec, void* dev_workspace,
               size_t ws_bytes, void* hip_stream) {
  if (!out) return GMPS_E_ARG;
  *out = nullptr;
  SvLayout L;
  if (!marked || !sv_layout(n, M, prec, &L)) return GMPS_E_ARG;
  std::unordered_set<uint64_t> seen;
  for (int j = 0; j < M; ++j) {
    if ((marked[j] >> n) != 0 || !seen.insert(marked[j]).second) return GMPS_E_ARG;
  }
  if (!dev_workspace || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) != 0)
    return GMPS_E_WORKSPACE;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return GMPS_E_UNSUPPORTED;
  gsv_state* s = new (std::nothrow) gsv_state();
  if (!s) return GMPS_E_ARG;
  s->n = n;
  s->N = int64_t(1) << n;
  s->M = M;
  s->f32 = prec == GMPS_MIXED;
  s->stream = reinterpret_cast<hipStream_t>(hip_stream);
  s->ws = reinterpret_cast<char*>(dev_workspace);
  s->psi = s->ws + L.psi;
  s->marked = reinterpret_cast<uint64_t*>(s->ws + L.marked);
  s->partial = reinterpret_cast<double*>(s->ws + L.partial);
  s->two_mu = reinterpret_cast<double*>(s->ws + L.two_mu);
  s->out = reinterpret_cast<double*>(s->ws + L.out);
  s->marked_h.assign(marked, marked + M);
  const int64_t npairs = s->N / 2;
  const int64_t per_block = (int64_t)kThreads * kPairsPerThread;
  s->blocks = (int)std::max<int64_t>(1, std::min<int64_t>((npairs + per_block - 1) / per_block, kMaxBlocks));
  int rc = GMPS_OK;
  if ((rc = hipfail(hipMemcpyAsync(s->marked, marked, sizeof(uint64_t) * M, hipMemcpyHostToDevice, s->stream))) ||
      (rc = hipfail(hipEventCreate(&s->ev0))) || (rc = hipfail(hipEventCreate(&s->ev1))) ||
      (rc = hipfail(hipStreamSynchronize(s->stream)))) {
    gsv_destroy(s);
    return rc;
  }
  *out = s;
  return GMPS_OK;
}

int gsv_init_uniform(gsv_state* s) {
  if (!s) return GMPS_E_ARG;
  GSV_HIP(s->f32 ? pass<float>(s, true) : pass<double>(s, true));
  return GMPS_OK;
}

int gsv_iterate(gsv_state* s, int64_t k) {
  if (!s || k < 0) return GMPS_E_ARG;
  GSV_HIP(hipEventRecord(s->ev0, s->stream));
  for (int64_t it = 0; it < k; ++it) GSV_HIP(s->f32 ? pass<float>(s, false) : pass<double>(s, false));
  GSV_HIP(hipEventRecord(s->ev1, s->stream));
  s->timed = true;
  return GMPS_OK;
}

int gsv_marked_prob(gsv_state* s, double* out_p) {
  if (!s || !out_p) return GMPS_E_ARG;
  const int64_t npairs = s->N / 2;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((npairs + kThreads - 1) / kThreads, kMaxBlocks));
  if (s->f32)
    sv_norm_kernel<float><<<nb, kThreads, 0, s->stream>>>(reinterpret_cast<const float*>(s->psi), npairs, s->out + 2);
  else
    sv_norm_kernel<double><<<nb, kThreads, 0, s->stream>>>(reinterpret_cast<const double*>(s->psi), npairs, s->out + 2);
  GSV_HIP(hipGetLastError());
  std::vector<double> part(nb);
  GSV_HIP(hipMemcpyAsync(part.data(), s->out + 2, sizeof(double) * nb, hipMemcpyDeviceToHost, s->stream));
  std::vector<double> amp(s->M);
  int rc = gsv_amplitudes(s, s->marked_h.data(), s->M, amp.data());
  if (rc != GMPS_OK) return rc;
  double nn = 0.0, pm = 0.0;
  for (double v : part) nn += v;
  for (double v : amp) pm += v * v;
  *out_p = pm / nn;
  return GMPS_OK;
}

int gsv_amplitudes(gsv_state* s, const uint64_t* xs, int64_t cnt, double* out) {
  if (!s || cnt < 0 || (cnt > 0 && (!xs || !out))) return GMPS_E_ARG;
  for (int64_t t = 0; t < cnt; ++t)
    if ((xs[t] >> s->n) != 0) return GMPS_E_ARG;
  if (cnt == 0) return GMPS_OK;
  // staged through a temporary device buffer in chunks that fit the read-out slots
  std::unordered_set<uint64_t> mk(s->marked_h.begin(), s->marked_h.end());
  const int64_t chunk = kMaxBlocks;  // xs and values share the 2*kMaxBlocks slots
  uint64_t* dxs = reinterpret_cast<uint64_t*>(s->out + 2);
  double* dval = s->out + 2 + kMaxBlocks;
  for (int64_t o = 0; o < cnt; o += chunk) {
    const int64_t c = std::min(chunk, cnt - o);
    GSV_HIP(hipMemcpyAsync(dxs, xs + o, sizeof(uint64_t) * c, hipMemcpyHostToDevice, s->stream));
    const int g = (int)((c + 255) / 256);
    if (s->f32)
      sv_gather_kernel<float><<<g, 256, 0, s->stream>>>(reinterpret_cast<const float*>(s->psi), dxs, c, dval);
    else
      sv_gather_kernel<double><<<g, 256, 0, s->stream>>>(reinterpret_cast<const double*>(s->psi), dxs, c, dval);
    GSV_HIP(hipGetLastError());
    GSV_HIP(hipMemcpyAsync(out + o, dval, sizeof(double) * c, hipMemcpyDeviceToHost, s->stream));
    GSV_HIP(hipStreamSynchronize(s->stream));
  }
  // the stored vector carries the coming iteration's oracle: undo it on marked entries
  for (int64_t t = 0; t < cnt; ++t)
    if (mk.count(xs[t])) out[t] = -out[t];
  return GMPS_OK;
}

int gsv_last_iterate_ms(gsv_state* s, double* ms) {
  if (!s || !ms) return GMPS_E_ARG;
  if (!s->timed) {
    *ms = 0.0;
    return GMPS_OK;
  }
  GSV_HIP(hipEventSynchronize(s->ev1));
  float f = 0.f;
  GSV_HIP(hipEventElapsedTime(&f, s->ev0, s->ev1));
  *ms = f;
  return GMPS_OK;
}

int gsv_destroy(gsv_state* s) {
  if (!s) return GMPS_OK;
  (void)hipStreamSynchronize(s->stream);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  delete s;
  return GMPS_OK;
}

}  // extern "C"
