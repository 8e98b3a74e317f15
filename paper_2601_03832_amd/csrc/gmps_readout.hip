// Set-up and read-out kernels of libgmps (gfx950): the uniform initial state, the marked
// probability of Eq. (6), single amplitudes and perfect sampling of the final chains.
// They serve both iterate kernels; a site slot holds (D, 2, D) elements with D = 2 * CM of
// the instance's class, and bonds[inst * 64 + l] gives bond l.
#include "gmps_device.h"

namespace gmps {

constexpr int kChiMax = 32;  // largest bond of any class
constexpr int kNumQueues = 1 + kNumWide;  // lane-group kernel and one per team class

__global__ void queue_reset_kernel(QueueState* q) {
  if (blockIdx.x == 0 && threadIdx.x < kNumQueues) q[threadIdx.x].next = 0u;
}

// a2: every instance <- |+>^n with all bonds 1; warm-start records emptied; the edge slots hold
// their sites, (1, 2, 1), in complex FP64.
template <class S>
__global__ void init_uniform_kernel(InstDev* inst, int B, const int64_t* site_start, int32_t* bonds,
                                    void* arena_v, int64_t total_sites, char* warm, cd* edge) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total_sites) return;
  // locate the instance owning global site t (site_start is the prefix sum of n)
  int lo = 0, hi = B;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (site_start[mid] <= t) lo = mid; else hi = mid;
  }
  InstDev& I = inst[lo];
  const int i = (int)(t - site_start[lo]);
  const int CM = class_cm(I.cls);
  const int D = 2 * CM;
  cx<S>* slot = reinterpret_cast<cx<S>*>(arena_v) + I.site_off + (int64_t)i * slot_elems(CM);
  const S h = (S)0.70710678118654752440;
  slot[0] = {h, (S)0};
  slot[D] = {h, (S)0};
  const int ei = edge_index(i, I.n, I.ew);
  if (edge && ei >= 0) {
    cd* es = edge + I.edge_off + (int64_t)ei * slot_elems(CM);
    es[0] = {0.70710678118654752440, 0.0};
    es[D] = {0.70710678118654752440, 0.0};
  }
  bonds[(int64_t)lo * kBondStride + i] = 1;
  if (i == I.n - 1) bonds[(int64_t)lo * kBondStride + I.n] = 1;
  if (warm) {
    if (is_wide(I.cls)) {
      double* base = reinterpret_cast<double*>(warm + I.warm_off);
      const int64_t rec = wide_warm_doubles(CM);
      for (int j = 0; j <= I.M; ++j) base[((int64_t)j * I.n + i) * rec] = 0.0;
    } else {
      WarmRec* base = reinterpret_cast<WarmRec*>(warm + I.warm_off);
      for (int j = 0; j <= I.M; ++j) base[(int64_t)j * I.n + i].r = 0;
    }
  }
  if (i == 0) {
    I.k_done = 0;
    I.status = 0;
    I.drift = 0.0;
    I.trunc_w = 0.0;
    I.flops64 = 0.0;
    I.flops32 = 0.0;
  }
}

// Element (a, s, b) of site i. With edge slots (team kernels; esl = the instance's first edge
// slot), an edge site is read in complex FP64 from its edge slot; its site slot keeps a
// storage-type copy.
template <class S>
__device__ __forceinline__ cd site_elem(const cx<S>* slot, const cd* esl, const InstDev& I, int i, int a, int s,
                                        int b, int D) {
  const int ei = esl ? edge_index(i, I.n, I.ew) : -1;
  if (ei >= 0) return esl[(int64_t)ei * (2 * D * D) + a * D * 2 + s * D + b];
  return up(slot[a * D * 2 + s * D + b]);
}

// -------------------------------------------------------------------------- marked prob
// Eq. (6) for one instance per 64-thread workgroup: <psi|psi> by left transfer matrices
// E <- sum_s A_s^dagger E A_s (E in LDS), and each <x|psi> for x in W by slice products
// v <- v A_i[:, x_i, :] with the lanes over the right bond.
// <psi|psi> of instance I by left transfer matrices E <- sum_s A_s^dagger E A_s, in LDS; the
// 64 threads of the workgroup call it together.
template <class S>
__device__ double norm2_of(const InstDev& I, const int32_t* bond, const cx<S>* base, const cd* esl,
                           cd (*E)[kChiMax], cd (*F)[2][kChiMax]) {
  const int tl = threadIdx.x;
  const int CM = class_cm(I.cls);
  const int D = 2 * CM;
  const int n = I.n;
  if (tl == 0) E[0][0] = {1.0, 0.0};
  __syncthreads();
  int chl = 1;
  for (int i = 0; i < n; ++i) {
    const int chr = bond[i + 1];
    const cx<S>* slot = base + (int64_t)i * slot_elems(CM);
    // F[a][s][bb] = sum_aa E[a][aa] A[aa][s][bb]
    for (int e = tl; e < chl * 2 * chr; e += 64) {
      const int a = e / (2 * chr), s = (e / chr) & 1, bb = e % chr;
      cd acc = {0.0, 0.0};
      for (int aa = 0; aa < chl; ++aa) acc = cfma(acc, E[a][aa], site_elem(slot, esl, I, i, aa, s, bb, D));
      F[a][s][bb] = acc;
    }
    __syncthreads();
    // E'[b1][bb] = sum_{s, a} conj(A[a][s][b1]) F[a][s][bb]; E itself is no longer read
    for (int e = tl; e < chr * chr; e += 64) {
      const int b1 = e / chr, bb = e % chr;
      cd acc = {0.0, 0.0};
      for (int s = 0; s < 2; ++s)
        for (int a = 0; a < chl; ++a) acc = acc + cmulc(site_elem(slot, esl, I, i, a, s, b1, D), F[a][s][bb]);
      E[b1][bb] = acc;
    }
    __syncthreads();
    chl = chr;
  }
  return E[0][0].re;
}

template <class S>
__global__ __launch_bounds__(64) void marked_prob_kernel(InstDev* inst, const uint64_t* marked,
                                                         const int32_t* bonds, const void* arena_v, int B,
                                                         const cd* edge_all, double* out) {
  __shared__ cd E[kChiMax][kChiMax];
  __shared__ cd F[kChiMax][2][kChiMax];
  __shared__ cd v[2][kChiMax];
  const int b = blockIdx.x;
  if (b >= B) return;
  const int tl = threadIdx.x;
  InstDev& I = inst[b];
  const int CM = class_cm(I.cls);
  const int D = 2 * CM;
  const int n = I.n;
  const cx<S>* base = reinterpret_cast<const cx<S>*>(arena_v) + I.site_off;
  const cd* esl = edge_all ? edge_all + I.edge_off : nullptr;
  const int32_t* bond = bonds + (int64_t)b * kBondStride;
  const double nn = norm2_of<S>(I, bond, base, esl, E, F);
  double acc = 0.0;
  for (int j = 0; j < I.M; ++j) {
    const uint64_t x = marked[I.marked_off + j];
    if (tl == 0) v[0][0] = {1.0, 0.0};
    __syncthreads();
    int cl = 1, cur = 0;
    for (int i = 0; i < n; ++i) {
      const int chr = bond[i + 1];
      const int s = (int)((x >> (n - 1 - i)) & 1ull);
      const cx<S>* slot = base + (int64_t)i * slot_elems(CM);
      if (tl < chr) {
        cd w = {0.0, 0.0};
        for (int a = 0; a < cl; ++a) w = cfma(w, v[cur][a], site_elem(slot, esl, I, i, a, s, tl, D));
        v[cur ^ 1][tl] = w;
      }
      __syncthreads();
      cur ^= 1;
      cl = chr;
    }
    acc += norm2(v[cur][0]);
    __syncthreads();
  }
  if (tl == 0) {
    const double p = acc / nn;
    if (!isfinite(p)) I.status |= GMPS_ST_NAN;
    out[b] = p;
  }
}

// ---------------------------------------------------------------------------- amplitudes
template <class S, int MAXC>
__device__ cd amplitude_of(const InstDev& I, const int32_t* bond, const cx<S>* base, const cd* esl, uint64_t x) {
  const int CM = class_cm(I.cls);
  const int D = 2 * CM;
  const int n = I.n;
  cd v[MAXC];
  v[0] = {1.0, 0.0};
  int chl = 1;
  for (int i = 0; i < n; ++i) {
    const int chr = bond[i + 1];
    const int s = (int)((x >> (n - 1 - i)) & 1ull);
    const cx<S>* slot = base + (int64_t)i * slot_elems(CM);
    cd w[MAXC];
#pragma unroll
    for (int b = 0; b < MAXC; ++b) {
      cd acc = {0.0, 0.0};
      if (b < chr) {
#pragma unroll
        for (int a = 0; a < MAXC; ++a)
          if (a < chl) acc = cfma(acc, v[a], site_elem(slot, esl, I, i, a, s, b, D));
      }
      w[b] = acc;
    }
#pragma unroll
    for (int b = 0; b < MAXC; ++b) v[b] = w[b];
    chl = chr;
  }
  return v[0];
}

// <s|psi> of one instance, |s> = |+>^n: slice products with (A[:, 0, :] + A[:, 1, :]) / sqrt(2),
// the lanes over the right bond.
template <class S>
__global__ __launch_bounds__(64) void overlap_uniform_kernel(const InstDev* inst, int which, const int32_t* bonds,
                                                             const void* arena_v, const cd* edge_all, double* out) {
  __shared__ cd v[2][kChiMax];
  const int tl = threadIdx.x;
  const InstDev& I = inst[which];
  const int CM = class_cm(I.cls);
  const int D = 2 * CM;
  const cx<S>* base = reinterpret_cast<const cx<S>*>(arena_v) + I.site_off;
  const cd* esl = edge_all ? edge_all + I.edge_off : nullptr;
  const int32_t* bond = bonds + (int64_t)which * kBondStride;
  if (tl == 0) v[0][0] = {1.0, 0.0};
  __syncthreads();
  int cl = 1, cur = 0;
  for (int i = 0; i < I.n; ++i) {
    const int chr = bond[i + 1];
    const cx<S>* slot = base + (int64_t)i * slot_elems(CM);
    if (tl < chr) {
      cd w = {0.0, 0.0};
      for (int a = 0; a < cl; ++a)
        w = cfma(w, v[cur][a], kInvSqrt2 * (site_elem(slot, esl, I, i, a, 0, tl, D) + site_elem(slot, esl, I, i, a, 1, tl, D)));
      v[cur ^ 1][tl] = w;
    }
    __syncthreads();
    cur ^= 1;
    cl = chr;
  }
  if (tl == 0) {
    out[0] = v[cur][0].re;
    out[1] = v[cur][0].im;
  }
}

hipError_t launch_overlap_uniform(bool mixed, const InstDev* inst, int which, const int32_t* bonds,
                                  const void* arena, const void* edge, double* out, hipStream_t st) {
  const cd* c = reinterpret_cast<const cd*>(edge);
  if (mixed)
    overlap_uniform_kernel<float><<<1, 64, 0, st>>>(inst, which, bonds, arena, c, out);
  else
    overlap_uniform_kernel<double><<<1, 64, 0, st>>>(inst, which, bonds, arena, c, out);
  return hipGetLastError();
}

// <psi|psi> of one instance (the amplitudes are reported for the normalised state).
template <class S>
__global__ __launch_bounds__(64) void norm_kernel(const InstDev* inst, int which, const int32_t* bonds,
                                                  const void* arena_v, const cd* edge_all, double* out) {
  __shared__ cd E[kChiMax][kChiMax];
  __shared__ cd F[kChiMax][2][kChiMax];
  const InstDev& I = inst[which];
  const cx<S>* base = reinterpret_cast<const cx<S>*>(arena_v) + I.site_off;
  const cd* esl = edge_all ? edge_all + I.edge_off : nullptr;
  const double nn = norm2_of<S>(I, bonds + (int64_t)which * kBondStride, base, esl, E, F);
  if (threadIdx.x == 0) out[0] = nn;
}

template <class S, int MAXC>
__global__ void amplitude_kernel(const InstDev* inst, int which, const int32_t* bonds, const void* arena_v,
                                 const cd* edge_all, const uint64_t* xs, int64_t cnt, double* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const InstDev& I = inst[which];
  const cx<S>* base = reinterpret_cast<const cx<S>*>(arena_v) + I.site_off;
  const cd a = amplitude_of<S, MAXC>(I, bonds + (int64_t)which * kBondStride, base,
                                     edge_all ? edge_all + I.edge_off : nullptr, xs[t]);
  out[2 * t] = a.re;
  out[2 * t + 1] = a.im;
}

// ------------------------------------------------------------------------------ sampling
// Philox4x64-10 (Salmon et al., SC'11).
__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

// One shot per thread: site by site, p(0 | prefix) = ||v A[:, 0, :]||^2 / (||v A[:, 0, :]||^2 +
// ||v A[:, 1, :]||^2) on the right-canonical chain, the uniform of the (instance, shot, site)
// triple decides the bit, and v moves to the chosen (normalised) branch.
template <class S, int MAXC>
__global__ void sample_kernel(const InstDev* inst, const uint64_t* marked, const int32_t* bonds,
                              const void* arena_v, const cd* edge_all, int B, int inst_base,
                              const int64_t* shot_off, uint64_t seed, uint64_t* bits, unsigned long long* hits) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= shot_off[B]) return;
  int lo = 0, hi = B;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (shot_off[mid] <= t) lo = mid; else hi = mid;
  }
  while (lo + 1 < B && shot_off[lo + 1] <= t) ++lo;  // skip instances with zero shots
  const InstDev& I = inst[lo];
  const int64_t shot = t - shot_off[lo];
  const int CM = class_cm(I.cls);
  const int D = 2 * CM;
  const int n = I.n;
  const cx<S>* base = reinterpret_cast<const cx<S>*>(arena_v) + I.site_off;
  const int32_t* bond = bonds + (int64_t)lo * kBondStride;
  const cd* esl = edge_all ? edge_all + I.edge_off : nullptr;
  cd v[MAXC];
  v[0] = {1.0, 0.0};
  int chl = 1;
  uint64_t x = 0;
  uint64_t words[4] = {0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    if ((i & 3) == 0) {
      words[0] = (uint64_t)shot;
      words[1] = (uint64_t)(i >> 2);
      words[2] = 0;
      words[3] = 0;
      philox4x64_10(words, seed, (uint64_t)(lo + inst_base));
    }
    const double u = (double)(words[i & 3] >> 11) * (1.0 / 9007199254740992.0);
    const int chr = bond[i + 1];
    const cx<S>* slot = base + (int64_t)i * slot_elems(CM);
    cd w0[MAXC], w1[MAXC];
    double q0 = 0.0, q1 = 0.0;
#pragma unroll
    for (int b = 0; b < MAXC; ++b) {
      cd a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
      if (b < chr) {
#pragma unroll
        for (int a = 0; a < MAXC; ++a)
          if (a < chl) {
            a0 = cfma(a0, v[a], site_elem(slot, esl, I, i, a, 0, b, D));
            a1 = cfma(a1, v[a], site_elem(slot, esl, I, i, a, 1, b, D));
          }
      }
      w0[b] = a0;
      w1[b] = a1;
      q0 += norm2(a0);
      q1 += norm2(a1);
    }
    const double p0 = q0 / (q0 + q1);
    const bool zero = u < p0;
    const double sc = 1.0 / sqrt(zero ? q0 : q1);
#pragma unroll
    for (int b = 0; b < MAXC; ++b) v[b] = sc * (zero ? w0[b] : w1[b]);
    if (!zero) x |= 1ull << (n - 1 - i);
    chl = chr;
  }
  if (bits) bits[t] = x;  // null: hits only
  for (int j = 0; j < I.M; ++j)
    if (marked[I.marked_off + j] == x) {
      atomicAdd(hits + lo, 1ull);
      break;
    }
}

// ------------------------------------------------------------------------- launch wrappers
hipError_t launch_queue_reset(QueueState* q, hipStream_t st) {
  queue_reset_kernel<<<1, 64, 0, st>>>(q);
  return hipGetLastError();
}

hipError_t launch_init(bool mixed, InstDev* inst, int B, const int64_t* site_start, int32_t* bonds, void* arena,
                       int64_t total_sites, char* warm, void* edge, hipStream_t st) {
  const int blk = 256;
  const int grid = (int)((total_sites + blk - 1) / blk);
  if (grid == 0) return hipSuccess;
  cd* c = reinterpret_cast<cd*>(edge);
  if (mixed)
    init_uniform_kernel<float><<<grid, blk, 0, st>>>(inst, B, site_start, bonds, arena, total_sites, warm, c);
  else
    init_uniform_kernel<double><<<grid, blk, 0, st>>>(inst, B, site_start, bonds, arena, total_sites, warm, c);
  return hipGetLastError();
}

hipError_t launch_prob(bool mixed, InstDev* inst, const uint64_t* marked, const int32_t* bonds, const void* arena,
                       const void* edge, int B, double* out, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  const cd* c = reinterpret_cast<const cd*>(edge);
  if (mixed)
    marked_prob_kernel<float><<<B, 64, 0, st>>>(inst, marked, bonds, arena, B, c, out);
  else
    marked_prob_kernel<double><<<B, 64, 0, st>>>(inst, marked, bonds, arena, B, c, out);
  return hipGetLastError();
}

// Register arrays are sized by the largest bond the batch can hold.
template <class S>
static void amp_launch(int maxc, int grid, hipStream_t st, const InstDev* inst, int which, const int32_t* bonds,
                       const void* arena, const cd* edge, const uint64_t* xs, int64_t cnt, double* out) {
  if (maxc <= 8)
    amplitude_kernel<S, 8><<<grid, 64, 0, st>>>(inst, which, bonds, arena, edge, xs, cnt, out);
  else if (maxc <= 17)
    amplitude_kernel<S, 17><<<grid, 64, 0, st>>>(inst, which, bonds, arena, edge, xs, cnt, out);
  else
    amplitude_kernel<S, 32><<<grid, 64, 0, st>>>(inst, which, bonds, arena, edge, xs, cnt, out);
}

hipError_t launch_amplitudes(bool mixed, int maxc, const InstDev* inst, int which, const int32_t* bonds,
                             const void* arena, const void* edge, const uint64_t* xs, int64_t cnt, double* out,
                             double* norm2, hipStream_t st) {
  const int grid = (int)((cnt + 63) / 64);
  if (grid == 0) return hipSuccess;
  const cd* c = reinterpret_cast<const cd*>(edge);
  if (mixed) {
    norm_kernel<float><<<1, 64, 0, st>>>(inst, which, bonds, arena, c, norm2);
    amp_launch<float>(maxc, grid, st, inst, which, bonds, arena, c, xs, cnt, out);
  } else {
    norm_kernel<double><<<1, 64, 0, st>>>(inst, which, bonds, arena, c, norm2);
    amp_launch<double>(maxc, grid, st, inst, which, bonds, arena, c, xs, cnt, out);
  }
  return hipGetLastError();
}

template <class S>
static void sample_launch(int maxc, int grid, hipStream_t st, const InstDev* inst, const uint64_t* marked,
                          const int32_t* bonds, const void* arena, const cd* edge, int B, int inst_base,
                          const int64_t* shot_off, uint64_t seed, uint64_t* bits, unsigned long long* hits) {
  if (maxc <= 8)
    sample_kernel<S, 8><<<grid, 64, 0, st>>>(inst, marked, bonds, arena, edge, B, inst_base, shot_off, seed, bits, hits);
  else if (maxc <= 17)
    sample_kernel<S, 17><<<grid, 64, 0, st>>>(inst, marked, bonds, arena, edge, B, inst_base, shot_off, seed, bits, hits);
  else
    sample_kernel<S, 32><<<grid, 64, 0, st>>>(inst, marked, bonds, arena, edge, B, inst_base, shot_off, seed, bits, hits);
}

// Instances inst_base .. inst_base + B - 1 (inst, bonds and hits point at the first of them);
// shot_off: [B + 1] offsets of their shots in bits.
hipError_t launch_sample(bool mixed, int maxc, const InstDev* inst, const uint64_t* marked, const int32_t* bonds,
                         const void* arena, const void* edge, int B, int inst_base, const int64_t* shot_off,
                         int64_t total, uint64_t seed, uint64_t* bits, unsigned long long* hits, hipStream_t st) {
  const int grid = (int)((total + 63) / 64);
  if (grid == 0) return hipSuccess;
  const cd* c = reinterpret_cast<const cd*>(edge);
  if (mixed)
    sample_launch<float>(maxc, grid, st, inst, marked, bonds, arena, c, B, inst_base, shot_off, seed, bits, hits);
  else
    sample_launch<double>(maxc, grid, st, inst, marked, bonds, arena, c, B, inst_base, shot_off, seed, bits, hits);
  return hipGetLastError();
}

}  // namespace gmps
