// Host emulation of one iterate kernel body on one instance: every lane of the workgroup is
// an OS thread (cross-lane operations and barriers synchronise the lanes they involve; see
// hip/hip_runtime.h here), every buffer is its own heap allocation of the size the library
// gives it, and the result goes to stdout for comparison with the oracle. Built with
// sanitizers by tests/test_host_emulation.py:
//   EMU_KIND 0: run_team (bond-2 MPO reflections), 1: run_team_pc (pre-contracted),
//            2: run_pipe (pipelined sweeps), 3: run_pipe pre-contracted, 4: run_team_circ (the
//            k-layer gate-level circuit of Fig. 1(A), built here as gmps_circuit_build does);
//            EMU_W: team class; EMU_S: double or float.
// stdin: n M cap k, then the M marked indices. stdout: status drift trunc_w, the bonds, then
// the 2^n amplitudes (re im per line).
#include "hip/hip_runtime.h"
#include "gmps_pipe.h"
#include "gmps_team.h"

#include <chrono>
#include <complex>
#include <iostream>
#include <vector>

thread_local emu_dim3 threadIdx;
thread_local emu_dim3 blockIdx;
emu_dim3 blockDim, gridDim;

namespace emu {
int32_t xch[kMaxThreads];
uint64_t bal[kMaxThreads / 64];
static std::atomic<int> arrive[6][kMaxThreads];
static std::atomic<int> gen[6][kMaxThreads];
static int sidx(int size) {
  switch (size) {
    case 4: return 0;
    case 8: return 1;
    case 16: return 2;
    case 32: return 3;
    case 64: return 4;
    default: return 5;
  }
}
void gsync(int base, int size, const char* what) {
  const int si = sidx(size);
  std::atomic<int>& a = arrive[si][base];
  std::atomic<int>& g = gen[si][base];
  const int my = g.load(std::memory_order_acquire);
  if (a.fetch_add(1, std::memory_order_acq_rel) + 1 == size) {
    a.store(0, std::memory_order_relaxed);
    g.fetch_add(1, std::memory_order_release);
    return;
  }
  auto t0 = std::chrono::steady_clock::now();
  long spins = 0;
  while (g.load(std::memory_order_acquire) == my) {
    if (++spins > 64) std::this_thread::yield();
    if ((spins & 0xFFFF) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120)) {
      std::fprintf(stderr, "emu: %s group [%d, %d) incomplete after 120 s (thread %u, %d arrived): divergent "
                   "lanes or a deadlock\n", what, base, base + size, threadIdx.x, a.load());
      std::abort();
    }
  }
}
}  // namespace emu

using namespace gmps;
using S = EMU_S;
constexpr int W = EMU_W;
constexpr int KIND = EMU_KIND;
constexpr int CM = kWide[W].CM, TW = kWide[W].TW;
constexpr bool kMixed = sizeof(S) == sizeof(float);
constexpr int NT = (KIND == 2 || KIND == 3) ? 128 : (TW < 64 ? 64 : TW);

// templates on every parameter, so that the branches for the other kernels are not instantiated
template <int K, class SS, int C, int T>
size_t lds_size() {
  if constexpr (K == 2)
    return sizeof(PipeLds<SS, C>) * (64 / T);
  else if constexpr (K == 3)
    return (sizeof(PipeLds<SS, C>) + sizeof(PipeOv<C>)) * (64 / T);
  else if constexpr (K == 4)
    return (sizeof(TeamLds<SS, C, T>) + sizeof(CircLds)) * TeamShape<C, T>::TEAMS;
  else
    return (sizeof(TeamLds<SS, C, T>) + (K == 1 ? sizeof(PcLds<C>) : 0)) * TeamShape<C, T>::TEAMS;
}
template <int K, class SS, int C, int T>
void body(const IterParams& P, const Bundle* bundle, char* lds) {
  if constexpr (K == 0)
    run_team<SS, C, T>(P, bundle, lds);
  else if constexpr (K == 1)
    run_team_pc<SS, C, T>(P, bundle, lds);
  else if constexpr (K == 2)
    run_pipe<SS, C, T>(P, bundle, lds);
  else if constexpr (K == 3)
    run_pipe<SS, C, T, true>(P, bundle, lds);
  else
    run_team_circ<SS, C, T>(P, bundle, lds);
}

int main() {
  int n, M, cap;
  long long k;
  std::cin >> n >> M >> cap >> k;
  std::vector<uint64_t> marked_h(M);
  for (auto& x : marked_h) std::cin >> x;
  const int exact = n / 2 < 30 ? std::min(M + 1, 1 << (n / 2)) : M + 1;
  const int eff = std::min(cap, exact);
  const int ew = edge_width(M);
  const int SLOT = slot_elems(CM);
  const int D = 2 * CM;
  if (eff > CM) {
    std::fprintf(stderr, "emu: cap %d exceeds the class\n", eff);
    return 2;
  }

  InstDev* inst = static_cast<InstDev*>(std::calloc(1, sizeof(InstDev)));
  uint64_t* marked = static_cast<uint64_t*>(std::malloc(sizeof(uint64_t) * M));
  int32_t* bonds = static_cast<int32_t*>(std::calloc(kBondStride, sizeof(int32_t)));
  cx<S>* arena = static_cast<cx<S>*>(std::calloc((size_t)n * SLOT, sizeof(cx<S>)));
  const int ne = edge_count(n, ew);
  cd* edge = static_cast<cd*>(std::calloc((size_t)ne * SLOT, sizeof(cd)));
  Bundle* bundle = static_cast<Bundle*>(std::calloc(1, sizeof(Bundle)));
  QueueState* queue = static_cast<QueueState*>(std::calloc(1, sizeof(QueueState)));
  std::memcpy(marked, marked_h.data(), sizeof(uint64_t) * M);

  inst->n = n;
  inst->M = M;
  inst->cap = eff;
  inst->cls = kWideBase + W;
  inst->whole = ((KIND == 1 || KIND == 3) && eff == exact && M <= CM) ? 1 : 0;
  inst->ew = ew;
  const double h = 0.70710678118654752440;
  for (int i = 0; i < n; ++i) {
    arena[(size_t)i * SLOT + 0] = {(S)h, (S)0};
    arena[(size_t)i * SLOT + D] = {(S)h, (S)0};
    const int ei = edge_index(i, n, ew);
    if (ei >= 0) {
      edge[(size_t)ei * SLOT + 0] = {h, 0.0};
      edge[(size_t)ei * SLOT + D] = {h, 0.0};
    }
    bonds[i] = 1;
  }
  bonds[n] = 1;
  bundle->inst[0] = 0;
  bundle->count = 1;
  bundle->cls = inst->cls;
  bundle->k = k;

  IterParams P{};
  P.inst = inst;
  P.marked = marked;
  P.bonds = bonds;
  P.arena = arena;
  P.bundles = bundle;
  P.queue = queue;
  P.trunc_tol = kMixed ? 5e-7 : 1e-12;  // the library's defaults
  P.skip_tol = 1e-15;
  P.rank_tol = P.trunc_tol;
  P.max_sweeps = 16;
  P.stoch_round = 0;
  P.warm = nullptr;
  P.edge = edge;
  // the gate-level circuit: k layers of Fig. 1(A), in its own heap block
  std::vector<uint32_t> gl;
  if (KIND == 4) {
    for (long long l = 0; l < k; ++l) {
      for (int t = 0; t < M; ++t) {
        for (int q = 0; q < n; ++q)
          if (!((marked_h[t] >> (n - 1 - q)) & 1ull)) gl.push_back(gate_word(kGateX, q));
        gl.push_back(gate_word(kGateMCZ, 0));
        for (int q = 0; q < n; ++q)
          if (!((marked_h[t] >> (n - 1 - q)) & 1ull)) gl.push_back(gate_word(kGateX, q));
      }
      for (int q = 0; q < n; ++q) gl.push_back(gate_word(kGateH, q));
      for (int q = 0; q < n; ++q) gl.push_back(gate_word(kGateX, q));
      gl.push_back(gate_word(kGateMCZ, 0));
      for (int q = 0; q < n; ++q) gl.push_back(gate_word(kGateX, q));
      for (int q = 0; q < n; ++q) gl.push_back(gate_word(kGateH, q));
    }
  }
  uint32_t* circ = static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * (gl.size() + 1)));
  if (!gl.empty()) std::memcpy(circ, gl.data(), sizeof(uint32_t) * gl.size());
  P.circuit = KIND == 4 ? circ : nullptr;
  inst->circ_off = 0;
  inst->circ_len = (int64_t)gl.size();

  const size_t lds_bytes = lds_size<KIND, S, CM, TW>();
  const size_t alloc = (lds_bytes + 15) / 16 * 16;
  char* lds = static_cast<char*>(std::aligned_alloc(16, alloc));
  std::memset(lds, 0xCD, alloc);
  blockDim.x = NT;
  gridDim.x = 1;
  std::vector<std::thread> th;
  for (int t = 0; t < NT; ++t)
    th.emplace_back([&, t] {
      threadIdx.x = (unsigned)t;
      blockIdx.x = 0;
      body<KIND, S, CM, TW>(P, bundle, lds);
    });
  for (auto& x : th) x.join();
  // contract the chain (an edge site from its complex-FP64 edge slot, as the read-outs do)
  std::vector<std::complex<double>> psi(1, 1.0);
  int chl = 1;
  for (int i = 0; i < n; ++i) {
    const int chr = bonds[i + 1];
    const int ei = edge_index(i, n, ew);
    const size_t rows = psi.size() / chl;
    std::vector<std::complex<double>> out(rows * 2 * chr);
    for (size_t r = 0; r < rows; ++r)
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < chr; ++c) {
          std::complex<double> acc = 0.0;
          for (int a = 0; a < chl; ++a) {
            const size_t off = (size_t)a * 2 * D + (size_t)b * D + c;
            const std::complex<double> e = ei >= 0 ? std::complex<double>(edge[(size_t)ei * SLOT + off].re, edge[(size_t)ei * SLOT + off].im)
                                                   : std::complex<double>(arena[(size_t)i * SLOT + off].re, arena[(size_t)i * SLOT + off].im);
            acc += psi[r * chl + a] * e;
          }
          out[(r * 2 + b) * chr + c] = acc;
        }
    psi.swap(out);
    chl = chr;
  }
  std::printf("%d %.17g %.17g %lld\n", inst->status, inst->drift, inst->trunc_w, (long long)inst->k_done);
  for (int l = 0; l <= n; ++l) std::printf("%d%c", bonds[l], l == n ? '\n' : ' ');
  for (auto& v : psi) std::printf("%.17g %.17g\n", v.real(), v.imag());
  std::free(inst);
  std::free(marked);
  std::free(bonds);
  std::free(arena);
  std::free(edge);
  std::free(bundle);
  std::free(queue);
  std::free(lds);
  std::free(circ);
  return 0;
}
