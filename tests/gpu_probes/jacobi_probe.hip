// Test probe, not part of the library: runs the team kernels' one-sided Jacobi (the in-wave
// variant for teams of up to 64 lanes, the LDS variant for wider teams) on caller-made tiles,
// one tile per team, in each team class's own shape, so that tests can check the properties the
// factorisation must have: J unitary, the rotated columns equal to M^H J, and those columns
// mutually orthogonal at convergence.
//
// Tiles are complex128 (re, im interleaved), 64 x 64 row-major with leading dimension 64, one
// per 4096 elements: tile t, row i, column c at t * 4096 + i * 64 + c. dims holds (rows, ncj) per
// tile; the kernel clamps rows to [0, the class's Jacobi rows] and ncj to an even number in
// [2, the class's Jacobi columns], so that any dims stay in bounds. Outputs: AJ (rows x ncj, the
// rotated columns), J (ncj x ncj) and the sweeps taken. All pointers are device pointers owned by
// the caller; the call is synchronous on the null stream and returns a hipError_t, or -1 for an
// unknown class.
#include <hip/hip_runtime.h>
#include "gmps_internal.h"
#include "gmps_team.h"

namespace {
using namespace gmps;
constexpr int kLd = 64, kTile = 64 * 64;

template <int W>
constexpr int probe_threads() { return TeamShape<kWide[W].CM, kWide[W].TW>::NT; }

template <int W>
__global__ __launch_bounds__(probe_threads<W>()) void jacobi_probe_kernel(
    const cd* A, const int* dims, cd* AJ, cd* J, int* sweeps, int ntiles, int max_sweeps) {
  constexpr int CM = kWide[W].CM, TW = kWide[W].TW;
  using T = TeamShape<CM, TW>;
  constexpr int PJ = T::PJ, RJ = T::RJ, RU = T::RU, KJ = T::KJ;
  constexpr int MAXR = T::D < PJ * RJ ? T::D : PJ * RJ;
  static_assert(MAXR <= kLd && KJ <= kLd, "a tile fits the probe's 64 x 64 layout");
  const int team = threadIdx.x / TW, tl = threadIdx.x % TW, base = threadIdx.x - tl;
  const int tile = blockIdx.x * T::TEAMS + team;
  const int tt = tile < ntiles ? tile : ntiles - 1;
  const int jc = tl / PJ, jh = tl % PJ;
  const int rows = min(max(dims[2 * tt], 0), MAXR);
  const int ncj = min(max(dims[2 * tt + 1] & ~1, 2), KJ);
  const cd* At = A + (size_t)tt * kTile;
  cd a[RJ], u[RU];
#pragma unroll
  for (int e = 0; e < RJ; ++e) {
    const int row = jh + PJ * e;
    a[e] = (row < rows && jc < ncj) ? At[row * kLd + jc] : cd{0.0, 0.0};
  }
#pragma unroll
  for (int e = 0; e < RU; ++e) u[e] = {(jh + PJ * e == jc && jc < ncj) ? 1.0 : 0.0, 0.0};
  int s;
  if constexpr (TW <= 64) {
    s = team_jacobi_wave<TW, PJ, RJ, RU>(a, u, base, jc, jh, ncj, kJacobiTol2, 1e-30, max_sweeps);
  } else {
    __shared__ cd XA[T::NBUF][KJ][PJ * RJ];
    __shared__ cd XU[T::NBUF][KJ][PJ * RU];
    __shared__ double XN[T::NBUF][KJ];
    __shared__ double colv[TW], colf[TW];
    s = team_jacobi_lds<PJ, RJ, RU, KJ, T::NBUF>(a, u, jc, jh, ncj, kJacobiTol2, 1e-30, max_sweeps, XA, XU, XN,
                                                 colv, colf);
  }
  if (tile >= ntiles) return;
  cd* AJt = AJ + (size_t)tile * kTile;
  cd* Jt = J + (size_t)tile * kTile;
#pragma unroll
  for (int e = 0; e < RJ; ++e) {
    const int row = jh + PJ * e;
    if (row < rows && jc < ncj) AJt[row * kLd + jc] = a[e];
  }
#pragma unroll
  for (int e = 0; e < RU; ++e) {
    const int row = jh + PJ * e;
    if (row < ncj && jc < ncj) Jt[row * kLd + jc] = u[e];
  }
  if (tl == 0) sweeps[tile] = s;
}

template <int W>
int launch(const cd* A, const int* dims, cd* AJ, cd* J, int* sweeps, int ntiles, int max_sweeps) {
  using T = TeamShape<kWide[W].CM, kWide[W].TW>;
  const int blocks = (ntiles + T::TEAMS - 1) / T::TEAMS;
  jacobi_probe_kernel<W><<<blocks, T::NT>>>(A, dims, AJ, J, sweeps, ntiles, max_sweeps);
  const hipError_t e = hipGetLastError();
  return e != hipSuccess ? (int)e : (int)hipDeviceSynchronize();
}
}  // namespace

extern "C" {
// Team class w (0..5: bond caps 2, 3, 5, 8, 17, 32); returns its Jacobi columns and rows.
int gmps_probe_jacobi_shape(int w, int* kj, int* maxrows) {
  switch (w) {
#define SHAPE(W)                                                                          \
  case W: {                                                                               \
    using T = TeamShape<kWide[W].CM, kWide[W].TW>;                                        \
    *kj = T::KJ;                                                                          \
    *maxrows = T::D < T::PJ * T::RJ ? T::D : T::PJ * T::RJ;                               \
    return 0;                                                                             \
  }
    SHAPE(0) SHAPE(1) SHAPE(2) SHAPE(3) SHAPE(4) SHAPE(5)
#undef SHAPE
    default: return -1;
  }
}

int gmps_probe_team_jacobi(int w, const double* A, const int* dims, double* AJ, double* J, int* sweeps, int ntiles,
                           int max_sweeps) {
  if (ntiles <= 0) return 0;
  const cd* a = reinterpret_cast<const cd*>(A);
  cd* aj = reinterpret_cast<cd*>(AJ);
  cd* j = reinterpret_cast<cd*>(J);
  switch (w) {
    case 0: return launch<0>(a, dims, aj, j, sweeps, ntiles, max_sweeps);
    case 1: return launch<1>(a, dims, aj, j, sweeps, ntiles, max_sweeps);
    case 2: return launch<2>(a, dims, aj, j, sweeps, ntiles, max_sweeps);
    case 3: return launch<3>(a, dims, aj, j, sweeps, ntiles, max_sweeps);
    case 4: return launch<4>(a, dims, aj, j, sweeps, ntiles, max_sweeps);
    case 5: return launch<5>(a, dims, aj, j, sweeps, ntiles, max_sweeps);
    default: return -1;
  }
}
}
