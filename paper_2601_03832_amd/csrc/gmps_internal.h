// Internal structures shared by the HIP kernels and the host runtime of libgmps.
#pragma once
#include <stdint.h>

namespace gmps {

// Device-side record of one Grover instance.
struct InstDev {
  int32_t n, M, cap, cls;  // qubits, marked count, bond cap, tile class
  int64_t marked_off;      // first marked index in the marked[] array
  int64_t site_off;        // complex-element offset of site 0's slot in the arena
  int64_t k_done;          // iterations applied since init
  int32_t status;          // GMPS_ST_* bits
  int32_t whole;           // pre-contracted path: the M oracle terms form one reflection
  double drift;            // largest |norm - 1| before a renormalisation
  double trunc_w;          // largest dropped-weight fraction of one truncation
  double flops64, flops32; // algorithmic flops spent so far
  int64_t warm_off;        // byte offset of this instance's first warm-start record
  int64_t edge_off;        // complex-FP64 offset of this instance's first edge slot
  int32_t ew;              // edge width: sites i < ew and i >= n - ew are edge sites
  int32_t pad_;
  int64_t circ_off;        // gate-level circuit: first gate of this instance's stream
  int64_t circ_len;        // gate-level circuit: gates in the stream
};

// Gate-level circuits (the Common method): one 32-bit word per gate, the gate type in bits
// 8..15 and the qubit (site) in bits 0..7; the n-controlled Z acts on every qubit.
enum : uint32_t { kGateH = 0u, kGateX = 1u, kGateMCZ = 2u };
__host__ __device__ constexpr uint32_t gate_word(uint32_t type, uint32_t q) { return (type << 8) | (q & 0xFFu); }

// Edge sites. A stored isometry changes the state by its rounding error d times the rest of
// the chain; the kernels fold the part of d inside the span of the stored vectors into the FP64
// carry, and the rest is orthogonal to every state whose support at that bond lies in that span.
// The Grover states (combinations of |s> and the M marked basis states) have supports of
// dimension up to M+1 at a bond, and the bond of site i is at most 2^min(i, n-i): within
// ew = ceil(log2(M+1)) sites of either end the stored span can be smaller than theirs, and a
// rounding error there would rotate the state at first order. Those sites (and always the
// norm-carrying end site) are therefore kept in complex FP64 in edge slots of their own, laid
// out like a site slot (D, 2, D); their site slots hold storage-type copies. Every other site
// (the bulk of the chain) is stored as complex64 on the mixed path.
__host__ __device__ constexpr int edge_width(int M) {
  int e = 1;
  while ((1 << e) < M + 1 && e < 31) ++e;
  return e;
}
__host__ __device__ constexpr int edge_count(int n, int ew) { return n <= 2 * ew ? n : 2 * ew; }
// edge slot of site i, or -1 for a bulk site
__host__ __device__ constexpr int edge_index(int i, int n, int ew) {
  return n <= 2 * ew ? i : (i < ew ? i : (i >= n - ew ? ew + (n - 1 - i) : -1));
}

// The Jacobi SVD at (reflection j, site i) starts from the unitary it produced at the same
// place in the previous iteration: the tile changes by O(theta) per iteration, so the
// warm start leaves an O(theta) off-diagonal and quadratic convergence needs ~2 sweeps.
// One record per (instance, reflection, site): the r x r unitary (FP64, stride KJMAX) and r.
constexpr int kWarmStride = 8;  // KJ <= 8 for every class
struct WarmRec {
  double u[kWarmStride * kWarmStride * 2];  // complex, row-major
  int32_t r;                                // dimension stored, 0 = none
  int32_t pad[3];
};

// A wave processes one bundle: up to kMaxBundle instances that share (class, n, M, k),
// one per lane group of G lanes.
constexpr int kMaxBundle = 8;
struct Bundle {
  int32_t inst[kMaxBundle];
  int32_t count;
  int32_t cls;
  int64_t k;
};

// Tile classes: CM is the largest bond after truncation and D = 2*CM the largest bond after
// a bond-2 MPO. The QR sweep keeps at most CM+1 columns (the rank bound of a tile after
// the MPO), so a QR tile has up to 2*(CM+1) rows: a lane group has G >= 2*CM+2 lanes. The
// SVD runs on M^H (up to 2*CM rows) over its own WS <= G lanes.
struct ClassCfg {
  int CM, G, WS;
};
constexpr int kNumClasses = 5;
constexpr ClassCfg kClasses[kNumClasses] = {{2, 8, 4}, {3, 8, 8}, {4, 16, 8}, {5, 16, 16}, {6, 16, 16}};
constexpr int kBondStride = 64;  // bonds[i * 64 + l], l = 0..n

// Team classes: one instance per team of TW threads (several teams share a 64-lane wave
// when TW < 64; a team of TW > 64 spans TW/64 waves of one workgroup). Inside a team the
// tile columns sit on column slots and the rows of a column are spread over the lanes of
// its slot, so column sums are short butterflies and all columns are updated at once.
struct WideCfg {
  int CM, TW;
};
constexpr int kWideBase = 8;  // class ids kWideBase + w select kWide[w]
constexpr int kNumWide = 6;
constexpr WideCfg kWide[kNumWide] = {{2, 16}, {3, 32}, {5, 64}, {8, 64}, {17, 192}, {32, 256}};
__host__ __device__ constexpr bool is_wide(int cls) { return cls >= kWideBase; }
__host__ __device__ constexpr int class_cm(int cls) {
  return cls >= kWideBase ? kWide[cls - kWideBase].CM : kClasses[cls].CM;
}
// Jacobi columns of a class (the QR rank bound CM+1, rounded up to even).
__host__ __device__ constexpr int class_kj(int CM) { return ((CM + 1) + 1) & ~1; }
// Doubles of one team-class warm-start record: r (as a double), a pad double, then the
// KJ x KJ complex unitary, row-major.
// Team classes with a pre-contracted reflection kernel (bond caps up to 17).
__host__ __device__ constexpr bool team_pc_class(int w) { return kWide[w].CM <= 17; }
// Team classes with the pipelined two-wave kernel (teams within one wave: bond caps up to 8).
__host__ __device__ constexpr bool team_pipe_class(int w) { return w >= 0 && kWide[w].TW <= 64; }
__host__ __device__ constexpr int64_t wide_warm_doubles(int CM) { return 2 + 2 * (int64_t)class_kj(CM) * class_kj(CM); }

// Elements of one site slot: (D, 2, D) with row stride 2*D and physical stride D.
__host__ __device__ constexpr int slot_elems(int CM) { return (2 * CM) * 2 * (2 * CM); }

struct QueueState {
  uint32_t next;      // next bundle to hand out
  int32_t nbundles;   // bundles in this launch
};

struct IterParams {
  InstDev* inst;
  const uint64_t* marked;
  int32_t* bonds;
  void* arena;
  const Bundle* bundles;
  QueueState* queue;
  double trunc_tol;  // relative singular-value cut of the truncation
  double skip_tol;   // relative column norm below which Jacobi leaves a column unrotated
  double rank_tol;   // relative trailing norm at which the QR sweep stops (numerical rank)
  int32_t max_sweeps;
  int32_t stoch_round;  // stochastic (1) or nearest (0) rounding of FP64 results stored as complex64
  void* warm;           // warm-start records (null: every Jacobi starts from the identity)
  void* edge;           // edge slots (complex FP64)
  const uint32_t* circuit;  // gate streams of the gate-level circuits (null: reflections)
};

}  // namespace gmps
