// Team iterate kernel of libgmps, device part: iterative Grover search on matrix product
// states (gfx950). Instantiated by gmps_team64.hip, gmps_team192.hip and gmps_team256.hip.
//
// One instance per team of TW threads. Teams of 16 or 32 threads share a 64-lane wave
// (a bundle of instances with the same n, M and k), a team of 192 or 256 threads spans
// the waves of one workgroup. Where the lane-group kernel keeps one tile row per lane and
// loops over columns, a team keeps the tile columns side by side:
//   QR layout      lane = PQ * slot + part (PQ = 4): slot c holds column c of the QR tile,
//                  its rows part, part + PQ, ... in registers (RQ of them).
//   Jacobi layout  lane = PJ * slot + part: slot c holds column c of M^H and column c of the
//                  accumulated unitary, rows strided by PJ.
// A column sum is then a butterfly over the PQ (PJ) lanes of a slot, and every column of a
// Householder update or a Jacobi round is processed at the same time. What one slot has to
// tell the others (a Householder vector, a Jacobi partner column, column norms for pivots
// and truncation) goes through LDS between barriers; all lanes of a team read the same LDS
// values and make the same team-wide decisions.
//
// The method is the one of the lane-group kernel (Section III-B): each reflection
// c0*I + c1*(P_0 x ... x P_{n-1}) is applied as a bond-2 MPO fused into a QR
// left-canonicalisation sweep, followed by a truncated-SVD sweep (one-sided Jacobi on
// M^H) and the renormalisation of site 0 after the diffusion. QR, SVD and norms are FP64;
// S (double or float) is the storage and contraction type.
#pragma once
#include "gmps_device.h"

namespace gmps {

template <int CM, int TW>
struct TeamShape {
  static constexpr int D = 2 * CM;                 // largest bond after a bond-2 MPO
  static constexpr int KQ = CM + 1;                // rank bound of a QR tile
  static constexpr int KJ = class_kj(CM);          // Jacobi columns (even)
  static constexpr int PQ = 4;                     // lanes per column slot, QR layout
  static constexpr int SQ = TW / PQ;               // column slots, QR layout
  static constexpr int RQ = (2 * KQ + PQ - 1) / PQ;
  static constexpr int PJ = (KJ * 16 <= TW) ? 16 : (KJ * 8 <= TW) ? 8 : (KJ * 4 <= TW) ? 4 : 2;
  static constexpr int RJ = (D + PJ - 1) / PJ;     // rows of M^H per lane
  static constexpr int RU = (KJ + PJ - 1) / PJ;    // rows of the Jacobi unitary per lane
  static constexpr int NT = TW < 64 ? 64 : TW;     // threads of the workgroup
  static constexpr int NBUF = CM >= 24 ? 1 : 2;    // Jacobi exchange buffers (LDS budget)
  static constexpr int TEAMS = NT / TW;
  static_assert(SQ >= D, "a QR tile column per slot");
  static_assert(KJ * PJ <= TW, "a Jacobi column per slot");
  static_assert(TW % 64 == 0 || 64 % TW == 0, "teams tile the workgroup");
  static_assert(PJ * RU >= KJ, "the warm start's Gram matrix fits the exchange buffer");
};

template <class S, int CM, int TW>
struct TeamLds {
  using T = TeamShape<CM, TW>;
  union {
    struct {                                  // QR sweep
      cd W[2][CM][2][CM];                     // staged MPO blocks [c0 A | c1 P A] of the site
      cd R[T::KQ][T::D];                      // R of the previous step, original column order
      cd V[T::KQ][T::PQ * T::RQ];             // Householder vectors of this step
      double tau[T::KQ];
    } q;
    struct {                                  // SVD sweep
      cd Q[T::KQ][2][T::KQ];                  // staged left-orthonormal site tensor
      cd Y[T::KQ][CM];                        // U Sigma of the previous step
      cd XA[T::NBUF][T::KJ][T::PJ * T::RJ];   // Jacobi partner exchange
      cd XU[T::NBUF][T::KJ][T::PJ * T::RU];   // (its first buffer also holds the Gram matrix
      double XN[T::NBUF][T::KJ];              //  of the warm start, before the Jacobi runs)
      cd W[T::KJ][T::KJ];                     // warm-start unitary
    } s;
  } u;
  double colv[TW];  // per-slot values (norms, singular values)
  double colf[TW];  // per-slot flags
  int32_t colr[TW];
  int32_t bond[kBondStride];
  int32_t rdim[kBondStride];
  // Q^H d of a compensated store: in the staging block when it holds KQ x KQ complex doubles,
  // else here
  static constexpr bool kZInW = sizeof(cd) * 4 * CM * CM >= sizeof(cd) * (CM + 1) * (CM + 1);
  cd zq[kZInW ? 1 : (CM + 1) * (CM + 1)];
  __device__ cd* zbuf() { return kZInW ? reinterpret_cast<cd*>(&u.q.W[0][0][0][0]) : zq; }
  // the kept rows and Z of a compensated truncation go into the (free) Jacobi exchange buffers
  static_assert(sizeof(u.s.XA) >= sizeof(cd) * 2 * CM * CM, "kept rows fit XA");
  static_assert(sizeof(u.s.XU) >= sizeof(cd) * CM * CM, "Z fits XU");
};

// LDS of a team's pre-contracted reflections, placed after the TeamLds of every team of the
// workgroup (launches of the pre-contracted kernels only).
template <int CM>
struct PcLds {
  cd ov[CM][CM];                // running overlap rows <p_t| psi>_{0..i} (double-buffered with
                                // the MPO block W[1], which these reflections leave unused)
  cd ovs[CM];                   // c1 <p_t|psi>
  uint32_t xbits[kBondStride];  // bit t of site i: qubit value of marked index t at site i
};


// Orders LDS and global-memory traffic of the workgroup: global stores of one wave are
// complete and visible to the others after it (site tensors written in one sweep are read
// by other waves in the next).
__device__ __forceinline__ void team_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ------------------------------------------------------------------ wave collectives
// A team that fits one wave (TW <= 64) exchanges values between its lanes without LDS
// round trips or barriers: butterflies over DPP / swizzle for sums and maxima (every lane
// ends with the same bits), ds_bpermute for reading another lane's register, and ballots.
__device__ __forceinline__ double shfl_f64(double v, int src_lane) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, lo);
  hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, hi);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ cd shfl_cd(cd v, int src_lane) { return {shfl_f64(v.re, src_lane), shfl_f64(v.im, src_lane)}; }

template <int G>
__device__ __forceinline__ double gmax(double v) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16 || G == 32, "group size");
  v = fmax(v, dpp_f64<0xB1>(v));
  if (G > 2) v = fmax(v, dpp_f64<0x4E>(v));
  if (G > 4) v = fmax(v, dpp_f64<0x141>(v));
  if (G > 8) v = fmax(v, dpp_f64<0x140>(v));
  if (G > 16) v = fmax(v, swap16_f64(v));
  return v;
}
// sum / maximum over the TW lanes of a team (TW <= 64, teams aligned to TW lanes)
template <int TW>
__device__ __forceinline__ double tsum(double v) {
  if constexpr (TW <= 32) {
    return gsum<TW>(v);
  } else {
    v = gsum<32>(v);
    return v + shfl_f64(v, __lane_id() ^ 32);
  }
}
template <int TW>
__device__ __forceinline__ double tmax(double v) {
  if constexpr (TW <= 32) {
    return gmax<TW>(v);
  } else {
    v = gmax<32>(v);
    return fmax(v, shfl_f64(v, __lane_id() ^ 32));
  }
}
// lanes of the team (first lane base) for which pred holds, as a wave lane mask
template <int TW>
__device__ __forceinline__ uint64_t tballot(bool pred, int base) {
  const uint64_t all = __ballot(pred);
  if constexpr (TW >= 64) return all;
  else return all & (((1ull << TW) - 1ull) << base);
}

// Jacobi rotation of the pair (i, j) with gamma = a_i^H a_j, |a_i|^2 = ni, |a_j|^2 = nj:
// with h = (nj - ni)/2 the rotation tangent is t = sign(h) |gamma| / (|h| + sqrt(h^2 + |gamma|^2)),
// the smaller root of the usual quadratic. Writing t = |gamma| r, the cosine 1/sqrt(1 + t^2) and
// s e^{i phi} = c r gamma involve no 1/|gamma|, and c^2 + |s|^2 = 1 to rounding however
// accurate r is (r only sets the angle), so r comes from the hardware estimates and one
// Newton step while c is refined to working precision. tg = t |gamma| is the squared norm
// the pair exchanges.
__device__ __forceinline__ void jacobi_rotation(cd g, double g2, double ni, double nj, double* cs, cd* se, double* tg) {
  const double h = 0.5 * (nj - ni);
  const double q2 = fma(h, h, g2);
  const double den = fabs(h) + q2 * __builtin_amdgcn_rsq(q2);
  double rr = __builtin_amdgcn_rcp(den);
  rr = fma(rr, fma(-den, rr, 1.0), rr);
  rr = copysign(rr, h);
  const double c = rsqrt_acc(fma(g2 * rr, rr, 1.0));
  *cs = c;
  *se = {c * rr * g.re, c * rr * g.im};
  *tg = g2 * rr;
}

// One term of the Gram element of a Jacobi pair, accumulated as conj(own) other. Both slots of
// the pair must arrive at the same gamma = conj(x) y (x the lower column) to the bit: the pair's
// 2x2 is unitary only if its two halves come from one rotation, and for near-equal norms and
// small |gamma| a rounding difference between the halves turns the phase by eps |x||y| / |gamma|.
// The real part is symmetric in the operands even when contracted to FMAs; the imaginary part
// is formed from two rounded products, so that swapping the operands negates it exactly. The
// upper slot's sum is then exactly conj(gamma), and it flips the sign of the imaginary part.
__device__ __forceinline__ void gram_acc(cd& g, cd own, cd oth) {
  g.re = fma(own.re, oth.re, fma(own.im, oth.im, g.re));
  double t;
  {
#pragma clang fp contract(off)
    t = own.re * oth.im - own.im * oth.re;
  }
  g.im = g.im + t;
}

// ----------------------------------------------------------------------- prefetched loads
// The site tensor A_i of the QR sweep, loaded one site ahead as (a, b) pairs with both
// physical values, so that staging can write both blocks of the bond-2 MPO applied to it:
// W[0][a][s][b] = c0 A[a][s][b] and W[1][a][s][b] = c1 (P A)[a][s][b], with (c0, c1) the
// reflection's coefficients at the last site and (1, 1) elsewhere. The contraction with R
// then reads W directly. Loads are unconditional, masked when staged (see APrefetch).
template <class S, int CM, int TW>
struct TeamAPre {
  static constexpr int NE = (CM * CM + TW - 1) / TW;
  cx<S> v0[NE], v1[NE];
  int chl_, chr_;
  __device__ __forceinline__ void load(const cx<S>* slot, int tl, int chl, int chr) {
    constexpr int D = 2 * CM;
    chl_ = chl;
    chr_ = chr;
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      const int ec = e < CM * CM ? e : CM * CM - 1;
      const int a = ec / CM, b = ec % CM;
      v0[t] = slot[a * 2 * D + b];
      v1[t] = slot[a * 2 * D + D + b];
    }
  }
  __device__ __forceinline__ void stage(cx<S> (*W)[CM][2][CM], int tl, bool diff, int xb, S c0, S c1) const {
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      if (e < CM * CM) {
        const int a = e / CM, b = e % CM;
        const bool ok = a < chl_ && b < chr_;
        const cx<S> a0 = ok ? v0[t] : czero<S>(), a1 = ok ? v1[t] : czero<S>();
        W[0][a][0][b] = c0 * a0;
        W[0][a][1][b] = c0 * a1;
        W[1][a][0][b] = c1 * proj_apply<S>(a0, a1, 0, diff, xb);
        W[1][a][1][b] = c1 * proj_apply<S>(a0, a1, 1, diff, xb);
      }
    }
  }
  // staged in complex FP64: from the prefetched values or, for an edge site (es non-null), from
  // its complex-FP64 edge slot
  __device__ __forceinline__ void stage64(cd (*W)[CM][2][CM], const cd* es, int tl, bool diff, int xb, double c0,
                                          double c1) const {
    constexpr int D = 2 * CM;
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      if (e < CM * CM) {
        const int a = e / CM, b = e % CM;
        const bool ok = a < chl_ && b < chr_;
        cd a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
        if (ok) {
          a0 = es ? es[a * 2 * D + b] : up(v0[t]);
          a1 = es ? es[a * 2 * D + D + b] : up(v1[t]);
        }
        W[0][a][0][b] = c0 * a0;
        W[0][a][1][b] = c0 * a1;
        W[1][a][0][b] = c1 * proj_apply<double>(a0, a1, 0, diff, xb);
        W[1][a][1][b] = c1 * proj_apply<double>(a0, a1, 1, diff, xb);
      }
    }
  }
  // stage64 for a gate-level circuit: the pending single-qubit product u (real 2x2, row-major)
  // acts on the physical index first, then the projector |xb><xb| of the n-controlled Z
  __device__ __forceinline__ void stage64u(cd (*W)[CM][2][CM], const cd* es, int tl, const double* u, int xb,
                                           double c0, double c1) const {
    constexpr int D = 2 * CM;
    const double u00 = u[0], u01 = u[1], u10 = u[2], u11 = u[3];
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      if (e < CM * CM) {
        const int a = e / CM, b = e % CM;
        const bool ok = a < chl_ && b < chr_;
        cd a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
        if (ok) {
          a0 = es ? es[a * 2 * D + b] : up(v0[t]);
          a1 = es ? es[a * 2 * D + D + b] : up(v1[t]);
        }
        const cd b0 = {u00 * a0.re + u01 * a1.re, u00 * a0.im + u01 * a1.im};
        const cd b1 = {u10 * a0.re + u11 * a1.re, u10 * a0.im + u11 * a1.im};
        W[0][a][0][b] = c0 * b0;
        W[0][a][1][b] = c0 * b1;
        W[1][a][0][b] = c1 * proj_apply<double>(b0, b1, 0, false, xb);
        W[1][a][1][b] = c1 * proj_apply<double>(b0, b1, 1, false, xb);
      }
    }
  }
  __device__ __forceinline__ void stage_a64(cd (*W)[CM][2][CM], const cd* es, int tl, double c0) const {
    constexpr int D = 2 * CM;
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      if (e < CM * CM) {
        const int a = e / CM, b = e % CM;
        const bool ok = a < chl_ && b < chr_;
        cd a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
        if (ok) {
          a0 = es ? es[a * 2 * D + b] : up(v0[t]);
          a1 = es ? es[a * 2 * D + D + b] : up(v1[t]);
        }
        W[0][a][0][b] = c0 * a0;
        W[0][a][1][b] = c0 * a1;
      }
    }
  }
  // the site tensor alone, scaled by c0 (pre-contracted reflections)
  __device__ __forceinline__ void stage_a(cx<S> (*W)[CM][2][CM], int tl, S c0) const {
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      if (e < CM * CM) {
        const int a = e / CM, b = e % CM;
        const bool ok = a < chl_ && b < chr_;
        W[0][a][0][b] = c0 * (ok ? v0[t] : czero<S>());
        W[0][a][1][b] = c0 * (ok ? v1[t] : czero<S>());
      }
    }
  }
};

// The Q_i tile (r_i, 2, r_{i+1}) of the SVD sweep, loaded by the team one site ahead.
template <class S, int KQ, int CM, int TW>
struct TeamQPre {
  static constexpr int NE = (KQ * 2 * KQ + TW - 1) / TW;
  cx<S> v[NE];
  int ri_, rn_;
  // unconditional loads from clamped indices, masked when staged (see APrefetch)
  __device__ __forceinline__ void load(const cx<S>* slot, int tl, int ri, int rn) {
    constexpr int D = 2 * CM;
    ri_ = ri;
    rn_ = rn;
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      const int ec = e < KQ * 2 * KQ ? e : KQ * 2 * KQ - 1;
      const int a = ec / (2 * KQ), s = (ec / KQ) & 1, b = ec % KQ;
      v[t] = slot[a * 2 * D + s * D + b];
    }
  }
  // staged in the storage type, or up-converted to complex FP64 (T = double)
  template <class T>
  __device__ __forceinline__ void stage(cx<T>* lds_q, int tl) const {
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      const int a = e / (2 * KQ), b = e % KQ;
      if (e < KQ * 2 * KQ) lds_q[e] = (a < ri_ && b < rn_) ? cvt<T>(v[t]) : czero<T>();
    }
  }
};

// A warm-start record: r (as a double), a pad double, then the KJ x KJ unitary. w is always
// readable (without warm starts it points at a dummy record and on is false); the loads are
// unconditional, masked when staged (see APrefetch).
template <int KJ, int TW>
struct TeamWPre {
  static constexpr int NE = (KJ * KJ + TW - 1) / TW;
  cd v[NE];
  double r0;
  bool on_;
  int ncj_;
  __device__ __forceinline__ void load(const double* w, bool on, int tl, int ncj) {
    on_ = on;
    ncj_ = ncj;
    r0 = w[0];
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      const int ec = e < KJ * KJ ? e : KJ * KJ - 1;
      v[t] = {w[2 + 2 * ec], w[3 + 2 * ec]};
    }
  }
  // the dimension the record holds (0 when warm starts are off)
  __device__ __forceinline__ int r() const { return on_ ? (int)r0 : 0; }
  __device__ __forceinline__ void stage(cd* lds_w, int tl) const {
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      const int ra = e / KJ, ca = e % KJ;
      if (e < KJ * KJ) lds_w[e] = (ra < ncj_ && ca < ncj_) ? v[t] : cd{0.0, 0.0};
    }
  }
};

// ------------------------------------------------------------------------------- QR
// Householder QR of the m x c tile X in the QR layout (x[e] = X[part + PQ*e][slot], zero
// outside the tile), with the rank stop and the projector-block pivoting of the lane-group
// kernel: columns below npiv (the A block, full rank) are eliminated in their own order;
// from step npiv on, the remaining column with the largest residual norm is taken, and
// the factorisation ends when that norm falls to rank2 * ||X||^2 or after min(m, c, KQ)
// steps. Columns never move: when it returns, x[] of every slot holds its column of R
// (rows below the rank k, original column order) and q[] of slots < k holds that column
// of the thin Q, so X = Q R + E with ||E||^2 = *dropped * ||X||^2. Returns k.
template <int PQ, int RQ, int KQ>
__device__ __forceinline__ int team_qr_lds(cd (&x)[RQ], cd (&q)[RQ], int qc, int qh, int m, int c, int npiv,
                                       double rank2, double* dropped, cd (*V)[PQ * RQ], double* tau,
                                       double* colv) {
  const bool colok = qc < c;
  double p0 = 0.0;
#pragma unroll
  for (int e = 0; e < RQ; ++e) p0 += norm2(x[e]);
  p0 = gsum<PQ>(p0);
  if (qh == 0) colv[qc] = colok ? p0 : 0.0;
  lds_sync();
  double t0 = 0.0;
  for (int k = 0; k < c; ++k) t0 += colv[k];
  const int kmax = min(min(m, c), KQ);
  int kr = kmax;
  bool used = false;
  lds_sync();
  for (int j = 0; j < kmax; ++j) {
    int p = j;
    if (j >= npiv) {
      double rn = 0.0;
#pragma unroll
      for (int e = 0; e < RQ; ++e) rn += (qh + PQ * e >= j) ? norm2(x[e]) : 0.0;
      rn = gsum<PQ>(rn);
      if (qh == 0) colv[qc] = (colok && !used) ? rn : -1.0;
      lds_sync();
      double best = -1.0;
      for (int k = 0; k < c; ++k) {
        const double v = colv[k];
        if (v > best) {
          best = v;
          p = k;
        }
      }
      if (best <= rank2 * t0) {
        kr = j;
        break;
      }
    }
    const bool piv = qc == p;
    cd xj = {0.0, 0.0};
    double sub = 0.0;
#pragma unroll
    for (int e = 0; e < RQ; ++e) {
      const int row = qh + PQ * e;
      if (row == j) xj = x[e];
      sub += (row > j && row < m) ? norm2(x[e]) : 0.0;
    }
    const cd alpha = gsum<PQ>(xj);
    sub = gsum<PQ>(sub);
    const double a2 = norm2(alpha);
    const bool refl = sub > 0.0;
    const double ra = a2 > 0.0 ? rsqrt_acc(a2) : 0.0;
    const double aa = a2 * ra;                          // |alpha|
    const double n2 = a2 + sub;
    const double nrm = refl ? n2 * rsqrt_acc(n2) : aa;  // norm of the column from row j down
    const cd ph = a2 > 0.0 ? cd{alpha.re * ra, alpha.im * ra} : cd{1.0, 0.0};
    const cd beta = {-ph.re * nrm, -ph.im * nrm};
    const double t = refl ? rcp_acc(nrm * (nrm + aa)) : 0.0;
    if (piv) {
#pragma unroll
      for (int e = 0; e < RQ; ++e) {
        const int row = qh + PQ * e;
        V[j][row] = !refl ? cd{0.0, 0.0} : (row == j ? alpha - beta : ((row > j && row < m) ? x[e] : cd{0.0, 0.0}));
        if (refl) x[e] = (row == j) ? beta : ((row > j) ? cd{0.0, 0.0} : x[e]);
      }
      if (qh == 0) tau[j] = t;
      used = true;
    }
    lds_sync();
    if (!piv && !used && colok) {
      const double tj = tau[j];
      if (tj != 0.0) {
        cd v[RQ];
        cd w = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < RQ; ++e) {
          v[e] = V[j][qh + PQ * e];
          w = w + cmulc(v[e], x[e]);
        }
        w = gsum<PQ>(w);
        const cd tw = tj * w;
#pragma unroll
        for (int e = 0; e < RQ; ++e) x[e] = x[e] - v[e] * tw;
      }
    }
  }
  lds_sync();
  double tr = 0.0;
#pragma unroll
  for (int e = 0; e < RQ; ++e) {
    const int row = qh + PQ * e;
    tr += (row >= kr && row < m) ? norm2(x[e]) : 0.0;
  }
  tr = gsum<PQ>(tr);
  if (qh == 0) colv[qc] = (colok && !used) ? tr : 0.0;
  lds_sync();
  double tk = 0.0;
  for (int k = 0; k < c; ++k) tk += colv[k];
  *dropped = t0 > 0.0 ? tk / t0 : 0.0;
  // thin Q = H_0 ... H_{k-1} [I; 0]; column t is untouched by H_j for j > t
#pragma unroll
  for (int e = 0; e < RQ; ++e) q[e] = {(qh + PQ * e == qc && qc < kr) ? 1.0 : 0.0, 0.0};
  for (int j = kr - 1; j >= 0; --j) {
    if (qc >= j && qc < kr) {
      const double tj = tau[j];
      if (tj != 0.0) {
        cd v[RQ];
        cd w = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < RQ; ++e) {
          v[e] = V[j][qh + PQ * e];
          w = w + cmulc(v[e], q[e]);
        }
        w = gsum<PQ>(w);
        const cd tw = tj * w;
#pragma unroll
        for (int e = 0; e < RQ; ++e) q[e] = q[e] - v[e] * tw;
      }
    }
  }
  return kr;
}

// ---------------------------------------------------------------------------- Jacobi SVD
// One-sided Jacobi on the first ncj (even) columns of a tile in the Jacobi layout
// (a[e] = row part + PJ*e of this slot's column), accumulating the unitary (u[e], same
// layout). Same rotation, skip and stopping rules as the lane-group kernel's jacobi_fixed;
// in round r of the round-robin schedule every slot meets its partner: the pair exchanges
// columns through LDS, both members form the same inner product to the bit (gram_acc), and
// each applies its half of the rotation to its own column. Returns the sweeps.
template <int PJ, int RJ, int RU, int KJ, int NBUF>
__device__ __forceinline__ int team_jacobi_lds(cd (&a)[RJ], cd (&u)[RU], int jc, int jh, int ncj, double tol2,
                                           double skip2, int max_sweeps, cd (*XA)[KJ][PJ * RJ],
                                           cd (*XU)[KJ][PJ * RU], double (*XN)[KJ], double* colv, double* colf) {
  const bool colok = jc < ncj;
  const int lastc = ncj - 1;
  int sweeps = 0;
  bool more = true;
  while (more && sweeps < max_sweeps) {
    ++sweeps;
    double nrm = 0.0;
#pragma unroll
    for (int e = 0; e < RJ; ++e) nrm += norm2(a[e]);
    nrm = gsum<PJ>(nrm);
    if (jh == 0) colv[jc] = colok ? nrm : 0.0;
    lds_sync();
    double amax = 0.0;
    for (int k = 0; k < ncj; ++k) amax = fmax(amax, colv[k]);
    const double floor2 = skip2 * amax;
    bool mv = false;
    for (int r = 0; r < lastc; ++r) {
      const int buf = NBUF == 2 ? (r & 1) : 0;
      const int pt = jc == lastc ? r : (jc == r ? lastc : (2 * r - jc + 2 * lastc) % lastc);
      if (colok) {
#pragma unroll
        for (int e = 0; e < RJ; ++e) XA[buf][jc][jh + PJ * e] = a[e];
#pragma unroll
        for (int e = 0; e < RU; ++e) XU[buf][jc][jh + PJ * e] = u[e];
        if (jh == 0) XN[buf][jc] = nrm;
      }
      lds_sync();
      cd b[RJ], ub[RU];
      double nb = 0.0;
      if (colok) {
#pragma unroll
        for (int e = 0; e < RJ; ++e) b[e] = XA[buf][pt][jh + PJ * e];
#pragma unroll
        for (int e = 0; e < RU; ++e) ub[e] = XU[buf][pt][jh + PJ * e];
        nb = XN[buf][pt];
      }
      // a single buffer is rewritten next round; every wave of the team takes this barrier
      if (NBUF == 1) lds_sync();
      if (colok) {
        const bool lo = jc < pt;
        cd g = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < RJ; ++e) gram_acc(g, a[e], b[e]);
        g = gsum<PJ>(g);
        if (!lo) g.im = -g.im;
        const double ni = lo ? nrm : nb, nj = lo ? nb : nrm;
        const double g2 = norm2(g);
        const double ab = ni * nj;
        if (g2 > tol2 * ab && fmin(ni, nj) > floor2 && g2 > 1e-300) {
          mv |= g2 > 1e-20 * ab;
          double cs, tg;
          cd se;
          jacobi_rotation(g, g2, ni, nj, &cs, &se, &tg);
          // lower column x: c x - conj(se) y; upper column y: se x + c y
          if (lo) {
#pragma unroll
            for (int e = 0; e < RJ; ++e) {
              const cd x0 = a[e], y0 = b[e];
              a[e].re = fma(cs, x0.re, fma(-se.re, y0.re, -se.im * y0.im));
              a[e].im = fma(cs, x0.im, fma(-se.re, y0.im, se.im * y0.re));
            }
#pragma unroll
            for (int e = 0; e < RU; ++e) {
              const cd x0 = u[e], y0 = ub[e];
              u[e].re = fma(cs, x0.re, fma(-se.re, y0.re, -se.im * y0.im));
              u[e].im = fma(cs, x0.im, fma(-se.re, y0.im, se.im * y0.re));
            }
          } else {
#pragma unroll
            for (int e = 0; e < RJ; ++e) {
              const cd x0 = b[e], y0 = a[e];
              a[e].re = fma(cs, y0.re, fma(se.re, x0.re, -se.im * x0.im));
              a[e].im = fma(cs, y0.im, fma(se.re, x0.im, se.im * x0.re));
            }
#pragma unroll
            for (int e = 0; e < RU; ++e) {
              const cd x0 = ub[e], y0 = u[e];
              u[e].re = fma(cs, y0.re, fma(se.re, x0.re, -se.im * x0.im));
              u[e].im = fma(cs, y0.im, fma(se.re, x0.im, se.im * x0.re));
            }
          }
          nrm = lo ? nrm - tg : nrm + tg;
        }
      }
    }
    if (jh == 0) colf[jc] = (colok && mv) ? 1.0 : 0.0;
    lds_sync();
    more = false;
    for (int k = 0; k < ncj; ++k) more |= colf[k] != 0.0;
  }
  return sweeps;
}

// The lower column x of a rotated pair becomes c x - conj(se) y, the upper column y becomes
// se x + c y; own is this slot's column, oth the partner's.
// Both are own' = c own + f oth with f = -conj(se) for the lower column and se for the upper.
template <int R>
__device__ __forceinline__ void rot_apply(cd (&own)[R], const cd (&oth)[R], bool lo, double cs, cd se) {
  const double fre = lo ? -se.re : se.re, fim = se.im;
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const cd o = own[e], p = oth[e];
    own[e].re = fma(cs, o.re, fma(fre, p.re, -fim * p.im));
    own[e].im = fma(cs, o.im, fma(fre, p.im, fim * p.re));
  }
}

// team_qr_lds for a team inside one wave: the same factorisation, with the pivot column
// read from its slot's lanes by ds_bpermute (every slot then forms the same Householder
// vector itself), the pivot search as a team maximum plus a ballot, and column sums as
// butterflies, so the steps need neither LDS round trips nor barriers. Only the pivot
// slot writes its Householder vector to V, for the formation of Q at the end.
template <int TW, int PQ, int RQ, int KQ, bool WL = false>
__device__ __forceinline__ int team_qr_wave(cd (&x)[RQ], cd (&q)[RQ], int base, int qc, int qh, int m, int c,
                                            int npiv, double rank2, double* dropped, cd (*V)[PQ * RQ],
                                            double* tau) {
  const bool colok = qc < c;
  double p0 = 0.0;
#pragma unroll
  for (int e = 0; e < RQ; ++e) p0 += norm2(x[e]);
  const double t0 = tsum<TW>(colok ? p0 : 0.0);
  const int kmax = min(min(m, c), KQ);
  int kr = kmax;
  bool used = false;
  for (int j = 0; j < kmax; ++j) {
    int p = j;
    if (j >= npiv) {
      double rn = 0.0;
#pragma unroll
      for (int e = 0; e < RQ; ++e) rn += (qh + PQ * e >= j) ? norm2(x[e]) : 0.0;
      rn = gsum<PQ>(rn);
      const double key = (colok && !used) ? rn : -1.0;
      const double best = tmax<TW>(key);
      // the lowest slot attaining the maximum
      const uint64_t hit = tballot<TW>(qh == 0 && key == best, base);
      if (hit) p = (__ffsll((long long)hit) - 1 - base) / PQ;
      if (best <= rank2 * t0) {
        kr = j;
        break;
      }
    }
    cd v[RQ];
    const int src = base + p * PQ + qh;
#pragma unroll
    for (int e = 0; e < RQ; ++e) v[e] = shfl_cd(x[e], src);
    cd xj = {0.0, 0.0};
    double sub = 0.0;
#pragma unroll
    for (int e = 0; e < RQ; ++e) {
      const int row = qh + PQ * e;
      if (row == j) xj = v[e];
      sub += (row > j && row < m) ? norm2(v[e]) : 0.0;
    }
    const cd alpha = gsum<PQ>(xj);
    sub = gsum<PQ>(sub);
    const double a2 = norm2(alpha);
    const bool refl = sub > 0.0;
    const double ra = a2 > 0.0 ? rsqrt_acc(a2) : 0.0;
    const double aa = a2 * ra;                          // |alpha|
    const double n2 = a2 + sub;
    const double nrm = refl ? n2 * rsqrt_acc(n2) : aa;  // norm of the column from row j down
    const cd ph = a2 > 0.0 ? cd{alpha.re * ra, alpha.im * ra} : cd{1.0, 0.0};
    const cd beta = {-ph.re * nrm, -ph.im * nrm};
    const double t = refl ? rcp_acc(nrm * (nrm + aa)) : 0.0;
    // reflector rows (rows >= m of the tile are zero; with no reflection t = 0 and v is unused)
#pragma unroll
    for (int e = 0; e < RQ; ++e) {
      const int row = qh + PQ * e;
      v[e] = row > j ? v[e] : (row == j ? alpha - beta : cd{0.0, 0.0});
    }
    // every slot of the trailing columns, the pivot included, applies H_j (no divergence);
    // the pivot column becomes (beta, ~0, ...) and is not touched again
    {
      cd w = {0.0, 0.0};
#pragma unroll
      for (int e = 0; e < RQ; ++e) w = w + cmulc(v[e], x[e]);
      w = gsum<PQ>(w);
      const cd tw = (!used && colok) ? t * w : cd{0.0, 0.0};
#pragma unroll
      for (int e = 0; e < RQ; ++e) x[e] = x[e] - v[e] * tw;
    }
    const bool piv = qc == p;
    if (piv) {
#pragma unroll
      for (int e = 0; e < RQ; ++e) V[j][qh + PQ * e] = v[e];
      if (qh == 0) tau[j] = t;
    }
    used = used || piv;
  }
  double tr = 0.0;
#pragma unroll
  for (int e = 0; e < RQ; ++e) {
    const int row = qh + PQ * e;
    tr += (row >= kr && row < m) ? norm2(x[e]) : 0.0;
  }
  const double tk = tsum<TW>((colok && !used) ? tr : 0.0);
  *dropped = t0 > 0.0 ? tk / t0 : 0.0;
  // V and tau of every step, read by all slots below (WL: the team is the whole wave and
  // the workgroup's other wave runs other code, so no workgroup barrier)
  if constexpr (WL) wave_sync(); else lds_sync();
#pragma unroll
  for (int e = 0; e < RQ; ++e) q[e] = {(qh + PQ * e == qc && qc < kr) ? 1.0 : 0.0, 0.0};
  for (int j = kr - 1; j >= 0; --j) {
    if (qc >= j && qc < kr) {
      const double tj = tau[j];
      if (tj != 0.0) {
        cd v[RQ];
        cd w = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < RQ; ++e) {
          v[e] = V[j][qh + PQ * e];
          w = w + cmulc(v[e], q[e]);
        }
        w = gsum<PQ>(w);
        const cd tw = tj * w;
#pragma unroll
        for (int e = 0; e < RQ; ++e) q[e] = q[e] - v[e] * tw;
      }
    }
  }
  return kr;
}

// team_jacobi_lds for a team inside one wave: partners read each other's columns with
// ds_bpermute, the column maximum and the continue flag are team reductions.
template <int TW, int PJ, int RJ, int RU>
// jstop: another sweep follows while some rotation of the sweep had a relative squared
// off-diagonal above it.
__device__ __forceinline__ int team_jacobi_wave(cd (&a)[RJ], cd (&u)[RU], int base, int jc, int jh, int ncj,
                                                double tol2, double skip2, int max_sweeps, double jstop = 1e-20) {
  const bool colok = jc < ncj;
  const int lastc = ncj - 1;
  int sweeps = 0;
  bool more = true;
  while (more && sweeps < max_sweeps) {
    ++sweeps;
    double nrm = 0.0;
#pragma unroll
    for (int e = 0; e < RJ; ++e) nrm += norm2(a[e]);
    nrm = gsum<PJ>(nrm);
    const double floor2 = skip2 * tmax<TW>(colok ? nrm : 0.0);
    bool mv = false;
    // round r: slot lastc meets r, slot r meets lastc, slot c meets (2r - c) mod lastc
    int t2 = colok && jc < lastc ? (lastc - jc) % lastc : 0;
    for (int r = 0; r < lastc; ++r) {
      const int pt = !colok ? jc : (jc == lastc ? r : (jc == r ? lastc : t2));
      t2 += 2;
      if (t2 >= lastc) t2 -= lastc;
      const int src = base + pt * PJ + jh;
      cd b[RJ], ub[RU];
#pragma unroll
      for (int e = 0; e < RJ; ++e) b[e] = shfl_cd(a[e], src);
#pragma unroll
      for (int e = 0; e < RU; ++e) ub[e] = shfl_cd(u[e], src);
      const double nb = shfl_f64(nrm, src);
      if (colok) {
        const bool lo = jc < pt;
        cd g = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < RJ; ++e) gram_acc(g, a[e], b[e]);
        g = gsum<PJ>(g);
        if (!lo) g.im = -g.im;
        const double ni = lo ? nrm : nb, nj = lo ? nb : nrm;
        const double g2 = norm2(g);
        const double ab = ni * nj;
        if (g2 > tol2 * ab && fmin(ni, nj) > floor2 && g2 > 1e-300) {
          mv |= g2 > jstop * ab;
          double cs, tg;
          cd se;
          jacobi_rotation(g, g2, ni, nj, &cs, &se, &tg);
          rot_apply<RJ>(a, b, lo, cs, se);
          rot_apply<RU>(u, ub, lo, cs, se);
          nrm = lo ? nrm - tg : nrm + tg;
        }
      }
    }
    more = tballot<TW>(mv, base) != 0ull;
  }
  return sweeps;
}


// ------------------------------------------------------------- compensated complex64 stores
// On the mixed path every arithmetic step is FP64 and only the isometries (all sites but the
// norm-carrying end site, which the centre record keeps in FP64) are stored as complex64. A
// stored isometry changes the state by its rounding error d times the rest of the chain. The
// part of d inside the span of the stored vectors is folded into the FP64 carry that moves on;
// the part outside that span is orthogonal to every state whose support at this bond lies in it,
// as the Grover states' supports do, so it does not rotate the state within their span and
// reaches the marked probability only at second order. Both helpers take workgroup barriers:
// every thread of the workgroup calls them.

// Thin Q of a QR step (QR layout: slot qc holds column qc, q[] in FP64, qs[] as stored): the
// carry R (RB, rows < kr, columns < Dr) becomes R - (Q^H d) R. QB [KQ][PQ*RQ] and ZB [KQ*KQ]
// are LDS scratch.
template <int PQ, int RQ, int KQ, int DR, class S>
__device__ __forceinline__ void comp_store_cols(const cd (&q)[RQ], const cx<S> (&qs)[RQ], int qc, int qh, int kr,
                                                int Dr, cd (*QB)[PQ * RQ], cd* ZB, cd (*RB)[DR]) {
  cd dq[RQ];
#pragma unroll
  for (int e = 0; e < RQ; ++e) dq[e] = up(qs[e]) - q[e];
  lds_sync();
  if (qc < kr) {
#pragma unroll
    for (int e = 0; e < RQ; ++e) QB[qc][qh + PQ * e] = q[e];
  }
  lds_sync();
  for (int a = 0; a < kr; ++a) {
    cd z = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < RQ; ++e) z = z + cmulc(QB[a][qh + PQ * e], dq[e]);
    z = gsum<PQ>(z);
    if (qh == 0 && qc < kr) ZB[a * KQ + qc] = z;
  }
  lds_sync();
  cd corr[RQ];
#pragma unroll
  for (int e = 0; e < RQ; ++e) {
    const int row = qh + PQ * e;
    cd cz = {0.0, 0.0};
    if (qc < Dr && row < kr)
      for (int b = 0; b < kr; ++b) cz = cfma(cz, ZB[row * KQ + b], RB[b][qc]);
    corr[e] = cz;
  }
  lds_sync();
  if (qc < Dr) {
#pragma unroll
    for (int e = 0; e < RQ; ++e) {
      const int row = qh + PQ * e;
      if (row < kr) RB[row][qc] = RB[row][qc] - corr[e];
    }
  }
}

// Kept vectors of a truncation (Jacobi layout: the slot kept at position pos holds v_pos in wv[],
// its stored value in vs[], and its column of the carry Y (rows jh + PJ e < ny) in yv[]): the
// carry becomes Y - Y Z with Z[p][q] = <v_q | d_p>. WB [CM*2CM] and ZT [CM*CM] are LDS scratch;
// Y holds the carry and is rewritten by the caller from yv[].
template <int PJ, int RJ, int RU, int CM, int KY, class S>
__device__ __forceinline__ void comp_store_rows(const cd (&wv)[RJ], const cx<S> (&vs)[RJ], cd (&yv)[RU], bool keep,
                                                int pos, int jh, int c, int ny, int chi, cd* WB, cd* ZT,
                                                cd (*Y)[KY]) {
  lds_sync();
  if (keep) {
#pragma unroll
    for (int e = 0; e < RJ; ++e) {
      const int row = jh + PJ * e;
      if (row < c) WB[pos * 2 * CM + row] = wv[e];
    }
#pragma unroll
    for (int e = 0; e < RU; ++e) {
      const int row = jh + PJ * e;
      if (row < ny) Y[row][pos] = yv[e];
    }
  }
  lds_sync();
  for (int q = 0; q < chi; ++q) {
    cd z = {0.0, 0.0};
#pragma unroll
    for (int e = 0; e < RJ; ++e) {
      const int row = jh + PJ * e;
      if (row < c) z = z + cmulc(WB[q * 2 * CM + row], up(vs[e]) - wv[e]);
    }
    z = gsum<PJ>(z);
    if (keep && jh == 0) ZT[pos * CM + q] = z;
  }
  lds_sync();
#pragma unroll
  for (int e = 0; e < RU; ++e) {
    const int row = jh + PJ * e;
    cd cz = {0.0, 0.0};
    if (keep && row < ny)
      for (int p = 0; p < chi; ++p) cz = cfma(cz, Y[row][p], ZT[p * CM + pos]);
    yv[e] = yv[e] - cz;
  }
  lds_sync();
}

// ------------------------------------------------------------------------------- one team
// Gate-level circuits (the Common method): per team, the product of the single-qubit gates each
// qubit has received since its site was last staged. H and X are real, so the products are real
// 2x2 matrices (row-major). The block sits after the workgroup's TeamLds blocks.
struct CircLds {
  double U[kBondStride][4];
};

template <class S, int CM, int TW>
__device__ void run_team(const IterParams& P, const Bundle* bdp, char* lds_base) {
  using T = TeamShape<CM, TW>;
  constexpr int D = T::D, KQ = T::KQ, KJ = T::KJ;
  constexpr int PQ = T::PQ, RQ = T::RQ, PJ = T::PJ, RJ = T::RJ, RU = T::RU;
  constexpr int SLOT = slot_elems(CM);
  constexpr bool kMixed = sizeof(S) == sizeof(float);
  constexpr int64_t WREC = wide_warm_doubles(CM);
  const int tid = threadIdx.x;
  const int team = tid / TW;
  const int tl = tid % TW;
  const int qc = tl / PQ, qh = tl % PQ;  // QR layout
  const int jc = tl / PJ, jh = tl % PJ;  // Jacobi layout
  const int base = tid - tl;             // first thread of the team (a lane, for TW <= 64)
  const bool real = team < bdp->count;
  // inst[] is indexed per lane: read it from memory, not from a register copy
  const int me = bdp->inst[real ? team : 0];
  TeamLds<S, CM, TW>& L = reinterpret_cast<TeamLds<S, CM, TW>*>(lds_base)[team];
  InstDev* I = P.inst + me;
  const int n = I->n;
  const int M = I->M;
  const int cap = I->cap < CM ? I->cap : CM;
  const int64_t k = bdp->k;
  cx<S>* arena = reinterpret_cast<cx<S>*>(P.arena) + I->site_off;
  cd* edges = reinterpret_cast<cd*>(P.edge) + I->edge_off;
  const int ew = I->ew;
  // the complex-FP64 slot of an edge site, or null for a bulk site
  auto eslot = [&](int i) -> cd* {
    const int ei = edge_index(i, n, ew);
    return ei >= 0 ? edges + (int64_t)ei * SLOT : nullptr;
  };
  const uint64_t* W = P.marked + I->marked_off;
  const double tol2 = P.trunc_tol * P.trunc_tol;
  const double rank2 = P.rank_tol * P.rank_tol;
  const double skip2 = P.skip_tol * P.skip_tol;
  const bool sr = P.stoch_round != 0;
  double* warm = P.warm ? reinterpret_cast<double*>(reinterpret_cast<char*>(P.warm) + I->warm_off) : nullptr;
  // without warm starts the record loads read this instance's own records area: the site
  // slots, which hold at least one record's worth of elements (never used)
  const double* wdummy = reinterpret_cast<const double*>(reinterpret_cast<cx<S>*>(P.arena) + I->site_off);
  // read once: a global load inside the sweeps would be waited for at its use
  const uint64_t k_done0 = (uint64_t)I->k_done;
  uint64_t rs_state = mix64(((uint64_t)me << 32) ^ (k_done0 * 0x9E3779B97F4A7C15ull) ^ (uint64_t)tl);

  for (int l = tl; l < kBondStride; l += TW) L.bond[l] = P.bonds[(int64_t)me * kBondStride + l];
  lds_sync();

  double f64 = 0.0, f32 = 0.0, drift = 0.0, truncw = 0.0;
  int status = 0;

  if (n == 1) {
    // A single site: the reflection is the 2x2 operator c0 I + c1 P itself.
    for (int64_t it = 0; it < k; ++it) {
      for (int j = 0; j <= M; ++j) {
        const bool diff = (j == M);
        const int xb = diff ? 0 : (int)(W[j] & 1);
        const double c0 = diff ? -1.0 : 1.0, c1 = diff ? 2.0 : -2.0;
        // the one site holds the norm: from and to its edge slot in FP64
        const cd a0 = edges[0], a1 = edges[D];
        cd o = {0.0, 0.0};
        if (tl < 2) {
          const cd pa = proj_apply<double>(a0, a1, tl, diff, xb);
          const cd as = sel(a0, a1, tl);
          o = {c0 * as.re + c1 * pa.re, c0 * as.im + c1 * pa.im};
        }
        const double nn = gsum<PQ>(tl < 2 ? norm2(o) : 0.0);
        if (diff) {
          const double nr = sqrt(nn);
          drift = fmax(drift, fabs(nr - 1.0));
          if (!(nn > 0.0) || !isfinite(nn)) status |= GMPS_ST_NAN;
          o = (1.0 / nr) * o;
        }
        team_sync_global();
        if (real && tl < 2) {
          arena[tl * D] = store_cast<S>(o, rs_state, sr);
          edges[tl * D] = o;
        }
        team_sync_global();
      }
    }
  } else {
    for (int64_t it = 0; it < k; ++it) {
      for (int j = 0; j <= M; ++j) {
        const bool diff = (j == M);
        const uint64_t xw = diff ? 0ull : W[j];
        const double c0 = diff ? -1.0 : 1.0, c1 = diff ? 2.0 : -2.0;

        // ---------------------------------------------- QR sweep with the MPO fused
        int r = 1;
        if (tl == 0) {
          L.rdim[0] = 1;
          // the first site's tile is [A | P A] itself: R = [1 1] over the two MPO blocks
          L.u.q.R[0][0] = {1.0, 0.0};
          L.u.q.R[0][1] = {1.0, 0.0};
        }
        TeamAPre<S, CM, TW> apre;
        apre.load(arena, tl, L.bond[0], L.bond[1]);
        lds_sync();
        for (int i = 0; i < n; ++i) {
          const int chl = L.bond[i], chr = L.bond[i + 1];
          const bool first = (i == 0), last = (i == n - 1);
          const int xb = diff ? 0 : (int)((xw >> (n - 1 - i)) & 1ull);
          const int Dl = first ? 1 : 2 * chl;
          const int Dr = last ? 1 : 2 * chr;
          cx<S>* slot = arena + (int64_t)i * SLOT;
          cd* es = eslot(i);
          apre.stage64(L.u.q.W, es, tl, diff, xb, last ? c0 : 1.0, last ? c1 : 1.0);
          if (i + 1 < n) apre.load(arena + (int64_t)(i + 1) * SLOT, tl, L.bond[i + 1], L.bond[i + 2]);
          lds_sync();
          // X = R_{i-1} * MPO(A_i): this slot's column, rows (a, s) = part + PQ*e
          cd x[RQ];
          {
            const int beta = (!last && qc >= chr) ? 1 : 0;
            const int bcol = qc - beta * chr;
#pragma unroll
            for (int e = 0; e < RQ; ++e) {
              const int row = qh + PQ * e;
              const int a = row >> 1, s = row & 1;
              cd acc = {0.0, 0.0};
              if (row < 2 * r && qc < Dr) {
                // the last site sums both MPO blocks into its one column
#pragma unroll
                for (int bl = 0; bl < 2; ++bl) {
                  if (last || bl == beta) {
#pragma unroll
                    for (int ap = 0; ap < CM; ++ap)
                      if (ap < chl) acc = cfma(acc, L.u.q.R[a][bl * chl + ap], L.u.q.W[bl][ap][s][bcol]);
                  }
                }
              }
              x[e] = acc;
            }
          }
          f64 += 8.0 * (double)r * Dl * 2.0 * Dr;
          if (last) {
            // the last site holds the norm: to its edge slot in FP64, to its site slot as stored
            if (real && qc == 0) {
#pragma unroll
              for (int e = 0; e < RQ; ++e) {
                const int row = qh + PQ * e;
                if (row < 2 * r) {
                  slot[(row >> 1) * 2 * D + (row & 1) * D] = store_cast<S>(x[e], rs_state, sr);
                  es[(row >> 1) * 2 * D + (row & 1) * D] = x[e];
                }
              }
            }
            if (tl == 0) {
              L.rdim[n - 1] = r;
              L.rdim[n] = 1;
            }
            break;
          }
          const int m = 2 * r;
          cd q[RQ];
          double qdrop = 0.0;
          int kr;
          if constexpr (TW <= 64)
            kr = team_qr_wave<TW, PQ, RQ, KQ>(x, q, base, qc, qh, m, Dr, chr, rank2, &qdrop, L.u.q.V, L.u.q.tau);
          else
            kr = team_qr_lds<PQ, RQ, KQ>(x, q, qc, qh, m, Dr, chr, rank2, &qdrop, L.u.q.V, L.u.q.tau, L.colv);
          truncw = fmax(truncw, qdrop);
          {
            const double mm = m, cc = Dr, kk = kr;
            f64 += 8.0 * (2.0 * mm * cc * kk - (mm + cc) * kk * kk + 2.0 * kk * kk * kk / 3.0) +
                   8.0 * (2.0 * mm * kk * kk - 2.0 * kk * kk * kk / 3.0);
          }
          cx<S> qs[RQ];  // Q as stored
#pragma unroll
          for (int e = 0; e < RQ; ++e) qs[e] = store_cast<S>(q[e], rs_state, sr);
          if (real && qc < kr) {
#pragma unroll
            for (int e = 0; e < RQ; ++e) {
              const int row = qh + PQ * e;
              if (row < m) {
                slot[(row >> 1) * 2 * D + (row & 1) * D + qc] = qs[e];
                if (es) es[(row >> 1) * 2 * D + (row & 1) * D + qc] = q[e];
              }
            }
          }
          if (qc < Dr) {
#pragma unroll
            for (int e = 0; e < RQ; ++e) {
              const int row = qh + PQ * e;
              if (row < kr) L.u.q.R[row][qc] = x[e];
            }
          }
          if (kMixed && !es) {
            comp_store_cols<PQ, RQ, KQ, D>(q, qs, qc, qh, kr, Dr, L.u.q.V, L.zbuf(), L.u.q.R);
            f64 += 8.0 * ((double)kr * kr * m + (double)kr * kr * Dr);
          }
          if (tl == 0) L.rdim[i + 1] = kr;
          r = kr;
          lds_sync();
        }
        // the QR sweep's site tensors are read by every wave of the team from here on
        team_sync_global();

        // ---------------------------------------------- truncated-SVD sweep
        // At site i the tile is M = Q_i (U Sigma)_{i+1} reshaped (r_i, 2 chi'); Jacobi runs on
        // the r_i columns of M^H: M^H J = V Sigma with J = U, so V^H = Sigma^{-1} (M^H J)^H
        // stays in site i and U Sigma = J Sigma moves left.
        if (tl == 0) L.u.s.Y[0][0] = {1.0, 0.0};
        TeamQPre<S, KQ, CM, TW> qpre;
        TeamWPre<KJ, TW> wpre;
        qpre.load(arena + (int64_t)(n - 1) * SLOT, tl, L.rdim[n - 1], L.rdim[n]);
        wpre.load(warm ? warm + ((int64_t)j * n + (n - 1)) * WREC : wdummy, warm != nullptr, tl, (L.rdim[n - 1] + 1) & ~1);
        for (int i = n - 1; i >= 1; --i) {
          const int ri = L.rdim[i], rn = L.rdim[i + 1];
          const int chn = L.bond[i + 1];
          const int c = 2 * chn;
          const int ncj = (ri + 1) & ~1;
          cx<S>* slot = arena + (int64_t)i * SLOT;
          cd* es = eslot(i);
          double* wrec = warm ? warm + ((int64_t)j * n + i) * WREC : nullptr;
          const bool use_warm = wrec && wpre.r() == ncj;
          // the stored unitary is a product of exact rotations, so its unitarity drifts by
          // ~1e-16 per use; one Newton-Schulz step every 64 iterations keeps it below ~1e-13
          const bool renorm_warm = use_warm && ((k_done0 + (uint64_t)it) & 63ull) == 0ull;
          if (es) {
            // an edge site (the first one holds the norm): from its complex-FP64 edge slot
            for (int e = tl; e < KQ * 2 * KQ; e += TW) {
              const int a = e / (2 * KQ), s = (e / KQ) & 1, b = e % KQ;
              (&L.u.s.Q[0][0][0])[e] = (a < ri && b < rn) ? es[a * 2 * D + s * D + b] : cd{0.0, 0.0};
            }
          } else {
            qpre.stage(&L.u.s.Q[0][0][0], tl);
          }
          if (use_warm) wpre.stage(&L.u.s.W[0][0], tl);
          if (i - 1 >= 1) {
            qpre.load(arena + (int64_t)(i - 1) * SLOT, tl, L.rdim[i - 1], L.rdim[i]);
            wpre.load(warm ? warm + ((int64_t)j * n + (i - 1)) * WREC : wdummy, warm != nullptr, tl,
                      (L.rdim[i - 1] + 1) & ~1);
          }
          lds_sync();
          // column jc of M^H: M^H[(s, jj)][a] = conj(sum_b Q[a][s][b] Y[b][jj])
          cd a[RJ];
#pragma unroll
          for (int e = 0; e < RJ; ++e) {
            const int row = jh + PJ * e;
            const int s = row >= chn ? 1 : 0;
            const int jj = row - s * chn;
            cd acc = {0.0, 0.0};
            if (jc < ri && row < c) {
#pragma unroll
              for (int b = 0; b < KQ; ++b)
                if (b < rn) acc = cfma(acc, L.u.s.Q[jc][s][b], L.u.s.Y[b][jj]);
            }
            a[e] = conj(acc);
          }
          f64 += 8.0 * (double)ri * 2.0 * rn * chn;
          if (renorm_warm) {
            // one Newton-Schulz polar step W <- W (3I - W^H W) / 2 (error e -> O(e^2))
            cd* WG = &L.u.s.XU[0][0][0];  // KJ x KJ, row-major
            for (int e = tl; e < KJ * KJ; e += TW) {
              const int ra = e / KJ, ca = e % KJ;
              cd g = {0.0, 0.0};
              for (int b = 0; b < ncj; ++b) g = g + cmulc(L.u.s.W[b][ra], L.u.s.W[b][ca]);
              WG[e] = g;
            }
            lds_sync();
            constexpr int NW = (KJ * KJ + TW - 1) / TW;
            cd wn[NW];
#pragma unroll
            for (int t = 0; t < NW; ++t) {
              const int e = tl + t * TW;
              const int ra = e / KJ, ca = e % KJ;
              cd acc = {0.0, 0.0};
              if (e < KJ * KJ)
                for (int b = 0; b < ncj; ++b) acc = cfma(acc, L.u.s.W[ra][b], WG[b * KJ + ca]);
              wn[t] = (e < KJ * KJ) ? 1.5 * L.u.s.W[ra][ca] - 0.5 * acc : cd{0.0, 0.0};
            }
            lds_sync();
#pragma unroll
            for (int t = 0; t < NW; ++t) {
              const int e = tl + t * TW;
              if (e < KJ * KJ) L.u.s.W[e / KJ][e % KJ] = wn[t];
            }
            lds_sync();
          }
          cd uu[RU];
          if (use_warm) {
            // start from the previous iteration's unitary: M^H <- M^H W
            if (jc < KJ) {
#pragma unroll
              for (int e = 0; e < RJ; ++e) L.u.s.XA[0][jc][jh + PJ * e] = a[e];
            }
            lds_sync();
#pragma unroll
            for (int e = 0; e < RJ; ++e) {
              const int row = jh + PJ * e;
              cd acc = {0.0, 0.0};
              if (jc < ncj)
                for (int b = 0; b < ncj; ++b) acc = cfma(acc, L.u.s.XA[0][b][row], L.u.s.W[b][jc]);
              a[e] = acc;
            }
#pragma unroll
            for (int e = 0; e < RU; ++e) {
              const int row = jh + PJ * e;
              uu[e] = (jc < ncj && row < ncj) ? L.u.s.W[row][jc] : cd{0.0, 0.0};
            }
            lds_sync();
          } else {
#pragma unroll
            for (int e = 0; e < RU; ++e) uu[e] = {(jh + PJ * e == jc && jc < ncj) ? 1.0 : 0.0, 0.0};
          }
          int sweeps;
          if constexpr (TW <= 64)
            sweeps = team_jacobi_wave<TW, PJ, RJ, RU>(a, uu, base, jc, jh, ncj, kJacobiTol2, skip2, P.max_sweeps);
          else
            sweeps = team_jacobi_lds<PJ, RJ, RU, KJ, T::NBUF>(a, uu, jc, jh, ncj, kJacobiTol2, skip2, P.max_sweeps,
                                                              L.u.s.XA, L.u.s.XU, L.u.s.XN, L.colv, L.colf);
          f64 += (double)sweeps * ri * (ri - 1) / 2.0 * 56.0 * c;
          // singular values, truncation and the kept order
          const bool colok = jc < ncj;
          double sg = 0.0;
#pragma unroll
          for (int e = 0; e < RJ; ++e) sg += norm2(a[e]);
          sg = gsum<PJ>(sg);
          // kept columns stay in their index order (so the bond basis, and the next warm
          // start, does not jump when Schmidt values are degenerate); dropped ones follow
          double stot, dropped;
          int chi_new, pos;
          bool keep;
          if constexpr (TW <= 64) {
            const double mine = colok ? sg : 0.0;
            const double smax = tmax<TW>(mine);
            stot = tsum<TW>(jh == 0 ? mine : 0.0);
            const int above = (int)tsum<TW>((jh == 0 && mine > 0.0 && mine >= tol2 * smax) ? 1.0 : 0.0);
            int rk = 0;
            for (int o = 0; o < ncj; ++o) {
              const double v = shfl_f64(mine, base + o * PJ);
              rk += (v > sg || (v == sg && o < jc)) ? 1 : 0;
            }
            chi_new = above < cap ? above : cap;
            if (chi_new < 1) chi_new = 1;
            keep = colok && rk < chi_new;
            const uint64_t kept = tballot<TW>(jh == 0 && keep, base);
            const int nk = __popcll(kept & ((1ull << (base + jc * PJ)) - 1ull));
            pos = keep ? nk : chi_new + (jc - nk);
            dropped = tsum<TW>((jh == 0 && colok && !keep) ? sg : 0.0);
          } else {
            if (jh == 0) L.colv[jc] = colok ? sg : 0.0;
            lds_sync();
            double smax = 0.0;
            stot = 0.0;
            for (int o = 0; o < ncj; ++o) {
              const double v = L.colv[o];
              smax = fmax(smax, v);
              stot += v;
            }
            int above = 0, rk = 0;
            for (int o = 0; o < ncj; ++o) {
              const double v = L.colv[o];
              above += (v > 0.0 && v >= tol2 * smax) ? 1 : 0;
              rk += (v > sg || (v == sg && o < jc)) ? 1 : 0;
            }
            chi_new = above < cap ? above : cap;
            if (chi_new < 1) chi_new = 1;
            if (jh == 0) L.colr[jc] = colok ? rk : KJ + jc;
            lds_sync();
            dropped = 0.0;
            int nk = 0, nd = 0;
            for (int o = 0; o < ncj; ++o) {
              const bool ko = L.colr[o] < chi_new;
              if (!ko) dropped += L.colv[o];
              if (o < jc) {
                nk += ko ? 1 : 0;
                nd += ko ? 0 : 1;
              }
            }
            keep = colok && rk < chi_new;
            pos = keep ? nk : chi_new + nd;
          }
          if (stot > 0.0) truncw = fmax(truncw, dropped / stot);
          if (!isfinite(stot)) status |= GMPS_ST_NAN;
          if (wrec && real) {
            // keep J with its columns in the kept order for the next iteration
            if (colok) {
#pragma unroll
              for (int e = 0; e < RU; ++e) {
                const int row = jh + PJ * e;
                if (row < ncj) {
                  wrec[2 + 2 * (row * KJ + pos)] = uu[e].re;
                  wrec[3 + 2 * (row * KJ + pos)] = uu[e].im;
                }
              }
            }
            if (tl == 0) wrec[0] = (double)ncj;
          }
          const double rs = keep ? rsqrt_acc(sg) : 0.0;  // 1/sigma
          cd wv[RJ];     // this slot's row of V^H
          cx<S> vs[RJ];  // ... as stored
#pragma unroll
          for (int e = 0; e < RJ; ++e) {
            wv[e] = rs * conj(a[e]);
            vs[e] = store_cast<S>(wv[e], rs_state, sr);
          }
          if (keep && real) {
#pragma unroll
            for (int e = 0; e < RJ; ++e) {
              const int row = jh + PJ * e;
              if (row < c) {
                const int s = row >= chn ? 1 : 0;
                const int jp = row - s * chn;
                slot[pos * 2 * D + s * D + jp] = vs[e];
                if (es) es[pos * 2 * D + s * D + jp] = wv[e];
              }
            }
          }
          cd yv[RU];  // this slot's column of the carry J Sigma
#pragma unroll
          for (int e = 0; e < RU; ++e) yv[e] = (sg * rs) * uu[e];
          if (kMixed && !es) {
            // the Jacobi exchange buffers are free: the kept rows and Z go there
            comp_store_rows<PJ, RJ, RU, CM>(wv, vs, yv, keep, pos, jh, c, ri, chi_new,
                                            reinterpret_cast<cd*>(&L.u.s.XA[0][0][0]),
                                            reinterpret_cast<cd*>(&L.u.s.XU[0][0][0]), L.u.s.Y);
            f64 += 8.0 * ((double)chi_new * chi_new * c + (double)chi_new * chi_new * ri);
          }
          if (keep) {
#pragma unroll
            for (int e = 0; e < RU; ++e) {
              const int row = jh + PJ * e;
              if (row < ri) L.u.s.Y[row][pos] = yv[e];
            }
          }
          if (tl == 0) L.bond[i] = chi_new;
          lds_sync();
        }
        // ---------------------------------------------- site 0 (holds the norm)
        team_sync_global();
        {
          const int rn = L.rdim[1], chn = L.bond[1];
          cx<S>* slot = arena;
          cd acc = {0.0, 0.0};
          const bool act = tl < 2 * chn;
          const int s = tl >= chn ? 1 : 0;
          const int jj = tl - s * chn;
          if (act) {
#pragma unroll
            for (int b = 0; b < KQ; ++b)
              if (b < rn) acc = cfma(acc, edges[s * D + b], L.u.s.Y[b][jj]);
          }
          f64 += 8.0 * 2.0 * rn * chn;
          double nn = 0.0;
          if constexpr (TW <= 64) {
            nn = tsum<TW>(act ? norm2(acc) : 0.0);
          } else {
            L.colv[tl] = act ? norm2(acc) : 0.0;
            lds_sync();
            for (int o = 0; o < 2 * chn; ++o) nn += L.colv[o];
          }
          if (!isfinite(nn) || !(nn > 0.0)) status |= GMPS_ST_NAN;
          const double nr = sqrt(nn);
          if (diff) drift = fmax(drift, fabs(nr - 1.0));
          // site 0 now holds the norm: to its edge slot in FP64, to its site slot as stored
          const cd outd = (diff ? 1.0 / nr : 1.0) * acc;
          const cx<S> out = store_cast<S>(outd, rs_state, sr);
          lds_sync();
          if (real && act) {
            slot[s * D + jj] = out;
            edges[s * D + jj] = outd;
          }
          if (tl == 0) L.bond[0] = 1;
          team_sync_global();
        }
      }
    }
  }

  // ------------------------------------------------------------------ write back
  if (real) {
    for (int l = tl; l < kBondStride; l += TW) P.bonds[(int64_t)me * kBondStride + l] = L.bond[l];
    if (tl == 0) {
      I->k_done += k;
      I->flops64 += f64;
      I->flops32 += f32;
      I->drift = fmax(I->drift, drift);
      I->trunc_w = fmax(I->trunc_w, truncw);
      if (drift > 1e-3) status |= GMPS_ST_DRIFT;
      if (truncw > 1e-8) status |= GMPS_ST_TRUNC;
      I->status |= status;
    }
  }
  team_sync_global();
}

// run_team for a gate-level circuit (the Common method; a separate function, so that the
// reflection kernels keep their own code): the reflections come from the instance's gate stream
// (P.circuit) instead of its marked set. Every n-controlled Z is a reflection about |1..1>
// (c0 = 1, c1 = -2, renormalised), the single-qubit gates before it are fused per qubit and
// applied as its sites are staged, and the gates after the last one are applied to the sites in
// place at the end. The stream holds k (M+1) n-controlled Z gates, as k layers of Fig. 1(A) do.
template <class S, int CM, int TW>
__device__ void run_team_circ(const IterParams& P, const Bundle* bdp, char* lds_base) {
  using T = TeamShape<CM, TW>;
  constexpr int D = T::D, KQ = T::KQ, KJ = T::KJ;
  constexpr int PQ = T::PQ, RQ = T::RQ, PJ = T::PJ, RJ = T::RJ, RU = T::RU;
  constexpr int SLOT = slot_elems(CM);
  constexpr bool kMixed = sizeof(S) == sizeof(float);
  constexpr int64_t WREC = wide_warm_doubles(CM);
  const int tid = threadIdx.x;
  const int team = tid / TW;
  const int tl = tid % TW;
  const int qc = tl / PQ, qh = tl % PQ;  // QR layout
  const int jc = tl / PJ, jh = tl % PJ;  // Jacobi layout
  const int base = tid - tl;             // first thread of the team (a lane, for TW <= 64)
  const bool real = team < bdp->count;
  // inst[] is indexed per lane: read it from memory, not from a register copy
  const int me = bdp->inst[real ? team : 0];
  TeamLds<S, CM, TW>& L = reinterpret_cast<TeamLds<S, CM, TW>*>(lds_base)[team];
  InstDev* I = P.inst + me;
  const int n = I->n;
  const int M = I->M;
  const int cap = I->cap < CM ? I->cap : CM;
  const int64_t k = bdp->k;
  cx<S>* arena = reinterpret_cast<cx<S>*>(P.arena) + I->site_off;
  cd* edges = reinterpret_cast<cd*>(P.edge) + I->edge_off;
  const int ew = I->ew;
  // the complex-FP64 slot of an edge site, or null for a bulk site
  auto eslot = [&](int i) -> cd* {
    const int ei = edge_index(i, n, ew);
    return ei >= 0 ? edges + (int64_t)ei * SLOT : nullptr;
  };
  const double tol2 = P.trunc_tol * P.trunc_tol;
  const double rank2 = P.rank_tol * P.rank_tol;
  const double skip2 = P.skip_tol * P.skip_tol;
  const bool sr = P.stoch_round != 0;
  double* warm = P.warm ? reinterpret_cast<double*>(reinterpret_cast<char*>(P.warm) + I->warm_off) : nullptr;
  // without warm starts the record loads read this instance's own records area: the site
  // slots, which hold at least one record's worth of elements (never used)
  const double* wdummy = reinterpret_cast<const double*>(reinterpret_cast<cx<S>*>(P.arena) + I->site_off);
  // read once: a global load inside the sweeps would be waited for at its use
  const uint64_t k_done0 = (uint64_t)I->k_done;
  uint64_t rs_state = mix64(((uint64_t)me << 32) ^ (k_done0 * 0x9E3779B97F4A7C15ull) ^ (uint64_t)tl);

  for (int l = tl; l < kBondStride; l += TW) L.bond[l] = P.bonds[(int64_t)me * kBondStride + l];
  lds_sync();

  double f64 = 0.0, f32 = 0.0, drift = 0.0, truncw = 0.0;
  int status = 0;

  if (n < 2) {
    // gmps_circuit_build refuses chains of one site
    status |= GMPS_ST_NAN;
  } else {
    // gate-level circuit: lane 0 of the team walks the stream; the walk takes no workgroup
    // barrier (the teams of a workgroup walk streams of different lengths), and every team
    // reaches the barrier after it once per n-controlled Z
    CircLds& C = reinterpret_cast<CircLds*>(lds_base + TeamShape<CM, TW>::TEAMS * sizeof(TeamLds<S, CM, TW>))[team];
    const uint32_t* gates = P.circuit + I->circ_off;
    const int64_t ngates = I->circ_len;
    int64_t gpos = 0;
    auto walk = [&]() {
      if (tl == 0) {
        for (int q = 0; q < n; ++q) {
          C.U[q][0] = 1.0;
          C.U[q][1] = 0.0;
          C.U[q][2] = 0.0;
          C.U[q][3] = 1.0;
        }
        while (gpos < ngates) {
          const uint32_t g = gates[gpos++];
          const uint32_t ty = g >> 8, q = g & 0xFFu;
          if (ty == kGateMCZ) break;
          double* u = C.U[q < (uint32_t)n ? q : 0];
          const double a = u[0], b = u[1], c = u[2], d = u[3];
          if (ty == kGateH) {
            u[0] = kInvSqrt2 * (a + c);
            u[1] = kInvSqrt2 * (b + d);
            u[2] = kInvSqrt2 * (a - c);
            u[3] = kInvSqrt2 * (b - d);
          } else {  // X
            u[0] = c;
            u[1] = d;
            u[2] = a;
            u[3] = b;
          }
        }
      }
      lds_sync();
    };
    for (int64_t it = 0; it < k; ++it) {
      for (int j = 0; j <= M; ++j) {
        // the next n-controlled Z, I - 2|1..1><1..1|, after the single-qubit gates before it
        walk();
        const bool diff = false;
        const uint64_t xw = ~0ull;
        const double c0 = 1.0, c1 = -2.0;
        const bool renorm = true;  // after every n-controlled Z

        // ---------------------------------------------- QR sweep with the MPO fused
        int r = 1;
        if (tl == 0) {
          L.rdim[0] = 1;
          // the first site's tile is [A | P A] itself: R = [1 1] over the two MPO blocks
          L.u.q.R[0][0] = {1.0, 0.0};
          L.u.q.R[0][1] = {1.0, 0.0};
        }
        TeamAPre<S, CM, TW> apre;
        apre.load(arena, tl, L.bond[0], L.bond[1]);
        lds_sync();
        for (int i = 0; i < n; ++i) {
          const int chl = L.bond[i], chr = L.bond[i + 1];
          const bool first = (i == 0), last = (i == n - 1);
          const int xb = diff ? 0 : (int)((xw >> (n - 1 - i)) & 1ull);
          const int Dl = first ? 1 : 2 * chl;
          const int Dr = last ? 1 : 2 * chr;
          cx<S>* slot = arena + (int64_t)i * SLOT;
          cd* es = eslot(i);
          apre.stage64u(L.u.q.W, es, tl, C.U[i], xb, last ? c0 : 1.0, last ? c1 : 1.0);
          if (i + 1 < n) apre.load(arena + (int64_t)(i + 1) * SLOT, tl, L.bond[i + 1], L.bond[i + 2]);
          lds_sync();
          // X = R_{i-1} * MPO(A_i): this slot's column, rows (a, s) = part + PQ*e
          cd x[RQ];
          {
            const int beta = (!last && qc >= chr) ? 1 : 0;
            const int bcol = qc - beta * chr;
#pragma unroll
            for (int e = 0; e < RQ; ++e) {
              const int row = qh + PQ * e;
              const int a = row >> 1, s = row & 1;
              cd acc = {0.0, 0.0};
              if (row < 2 * r && qc < Dr) {
                // the last site sums both MPO blocks into its one column
#pragma unroll
                for (int bl = 0; bl < 2; ++bl) {
                  if (last || bl == beta) {
#pragma unroll
                    for (int ap = 0; ap < CM; ++ap)
                      if (ap < chl) acc = cfma(acc, L.u.q.R[a][bl * chl + ap], L.u.q.W[bl][ap][s][bcol]);
                  }
                }
              }
              x[e] = acc;
            }
          }
          f64 += 8.0 * (double)r * Dl * 2.0 * Dr;
          if (last) {
            // the last site holds the norm: to its edge slot in FP64, to its site slot as stored
            if (real && qc == 0) {
#pragma unroll
              for (int e = 0; e < RQ; ++e) {
                const int row = qh + PQ * e;
                if (row < 2 * r) {
                  slot[(row >> 1) * 2 * D + (row & 1) * D] = store_cast<S>(x[e], rs_state, sr);
                  es[(row >> 1) * 2 * D + (row & 1) * D] = x[e];
                }
              }
            }
            if (tl == 0) {
              L.rdim[n - 1] = r;
              L.rdim[n] = 1;
            }
            break;
          }
          const int m = 2 * r;
          cd q[RQ];
          double qdrop = 0.0;
          int kr;
          if constexpr (TW <= 64)
            kr = team_qr_wave<TW, PQ, RQ, KQ>(x, q, base, qc, qh, m, Dr, chr, rank2, &qdrop, L.u.q.V, L.u.q.tau);
          else
            kr = team_qr_lds<PQ, RQ, KQ>(x, q, qc, qh, m, Dr, chr, rank2, &qdrop, L.u.q.V, L.u.q.tau, L.colv);
          truncw = fmax(truncw, qdrop);
          {
            const double mm = m, cc = Dr, kk = kr;
            f64 += 8.0 * (2.0 * mm * cc * kk - (mm + cc) * kk * kk + 2.0 * kk * kk * kk / 3.0) +
                   8.0 * (2.0 * mm * kk * kk - 2.0 * kk * kk * kk / 3.0);
          }
          cx<S> qs[RQ];  // Q as stored
#pragma unroll
          for (int e = 0; e < RQ; ++e) qs[e] = store_cast<S>(q[e], rs_state, sr);
          if (real && qc < kr) {
#pragma unroll
            for (int e = 0; e < RQ; ++e) {
              const int row = qh + PQ * e;
              if (row < m) {
                slot[(row >> 1) * 2 * D + (row & 1) * D + qc] = qs[e];
                if (es) es[(row >> 1) * 2 * D + (row & 1) * D + qc] = q[e];
              }
            }
          }
          if (qc < Dr) {
#pragma unroll
            for (int e = 0; e < RQ; ++e) {
              const int row = qh + PQ * e;
              if (row < kr) L.u.q.R[row][qc] = x[e];
            }
          }
          if (kMixed && !es) {
            comp_store_cols<PQ, RQ, KQ, D>(q, qs, qc, qh, kr, Dr, L.u.q.V, L.zbuf(), L.u.q.R);
            f64 += 8.0 * ((double)kr * kr * m + (double)kr * kr * Dr);
          }
          if (tl == 0) L.rdim[i + 1] = kr;
          r = kr;
          lds_sync();
        }
        // the QR sweep's site tensors are read by every wave of the team from here on
        team_sync_global();

        // ---------------------------------------------- truncated-SVD sweep
        // At site i the tile is M = Q_i (U Sigma)_{i+1} reshaped (r_i, 2 chi'); Jacobi runs on
        // the r_i columns of M^H: M^H J = V Sigma with J = U, so V^H = Sigma^{-1} (M^H J)^H
        // stays in site i and U Sigma = J Sigma moves left.
        if (tl == 0) L.u.s.Y[0][0] = {1.0, 0.0};
        TeamQPre<S, KQ, CM, TW> qpre;
        TeamWPre<KJ, TW> wpre;
        qpre.load(arena + (int64_t)(n - 1) * SLOT, tl, L.rdim[n - 1], L.rdim[n]);
        wpre.load(warm ? warm + ((int64_t)j * n + (n - 1)) * WREC : wdummy, warm != nullptr, tl, (L.rdim[n - 1] + 1) & ~1);
        for (int i = n - 1; i >= 1; --i) {
          const int ri = L.rdim[i], rn = L.rdim[i + 1];
          const int chn = L.bond[i + 1];
          const int c = 2 * chn;
          const int ncj = (ri + 1) & ~1;
          cx<S>* slot = arena + (int64_t)i * SLOT;
          cd* es = eslot(i);
          double* wrec = warm ? warm + ((int64_t)j * n + i) * WREC : nullptr;
          const bool use_warm = wrec && wpre.r() == ncj;
          // the stored unitary is a product of exact rotations, so its unitarity drifts by
          // ~1e-16 per use; one Newton-Schulz step every 64 iterations keeps it below ~1e-13
          const bool renorm_warm = use_warm && ((k_done0 + (uint64_t)it) & 63ull) == 0ull;
          if (es) {
            // an edge site (the first one holds the norm): from its complex-FP64 edge slot
            for (int e = tl; e < KQ * 2 * KQ; e += TW) {
              const int a = e / (2 * KQ), s = (e / KQ) & 1, b = e % KQ;
              (&L.u.s.Q[0][0][0])[e] = (a < ri && b < rn) ? es[a * 2 * D + s * D + b] : cd{0.0, 0.0};
            }
          } else {
            qpre.stage(&L.u.s.Q[0][0][0], tl);
          }
          if (use_warm) wpre.stage(&L.u.s.W[0][0], tl);
          if (i - 1 >= 1) {
            qpre.load(arena + (int64_t)(i - 1) * SLOT, tl, L.rdim[i - 1], L.rdim[i]);
            wpre.load(warm ? warm + ((int64_t)j * n + (i - 1)) * WREC : wdummy, warm != nullptr, tl,
                      (L.rdim[i - 1] + 1) & ~1);
          }
          lds_sync();
          // column jc of M^H: M^H[(s, jj)][a] = conj(sum_b Q[a][s][b] Y[b][jj])
          cd a[RJ];
#pragma unroll
          for (int e = 0; e < RJ; ++e) {
            const int row = jh + PJ * e;
            const int s = row >= chn ? 1 : 0;
            const int jj = row - s * chn;
            cd acc = {0.0, 0.0};
            if (jc < ri && row < c) {
#pragma unroll
              for (int b = 0; b < KQ; ++b)
                if (b < rn) acc = cfma(acc, L.u.s.Q[jc][s][b], L.u.s.Y[b][jj]);
            }
            a[e] = conj(acc);
          }
          f64 += 8.0 * (double)ri * 2.0 * rn * chn;
          if (renorm_warm) {
            // one Newton-Schulz polar step W <- W (3I - W^H W) / 2 (error e -> O(e^2))
            cd* WG = &L.u.s.XU[0][0][0];  // KJ x KJ, row-major
            for (int e = tl; e < KJ * KJ; e += TW) {
              const int ra = e / KJ, ca = e % KJ;
              cd g = {0.0, 0.0};
              for (int b = 0; b < ncj; ++b) g = g + cmulc(L.u.s.W[b][ra], L.u.s.W[b][ca]);
              WG[e] = g;
            }
            lds_sync();
            constexpr int NW = (KJ * KJ + TW - 1) / TW;
            cd wn[NW];
#pragma unroll
            for (int t = 0; t < NW; ++t) {
              const int e = tl + t * TW;
              const int ra = e / KJ, ca = e % KJ;
              cd acc = {0.0, 0.0};
              if (e < KJ * KJ)
                for (int b = 0; b < ncj; ++b) acc = cfma(acc, L.u.s.W[ra][b], WG[b * KJ + ca]);
              wn[t] = (e < KJ * KJ) ? 1.5 * L.u.s.W[ra][ca] - 0.5 * acc : cd{0.0, 0.0};
            }
            lds_sync();
#pragma unroll
            for (int t = 0; t < NW; ++t) {
              const int e = tl + t * TW;
              if (e < KJ * KJ) L.u.s.W[e / KJ][e % KJ] = wn[t];
            }
            lds_sync();
          }
          cd uu[RU];
          if (use_warm) {
            // start from the previous iteration's unitary: M^H <- M^H W
            if (jc < KJ) {
#pragma unroll
              for (int e = 0; e < RJ; ++e) L.u.s.XA[0][jc][jh + PJ * e] = a[e];
            }
            lds_sync();
#pragma unroll
            for (int e = 0; e < RJ; ++e) {
              const int row = jh + PJ * e;
              cd acc = {0.0, 0.0};
              if (jc < ncj)
                for (int b = 0; b < ncj; ++b) acc = cfma(acc, L.u.s.XA[0][b][row], L.u.s.W[b][jc]);
              a[e] = acc;
            }
#pragma unroll
            for (int e = 0; e < RU; ++e) {
              const int row = jh + PJ * e;
              uu[e] = (jc < ncj && row < ncj) ? L.u.s.W[row][jc] : cd{0.0, 0.0};
            }
            lds_sync();
          } else {
#pragma unroll
            for (int e = 0; e < RU; ++e) uu[e] = {(jh + PJ * e == jc && jc < ncj) ? 1.0 : 0.0, 0.0};
          }
          int sweeps;
          if constexpr (TW <= 64)
            sweeps = team_jacobi_wave<TW, PJ, RJ, RU>(a, uu, base, jc, jh, ncj, kJacobiTol2, skip2, P.max_sweeps);
          else
            sweeps = team_jacobi_lds<PJ, RJ, RU, KJ, T::NBUF>(a, uu, jc, jh, ncj, kJacobiTol2, skip2, P.max_sweeps,
                                                              L.u.s.XA, L.u.s.XU, L.u.s.XN, L.colv, L.colf);
          f64 += (double)sweeps * ri * (ri - 1) / 2.0 * 56.0 * c;
          // singular values, truncation and the kept order
          const bool colok = jc < ncj;
          double sg = 0.0;
#pragma unroll
          for (int e = 0; e < RJ; ++e) sg += norm2(a[e]);
          sg = gsum<PJ>(sg);
          // kept columns stay in their index order (so the bond basis, and the next warm
          // start, does not jump when Schmidt values are degenerate); dropped ones follow
          double stot, dropped;
          int chi_new, pos;
          bool keep;
          if constexpr (TW <= 64) {
            const double mine = colok ? sg : 0.0;
            const double smax = tmax<TW>(mine);
            stot = tsum<TW>(jh == 0 ? mine : 0.0);
            const int above = (int)tsum<TW>((jh == 0 && mine > 0.0 && mine >= tol2 * smax) ? 1.0 : 0.0);
            int rk = 0;
            for (int o = 0; o < ncj; ++o) {
              const double v = shfl_f64(mine, base + o * PJ);
              rk += (v > sg || (v == sg && o < jc)) ? 1 : 0;
            }
            chi_new = above < cap ? above : cap;
            if (chi_new < 1) chi_new = 1;
            keep = colok && rk < chi_new;
            const uint64_t kept = tballot<TW>(jh == 0 && keep, base);
            const int nk = __popcll(kept & ((1ull << (base + jc * PJ)) - 1ull));
            pos = keep ? nk : chi_new + (jc - nk);
            dropped = tsum<TW>((jh == 0 && colok && !keep) ? sg : 0.0);
          } else {
            if (jh == 0) L.colv[jc] = colok ? sg : 0.0;
            lds_sync();
            double smax = 0.0;
            stot = 0.0;
            for (int o = 0; o < ncj; ++o) {
              const double v = L.colv[o];
              smax = fmax(smax, v);
              stot += v;
            }
            int above = 0, rk = 0;
            for (int o = 0; o < ncj; ++o) {
              const double v = L.colv[o];
              above += (v > 0.0 && v >= tol2 * smax) ? 1 : 0;
              rk += (v > sg || (v == sg && o < jc)) ? 1 : 0;
            }
            chi_new = above < cap ? above : cap;
            if (chi_new < 1) chi_new = 1;
            if (jh == 0) L.colr[jc] = colok ? rk : KJ + jc;
            lds_sync();
            dropped = 0.0;
            int nk = 0, nd = 0;
            for (int o = 0; o < ncj; ++o) {
              const bool ko = L.colr[o] < chi_new;
              if (!ko) dropped += L.colv[o];
              if (o < jc) {
                nk += ko ? 1 : 0;
                nd += ko ? 0 : 1;
              }
            }
            keep = colok && rk < chi_new;
            pos = keep ? nk : chi_new + nd;
          }
          if (stot > 0.0) truncw = fmax(truncw, dropped / stot);
          if (!isfinite(stot)) status |= GMPS_ST_NAN;
          if (wrec && real) {
            // keep J with its columns in the kept order for the next iteration
            if (colok) {
#pragma unroll
              for (int e = 0; e < RU; ++e) {
                const int row = jh + PJ * e;
                if (row < ncj) {
                  wrec[2 + 2 * (row * KJ + pos)] = uu[e].re;
                  wrec[3 + 2 * (row * KJ + pos)] = uu[e].im;
                }
              }
            }
            if (tl == 0) wrec[0] = (double)ncj;
          }
          const double rs = keep ? rsqrt_acc(sg) : 0.0;  // 1/sigma
          cd wv[RJ];     // this slot's row of V^H
          cx<S> vs[RJ];  // ... as stored
#pragma unroll
          for (int e = 0; e < RJ; ++e) {
            wv[e] = rs * conj(a[e]);
            vs[e] = store_cast<S>(wv[e], rs_state, sr);
          }
          if (keep && real) {
#pragma unroll
            for (int e = 0; e < RJ; ++e) {
              const int row = jh + PJ * e;
              if (row < c) {
                const int s = row >= chn ? 1 : 0;
                const int jp = row - s * chn;
                slot[pos * 2 * D + s * D + jp] = vs[e];
                if (es) es[pos * 2 * D + s * D + jp] = wv[e];
              }
            }
          }
          cd yv[RU];  // this slot's column of the carry J Sigma
#pragma unroll
          for (int e = 0; e < RU; ++e) yv[e] = (sg * rs) * uu[e];
          if (kMixed && !es) {
            // the Jacobi exchange buffers are free: the kept rows and Z go there
            comp_store_rows<PJ, RJ, RU, CM>(wv, vs, yv, keep, pos, jh, c, ri, chi_new,
                                            reinterpret_cast<cd*>(&L.u.s.XA[0][0][0]),
                                            reinterpret_cast<cd*>(&L.u.s.XU[0][0][0]), L.u.s.Y);
            f64 += 8.0 * ((double)chi_new * chi_new * c + (double)chi_new * chi_new * ri);
          }
          if (keep) {
#pragma unroll
            for (int e = 0; e < RU; ++e) {
              const int row = jh + PJ * e;
              if (row < ri) L.u.s.Y[row][pos] = yv[e];
            }
          }
          if (tl == 0) L.bond[i] = chi_new;
          lds_sync();
        }
        // ---------------------------------------------- site 0 (holds the norm)
        team_sync_global();
        {
          const int rn = L.rdim[1], chn = L.bond[1];
          cx<S>* slot = arena;
          cd acc = {0.0, 0.0};
          const bool act = tl < 2 * chn;
          const int s = tl >= chn ? 1 : 0;
          const int jj = tl - s * chn;
          if (act) {
#pragma unroll
            for (int b = 0; b < KQ; ++b)
              if (b < rn) acc = cfma(acc, edges[s * D + b], L.u.s.Y[b][jj]);
          }
          f64 += 8.0 * 2.0 * rn * chn;
          double nn = 0.0;
          if constexpr (TW <= 64) {
            nn = tsum<TW>(act ? norm2(acc) : 0.0);
          } else {
            L.colv[tl] = act ? norm2(acc) : 0.0;
            lds_sync();
            for (int o = 0; o < 2 * chn; ++o) nn += L.colv[o];
          }
          if (!isfinite(nn) || !(nn > 0.0)) status |= GMPS_ST_NAN;
          const double nr = sqrt(nn);
          if (renorm) drift = fmax(drift, fabs(nr - 1.0));
          // site 0 now holds the norm: to its edge slot in FP64, to its site slot as stored
          const cd outd = (renorm ? 1.0 / nr : 1.0) * acc;
          const cx<S> out = store_cast<S>(outd, rs_state, sr);
          lds_sync();
          if (real && act) {
            slot[s * D + jj] = out;
            edges[s * D + jj] = outd;
          }
          if (tl == 0) L.bond[0] = 1;
          team_sync_global();
        }
      }
    }
    {
      // the gates after the last n-controlled Z act on the stored sites in place (a unitary on
      // the physical index keeps the chain right-canonical and its norm)
      walk();
      for (int i = 0; i < n; ++i) {
        const int chl = L.bond[i], chr = L.bond[i + 1];
        cx<S>* slot = arena + (int64_t)i * SLOT;
        cd* es = eslot(i);
        const double u00 = C.U[i][0], u01 = C.U[i][1], u10 = C.U[i][2], u11 = C.U[i][3];
        for (int e = tl; e < CM * CM; e += TW) {
          const int a = e / CM, b = e % CM;
          if (real && a < chl && b < chr) {
            const cd a0 = es ? es[a * 2 * D + b] : up(slot[a * 2 * D + b]);
            const cd a1 = es ? es[a * 2 * D + D + b] : up(slot[a * 2 * D + D + b]);
            const cd b0 = {u00 * a0.re + u01 * a1.re, u00 * a0.im + u01 * a1.im};
            const cd b1 = {u10 * a0.re + u11 * a1.re, u10 * a0.im + u11 * a1.im};
            slot[a * 2 * D + b] = store_cast<S>(b0, rs_state, sr);
            slot[a * 2 * D + D + b] = store_cast<S>(b1, rs_state, sr);
            if (es) {
              es[a * 2 * D + b] = b0;
              es[a * 2 * D + D + b] = b1;
            }
          }
        }
      }
      team_sync_global();
    }
  }

  // ------------------------------------------------------------------ write back
  if (real) {
    for (int l = tl; l < kBondStride; l += TW) P.bonds[(int64_t)me * kBondStride + l] = L.bond[l];
    if (tl == 0) {
      I->k_done += k;
      I->flops64 += f64;
      I->flops32 += f32;
      I->drift = fmax(I->drift, drift);
      I->trunc_w = fmax(I->trunc_w, truncw);
      if (drift > 1e-3) status |= GMPS_ST_DRIFT;
      if (truncw > 1e-8) status |= GMPS_ST_TRUNC;
      I->status |= status;
    }
  }
  team_sync_global();
}

// Persistent kernel of one team class W: a workgroup takes bundles from the class's queue
// until it is empty.
template <class S, int W>
__global__ __launch_bounds__(kWide[W].TW < 64 ? 64 : kWide[W].TW) void grover_team_kernel(IterParams P) {
  extern __shared__ __align__(16) char lds[];
  __shared__ unsigned int next_bundle;
  for (;;) {
    if (threadIdx.x == 0) next_bundle = atomicAdd(&P.queue->next, 1u);
    lds_sync();
    const unsigned int bi = next_bundle;
    lds_sync();
    if ((int)bi >= P.queue->nbundles) break;
    run_team<S, kWide[W].CM, kWide[W].TW>(P, P.bundles + bi, lds);
  }
}

// Persistent kernel of the gate-level circuits (the Common method) for team class W.
template <class S, int W>
__global__ __launch_bounds__(kWide[W].TW < 64 ? 64 : kWide[W].TW) void grover_team_circ_kernel(IterParams P) {
  extern __shared__ __align__(16) char lds[];
  __shared__ unsigned int next_bundle;
  for (;;) {
    if (threadIdx.x == 0) next_bundle = atomicAdd(&P.queue->next, 1u);
    lds_sync();
    const unsigned int bi = next_bundle;
    lds_sync();
    if ((int)bi >= P.queue->nbundles) break;
    run_team_circ<S, kWide[W].CM, kWide[W].TW>(P, P.bundles + bi, lds);
  }
}

// The pre-contracted reflections' version of run_team (classes with bond caps up to 17).
template <class S, int CM, int TW>
__device__ void run_team_pc(const IterParams& P, const Bundle* bdp, char* lds_base) {
  using T = TeamShape<CM, TW>;
  constexpr int D = T::D, KQ = T::KQ, KJ = T::KJ;
  constexpr int PQ = T::PQ, RQ = T::RQ, PJ = T::PJ, RJ = T::RJ, RU = T::RU;
  constexpr int SLOT = slot_elems(CM);
  constexpr bool kMixed = sizeof(S) == sizeof(float);
  constexpr int64_t WREC = wide_warm_doubles(CM);
  const int tid = threadIdx.x;
  const int team = tid / TW;
  const int tl = tid % TW;
  const int qc = tl / PQ, qh = tl % PQ;  // QR layout
  const int jc = tl / PJ, jh = tl % PJ;  // Jacobi layout
  const int base = tid - tl;             // first thread of the team (a lane, for TW <= 64)
  const bool real = team < bdp->count;
  // inst[] is indexed per lane: read it from memory, not from a register copy
  const int me = bdp->inst[real ? team : 0];
  TeamLds<S, CM, TW>& L = reinterpret_cast<TeamLds<S, CM, TW>*>(lds_base)[team];
  // pre-contracted kernels only: the extra block behind the teams' TeamLds
  PcLds<CM>& X = reinterpret_cast<PcLds<CM>*>(lds_base + T::TEAMS * sizeof(TeamLds<S, CM, TW>))[team];
  InstDev* I = P.inst + me;
  const int n = I->n;
  const int M = I->M;
  const int cap = I->cap < CM ? I->cap : CM;
  const int64_t k = bdp->k;
  cx<S>* arena = reinterpret_cast<cx<S>*>(P.arena) + I->site_off;
  cd* edges = reinterpret_cast<cd*>(P.edge) + I->edge_off;
  const int ew = I->ew;
  // the complex-FP64 slot of an edge site, or null for a bulk site
  auto eslot = [&](int i) -> cd* {
    const int ei = edge_index(i, n, ew);
    return ei >= 0 ? edges + (int64_t)ei * SLOT : nullptr;
  };
  const uint64_t* W = P.marked + I->marked_off;
  const double tol2 = P.trunc_tol * P.trunc_tol;
  const double rank2 = P.rank_tol * P.rank_tol;
  const double skip2 = P.skip_tol * P.skip_tol;
  const bool sr = P.stoch_round != 0;
  double* warm = P.warm ? reinterpret_cast<double*>(reinterpret_cast<char*>(P.warm) + I->warm_off) : nullptr;
  // without warm starts the record loads read this instance's own records area: the site
  // slots, which hold at least one record's worth of elements (never used)
  const double* wdummy = reinterpret_cast<const double*>(reinterpret_cast<cx<S>*>(P.arena) + I->site_off);
  // read once: a global load inside the sweeps would be waited for at its use
  const uint64_t k_done0 = (uint64_t)I->k_done;
  uint64_t rs_state = mix64(((uint64_t)me << 32) ^ (k_done0 * 0x9E3779B97F4A7C15ull) ^ (uint64_t)tl);

  for (int l = tl; l < kBondStride; l += TW) L.bond[l] = P.bonds[(int64_t)me * kBondStride + l];
  lds_sync();

  double f64 = 0.0, f32 = 0.0, drift = 0.0, truncw = 0.0;
  int status = 0;

  if (n == 1) {
    // A single site: the reflection is the 2x2 operator c0 I + c1 P itself.
    for (int64_t it = 0; it < k; ++it) {
      for (int j = 0; j <= M; ++j) {
        const bool diff = (j == M);
        const int xb = diff ? 0 : (int)(W[j] & 1);
        const double c0 = diff ? -1.0 : 1.0, c1 = diff ? 2.0 : -2.0;
        // the one site holds the norm: from and to its edge slot in FP64
        const cd a0 = edges[0], a1 = edges[D];
        cd o = {0.0, 0.0};
        if (tl < 2) {
          const cd pa = proj_apply<double>(a0, a1, tl, diff, xb);
          const cd as = sel(a0, a1, tl);
          o = {c0 * as.re + c1 * pa.re, c0 * as.im + c1 * pa.im};
        }
        const double nn = gsum<PQ>(tl < 2 ? norm2(o) : 0.0);
        if (diff) {
          const double nr = sqrt(nn);
          drift = fmax(drift, fabs(nr - 1.0));
          if (!(nn > 0.0) || !isfinite(nn)) status |= GMPS_ST_NAN;
          o = (1.0 / nr) * o;
        }
        team_sync_global();
        if (real && tl < 2) {
          arena[tl * D] = store_cast<S>(o, rs_state, sr);
          edges[tl * D] = o;
        }
        team_sync_global();
      }
    }
  } else {
    // Pre-contracted reflections (see the option's description): a reflection
    // c0 I + c1 sum_t |p_t><p_t| with product states p_t maps psi to c0 psi + c1 sum_t
    // <p_t|psi> p_t, an MPS of bond chi + T (T terms) whose site blocks are diag(A_i, e_t(i))
    // with e_t(i) the one-site factor of p_t. A left-to-right pass contracts the overlaps
    // first, and c1 <p_t|psi> enters at the first site, so every term column of the QR tiles
    // carries its physical weight: with unit-weight columns the QR would measure them against
    // the rounding noise of psi's small Schmidt directions and keep spurious ranks. All M
    // oracle terms go into one reflection when the bond cap is lossless (every state then has
    // rank <= M+1) and chi + M fits the tile; otherwise each marked index is its own
    // reflection (T = 1).
    constexpr bool sumv = true;
    const bool whole = sumv && I->whole != 0;
    if (whole) {
      for (int l = tl; l < n; l += TW) {
        uint32_t bits = 0u;
        for (int t = 0; t < M; ++t) bits |= (uint32_t)((W[t] >> (n - 1 - l)) & 1ull) << t;
        X.xbits[l] = bits;
      }
      lds_sync();
    }
    constexpr int NV = (CM * CM + TW - 1) / TW;  // overlap elements per thread
    static_assert(sizeof(L.u.q.W[1]) >= sizeof(X.ov), "second overlap buffer fits W[1]");
    static_assert(sizeof(L.u.q.R) >= sizeof(L.u.q.W[0]), "second staging buffer fits R");
    cd (*const ovb[2])[CM] = {X.ov, reinterpret_cast<cd (*)[CM]>(&L.u.q.W[1][0][0][0])};
    cx<S> (*const stg[2])[CM][2][CM] = {reinterpret_cast<cx<S> (*)[CM][2][CM]>(&L.u.q.W[0][0][0][0]),
                                        reinterpret_cast<cx<S> (*)[CM][2][CM]>(&L.u.q.R[0][0])};
    const int nref = whole ? 2 : M + 1;
    for (int64_t it = 0; it < k; ++it) {
      for (int j = 0; j < nref; ++j) {
        const bool diff = (j == nref - 1);
        const uint64_t xw = (diff || whole) ? 0ull : W[j];
        const double c0 = diff ? -1.0 : 1.0, c1 = diff ? 2.0 : -2.0;
        const int T = !sumv ? 0 : (diff || !whole) ? 1 : M;

        if (sumv) {
          // ---------------------------------------------- overlaps <p_t|psi>, left to right:
          // v_t <- v_t A_i[:, p_t(i), :]; site tensors staged alternately in W[0] and in the
          // R block (free until the QR sweep), rows alternately in the two overlap buffers,
          // so one barrier per site orders every write after the reads it replaces
          if (tl < T) X.ov[tl][0] = {1.0, 0.0};
          TeamAPre<S, CM, TW> opre;
          opre.load(arena, tl, L.bond[0], L.bond[1]);
          for (int i = 0; i < n; ++i) {
            const int chl = L.bond[i], chr = L.bond[i + 1];
            const int xb = diff ? 0 : (int)((xw >> (n - 1 - i)) & 1ull);
            const uint32_t tb = whole ? X.xbits[i] : (uint32_t)xb;
            cx<S> (*const A)[CM][2][CM] = stg[i & 1];
            const cd* oes = eslot(i);
            opre.stage_a(A, tl, (S)1.0);
            if (i + 1 < n) opre.load(arena + (int64_t)(i + 1) * SLOT, tl, L.bond[i + 1], L.bond[i + 2]);
            lds_sync();
            cd (*const vin)[CM] = ovb[i & 1];
            cd (*const vout)[CM] = ovb[(i + 1) & 1];
            for (int t = 0; t < NV; ++t) {
              const int el = tl + t * TW;
              const int tt = el / CM, col = el % CM;
              if (tt < T && col < chr) {
                const int xs = (int)((tb >> tt) & 1u);
                cd acc = {0.0, 0.0};
                for (int b = 0; b < chl; ++b) {
                  // an edge site from its complex-FP64 edge slot
                  const cd a0 = oes ? oes[b * 2 * D + col] : up(A[0][b][0][col]);
                  const cd a1 = oes ? oes[b * 2 * D + D + col] : up(A[0][b][1][col]);
                  const cd av = diff ? kInvSqrt2 * (a0 + a1) : (xs ? a1 : a0);
                  acc = cfma(acc, vin[tt][b], av);
                }
                vout[tt][col] = acc;
              }
            }
            f64 += 8.0 * (double)T * chl * chr;
          }
          lds_sync();
          if (tl < T) X.ovs[tl] = c1 * ovb[n & 1][tl][0];
          lds_sync();
        }

        // ---------------------------------------------- QR sweep with the MPO fused
        int r = 1;
        if (tl == 0) {
          L.rdim[0] = 1;
          // the first site's tile is [A | P A] itself: R = [1 1] over the two MPO blocks
          // (pre-contracted: [A | e_1 .. e_T], R = [1, c1 <p_1|psi>, .., c1 <p_T|psi>])
          L.u.q.R[0][0] = {1.0, 0.0};
          if (sumv)
            for (int t = 0; t < T; ++t) L.u.q.R[0][1 + t] = X.ovs[t];
          else
            L.u.q.R[0][1] = {1.0, 0.0};
        }
        TeamAPre<S, CM, TW> apre;
        apre.load(arena, tl, L.bond[0], L.bond[1]);
        lds_sync();
        for (int i = 0; i < n; ++i) {
          const int chl = L.bond[i], chr = L.bond[i + 1];
          const bool first = (i == 0), last = (i == n - 1);
          const int xb = diff ? 0 : (int)((xw >> (n - 1 - i)) & 1ull);
          // qubit values of the terms at this site (oracle terms; unused by the diffusion)
          const uint32_t tb = whole ? X.xbits[i] : (uint32_t)xb;
          const int Dl = first ? 1 : (sumv ? chl + T : 2 * chl);
          const int Dr = last ? 1 : (sumv ? chr + T : 2 * chr);
          cx<S>* slot = arena + (int64_t)i * SLOT;
          cd* es = eslot(i);
          if (sumv) {
            apre.stage_a64(L.u.q.W, es, tl, last ? c0 : 1.0);
          } else {
            apre.stage64(L.u.q.W, es, tl, diff, xb, last ? c0 : 1.0, last ? c1 : 1.0);
          }
          if (i + 1 < n) apre.load(arena + (int64_t)(i + 1) * SLOT, tl, L.bond[i + 1], L.bond[i + 2]);
          lds_sync();
          // X = R_{i-1} * MPO(A_i): this slot's column, rows (a, s) = part + PQ*e
          cd x[RQ];
          if (!sumv) {
            const int beta = (!last && qc >= chr) ? 1 : 0;
            const int bcol = qc - beta * chr;
#pragma unroll
            for (int e = 0; e < RQ; ++e) {
              const int row = qh + PQ * e;
              const int a = row >> 1, s = row & 1;
              cd acc = {0.0, 0.0};
              if (row < 2 * r && qc < Dr) {
                // the last site sums both MPO blocks into its one column
#pragma unroll
                for (int bl = 0; bl < 2; ++bl) {
                  if (last || bl == beta) {
#pragma unroll
                    for (int ap = 0; ap < CM; ++ap)
                      if (ap < chl) acc = cfma(acc, L.u.q.R[a][bl * chl + ap], L.u.q.W[bl][ap][s][bcol]);
                  }
                }
              }
              x[e] = acc;
            }
          } else {
            // columns < chr (or the last site's one column): R_A A_i in the storage
            // precision; term columns chr + t: R[:, chl + t] e_t(s), exact in FP64 (the last
            // site adds them to its one column)
            const bool acol = last || qc < chr;
            const int ct = qc - chr;
#pragma unroll
            for (int e = 0; e < RQ; ++e) {
              const int row = qh + PQ * e;
              const int a = row >> 1, s = row & 1;
              cd xv = {0.0, 0.0};
              if (row < 2 * r && qc < Dr) {
                if (acol) {
                  const int bcol = last ? 0 : qc;
                  cd acc = {0.0, 0.0};
#pragma unroll
                  for (int ap = 0; ap < CM; ++ap)
                    if (ap < chl) acc = cfma(acc, L.u.q.R[a][ap], L.u.q.W[0][ap][s][bcol]);
                  xv = acc;
                  if (last) {
                    for (int t = 0; t < T; ++t) {
                      const double es = diff ? kInvSqrt2 : ((int)((tb >> t) & 1u) == s ? 1.0 : 0.0);
                      xv = xv + es * L.u.q.R[a][chl + t];
                    }
                  }
                } else {
                  const double es = diff ? kInvSqrt2 : ((int)((tb >> ct) & 1u) == s ? 1.0 : 0.0);
                  xv = es * L.u.q.R[a][chl + ct];
                }
              }
              x[e] = xv;
            }
          }
          f64 += 8.0 * (sumv ? (double)r * chl * 2.0 * (last ? 1 : chr) : (double)r * Dl * 2.0 * Dr);
          if (last) {
            // the last site holds the norm: to its edge slot in FP64, to its site slot as stored
            if (real && qc == 0) {
#pragma unroll
              for (int e = 0; e < RQ; ++e) {
                const int row = qh + PQ * e;
                if (row < 2 * r) {
                  slot[(row >> 1) * 2 * D + (row & 1) * D] = store_cast<S>(x[e], rs_state, sr);
                  es[(row >> 1) * 2 * D + (row & 1) * D] = x[e];
                }
              }
            }
            if (tl == 0) {
              L.rdim[n - 1] = r;
              L.rdim[n] = 1;
            }
            break;
          }
          const int m = 2 * r;
          cd q[RQ];
          double qdrop = 0.0;
          int kr;
          if constexpr (TW <= 64)
            kr = team_qr_wave<TW, PQ, RQ, KQ>(x, q, base, qc, qh, m, Dr, chr, rank2, &qdrop, L.u.q.V, L.u.q.tau);
          else
            kr = team_qr_lds<PQ, RQ, KQ>(x, q, qc, qh, m, Dr, chr, rank2, &qdrop, L.u.q.V, L.u.q.tau, L.colv);
          truncw = fmax(truncw, qdrop);
          {
            const double mm = m, cc = Dr, kk = kr;
            f64 += 8.0 * (2.0 * mm * cc * kk - (mm + cc) * kk * kk + 2.0 * kk * kk * kk / 3.0) +
                   8.0 * (2.0 * mm * kk * kk - 2.0 * kk * kk * kk / 3.0);
          }
          cx<S> qs[RQ];  // Q as stored
#pragma unroll
          for (int e = 0; e < RQ; ++e) qs[e] = store_cast<S>(q[e], rs_state, sr);
          if (real && qc < kr) {
#pragma unroll
            for (int e = 0; e < RQ; ++e) {
              const int row = qh + PQ * e;
              if (row < m) {
                slot[(row >> 1) * 2 * D + (row & 1) * D + qc] = qs[e];
                if (es) es[(row >> 1) * 2 * D + (row & 1) * D + qc] = q[e];
              }
            }
          }
          if (qc < Dr) {
#pragma unroll
            for (int e = 0; e < RQ; ++e) {
              const int row = qh + PQ * e;
              if (row < kr) L.u.q.R[row][qc] = x[e];
            }
          }
          if (kMixed && !es) {
            comp_store_cols<PQ, RQ, KQ, D>(q, qs, qc, qh, kr, Dr, L.u.q.V, L.zbuf(), L.u.q.R);
            f64 += 8.0 * ((double)kr * kr * m + (double)kr * kr * Dr);
          }
          if (tl == 0) L.rdim[i + 1] = kr;
          r = kr;
          lds_sync();
        }
        // the QR sweep's site tensors are read by every wave of the team from here on
        team_sync_global();

        // ---------------------------------------------- truncated-SVD sweep
        // At site i the tile is M = Q_i (U Sigma)_{i+1} reshaped (r_i, 2 chi'); Jacobi runs on
        // the r_i columns of M^H: M^H J = V Sigma with J = U, so V^H = Sigma^{-1} (M^H J)^H
        // stays in site i and U Sigma = J Sigma moves left.
        if (tl == 0) L.u.s.Y[0][0] = {1.0, 0.0};
        TeamQPre<S, KQ, CM, TW> qpre;
        TeamWPre<KJ, TW> wpre;
        qpre.load(arena + (int64_t)(n - 1) * SLOT, tl, L.rdim[n - 1], L.rdim[n]);
        wpre.load(warm ? warm + ((int64_t)j * n + (n - 1)) * WREC : wdummy, warm != nullptr, tl, (L.rdim[n - 1] + 1) & ~1);
        for (int i = n - 1; i >= 1; --i) {
          const int ri = L.rdim[i], rn = L.rdim[i + 1];
          const int chn = L.bond[i + 1];
          const int c = 2 * chn;
          const int ncj = (ri + 1) & ~1;
          cx<S>* slot = arena + (int64_t)i * SLOT;
          cd* es = eslot(i);
          double* wrec = warm ? warm + ((int64_t)j * n + i) * WREC : nullptr;
          const bool use_warm = wrec && wpre.r() == ncj;
          // the stored unitary is a product of exact rotations, so its unitarity drifts by
          // ~1e-16 per use; one Newton-Schulz step every 64 iterations keeps it below ~1e-13
          const bool renorm_warm = use_warm && ((k_done0 + (uint64_t)it) & 63ull) == 0ull;
          if (es) {
            // an edge site (the first one holds the norm): from its complex-FP64 edge slot
            for (int e = tl; e < KQ * 2 * KQ; e += TW) {
              const int a = e / (2 * KQ), s = (e / KQ) & 1, b = e % KQ;
              (&L.u.s.Q[0][0][0])[e] = (a < ri && b < rn) ? es[a * 2 * D + s * D + b] : cd{0.0, 0.0};
            }
          } else {
            qpre.stage(&L.u.s.Q[0][0][0], tl);
          }
          if (use_warm) wpre.stage(&L.u.s.W[0][0], tl);
          if (i - 1 >= 1) {
            qpre.load(arena + (int64_t)(i - 1) * SLOT, tl, L.rdim[i - 1], L.rdim[i]);
            wpre.load(warm ? warm + ((int64_t)j * n + (i - 1)) * WREC : wdummy, warm != nullptr, tl,
                      (L.rdim[i - 1] + 1) & ~1);
          }
          lds_sync();
          // column jc of M^H: M^H[(s, jj)][a] = conj(sum_b Q[a][s][b] Y[b][jj])
          cd a[RJ];
#pragma unroll
          for (int e = 0; e < RJ; ++e) {
            const int row = jh + PJ * e;
            const int s = row >= chn ? 1 : 0;
            const int jj = row - s * chn;
            cd acc = {0.0, 0.0};
            if (jc < ri && row < c) {
#pragma unroll
              for (int b = 0; b < KQ; ++b)
                if (b < rn) acc = cfma(acc, L.u.s.Q[jc][s][b], L.u.s.Y[b][jj]);
            }
            a[e] = conj(acc);
          }
          f64 += 8.0 * (double)ri * 2.0 * rn * chn;
          if (renorm_warm) {
            // one Newton-Schulz polar step W <- W (3I - W^H W) / 2 (error e -> O(e^2))
            cd* WG = &L.u.s.XU[0][0][0];  // KJ x KJ, row-major
            for (int e = tl; e < KJ * KJ; e += TW) {
              const int ra = e / KJ, ca = e % KJ;
              cd g = {0.0, 0.0};
              for (int b = 0; b < ncj; ++b) g = g + cmulc(L.u.s.W[b][ra], L.u.s.W[b][ca]);
              WG[e] = g;
            }
            lds_sync();
            constexpr int NW = (KJ * KJ + TW - 1) / TW;
            cd wn[NW];
#pragma unroll
            for (int t = 0; t < NW; ++t) {
              const int e = tl + t * TW;
              const int ra = e / KJ, ca = e % KJ;
              cd acc = {0.0, 0.0};
              if (e < KJ * KJ)
                for (int b = 0; b < ncj; ++b) acc = cfma(acc, L.u.s.W[ra][b], WG[b * KJ + ca]);
              wn[t] = (e < KJ * KJ) ? 1.5 * L.u.s.W[ra][ca] - 0.5 * acc : cd{0.0, 0.0};
            }
            lds_sync();
#pragma unroll
            for (int t = 0; t < NW; ++t) {
              const int e = tl + t * TW;
              if (e < KJ * KJ) L.u.s.W[e / KJ][e % KJ] = wn[t];
            }
            lds_sync();
          }
          cd uu[RU];
          if (use_warm) {
            // start from the previous iteration's unitary: M^H <- M^H W
            if (jc < KJ) {
#pragma unroll
              for (int e = 0; e < RJ; ++e) L.u.s.XA[0][jc][jh + PJ * e] = a[e];
            }
            lds_sync();
#pragma unroll
            for (int e = 0; e < RJ; ++e) {
              const int row = jh + PJ * e;
              cd acc = {0.0, 0.0};
              if (jc < ncj)
                for (int b = 0; b < ncj; ++b) acc = cfma(acc, L.u.s.XA[0][b][row], L.u.s.W[b][jc]);
              a[e] = acc;
            }
#pragma unroll
            for (int e = 0; e < RU; ++e) {
              const int row = jh + PJ * e;
              uu[e] = (jc < ncj && row < ncj) ? L.u.s.W[row][jc] : cd{0.0, 0.0};
            }
            lds_sync();
          } else {
#pragma unroll
            for (int e = 0; e < RU; ++e) uu[e] = {(jh + PJ * e == jc && jc < ncj) ? 1.0 : 0.0, 0.0};
          }
          int sweeps;
          if constexpr (TW <= 64)
            sweeps = team_jacobi_wave<TW, PJ, RJ, RU>(a, uu, base, jc, jh, ncj, kJacobiTol2, skip2, P.max_sweeps);
          else
            sweeps = team_jacobi_lds<PJ, RJ, RU, KJ, T::NBUF>(a, uu, jc, jh, ncj, kJacobiTol2, skip2, P.max_sweeps,
                                                              L.u.s.XA, L.u.s.XU, L.u.s.XN, L.colv, L.colf);
          f64 += (double)sweeps * ri * (ri - 1) / 2.0 * 56.0 * c;
          // singular values, truncation and the kept order
          const bool colok = jc < ncj;
          double sg = 0.0;
#pragma unroll
          for (int e = 0; e < RJ; ++e) sg += norm2(a[e]);
          sg = gsum<PJ>(sg);
          // kept columns stay in their index order (so the bond basis, and the next warm
          // start, does not jump when Schmidt values are degenerate); dropped ones follow
          double stot, dropped;
          int chi_new, pos;
          bool keep;
          if constexpr (TW <= 64) {
            const double mine = colok ? sg : 0.0;
            const double smax = tmax<TW>(mine);
            stot = tsum<TW>(jh == 0 ? mine : 0.0);
            const int above = (int)tsum<TW>((jh == 0 && mine > 0.0 && mine >= tol2 * smax) ? 1.0 : 0.0);
            int rk = 0;
            for (int o = 0; o < ncj; ++o) {
              const double v = shfl_f64(mine, base + o * PJ);
              rk += (v > sg || (v == sg && o < jc)) ? 1 : 0;
            }
            chi_new = above < cap ? above : cap;
            if (chi_new < 1) chi_new = 1;
            keep = colok && rk < chi_new;
            const uint64_t kept = tballot<TW>(jh == 0 && keep, base);
            const int nk = __popcll(kept & ((1ull << (base + jc * PJ)) - 1ull));
            pos = keep ? nk : chi_new + (jc - nk);
            dropped = tsum<TW>((jh == 0 && colok && !keep) ? sg : 0.0);
          } else {
            if (jh == 0) L.colv[jc] = colok ? sg : 0.0;
            lds_sync();
            double smax = 0.0;
            stot = 0.0;
            for (int o = 0; o < ncj; ++o) {
              const double v = L.colv[o];
              smax = fmax(smax, v);
              stot += v;
            }
            int above = 0, rk = 0;
            for (int o = 0; o < ncj; ++o) {
              const double v = L.colv[o];
              above += (v > 0.0 && v >= tol2 * smax) ? 1 : 0;
              rk += (v > sg || (v == sg && o < jc)) ? 1 : 0;
            }
            chi_new = above < cap ? above : cap;
            if (chi_new < 1) chi_new = 1;
            if (jh == 0) L.colr[jc] = colok ? rk : KJ + jc;
            lds_sync();
            dropped = 0.0;
            int nk = 0, nd = 0;
            for (int o = 0; o < ncj; ++o) {
              const bool ko = L.colr[o] < chi_new;
              if (!ko) dropped += L.colv[o];
              if (o < jc) {
                nk += ko ? 1 : 0;
                nd += ko ? 0 : 1;
              }
            }
            keep = colok && rk < chi_new;
            pos = keep ? nk : chi_new + nd;
          }
          if (stot > 0.0) truncw = fmax(truncw, dropped / stot);
          if (!isfinite(stot)) status |= GMPS_ST_NAN;
          if (wrec && real) {
            // keep J with its columns in the kept order for the next iteration
            if (colok) {
#pragma unroll
              for (int e = 0; e < RU; ++e) {
                const int row = jh + PJ * e;
                if (row < ncj) {
                  wrec[2 + 2 * (row * KJ + pos)] = uu[e].re;
                  wrec[3 + 2 * (row * KJ + pos)] = uu[e].im;
                }
              }
            }
            if (tl == 0) wrec[0] = (double)ncj;
          }
          const double rs = keep ? rsqrt_acc(sg) : 0.0;  // 1/sigma
          cd wv[RJ];     // this slot's row of V^H
          cx<S> vs[RJ];  // ... as stored
#pragma unroll
          for (int e = 0; e < RJ; ++e) {
            wv[e] = rs * conj(a[e]);
            vs[e] = store_cast<S>(wv[e], rs_state, sr);
          }
          if (keep && real) {
#pragma unroll
            for (int e = 0; e < RJ; ++e) {
              const int row = jh + PJ * e;
              if (row < c) {
                const int s = row >= chn ? 1 : 0;
                const int jp = row - s * chn;
                slot[pos * 2 * D + s * D + jp] = vs[e];
                if (es) es[pos * 2 * D + s * D + jp] = wv[e];
              }
            }
          }
          cd yv[RU];  // this slot's column of the carry J Sigma
#pragma unroll
          for (int e = 0; e < RU; ++e) yv[e] = (sg * rs) * uu[e];
          if (kMixed && !es) {
            // the Jacobi exchange buffers are free: the kept rows and Z go there
            comp_store_rows<PJ, RJ, RU, CM>(wv, vs, yv, keep, pos, jh, c, ri, chi_new,
                                            reinterpret_cast<cd*>(&L.u.s.XA[0][0][0]),
                                            reinterpret_cast<cd*>(&L.u.s.XU[0][0][0]), L.u.s.Y);
            f64 += 8.0 * ((double)chi_new * chi_new * c + (double)chi_new * chi_new * ri);
          }
          if (keep) {
#pragma unroll
            for (int e = 0; e < RU; ++e) {
              const int row = jh + PJ * e;
              if (row < ri) L.u.s.Y[row][pos] = yv[e];
            }
          }
          if (tl == 0) L.bond[i] = chi_new;
          lds_sync();
        }
        // ---------------------------------------------- site 0 (holds the norm)
        team_sync_global();
        {
          const int rn = L.rdim[1], chn = L.bond[1];
          cx<S>* slot = arena;
          cd acc = {0.0, 0.0};
          const bool act = tl < 2 * chn;
          const int s = tl >= chn ? 1 : 0;
          const int jj = tl - s * chn;
          if (act) {
#pragma unroll
            for (int b = 0; b < KQ; ++b)
              if (b < rn) acc = cfma(acc, edges[s * D + b], L.u.s.Y[b][jj]);
          }
          f64 += 8.0 * 2.0 * rn * chn;
          double nn = 0.0;
          if constexpr (TW <= 64) {
            nn = tsum<TW>(act ? norm2(acc) : 0.0);
          } else {
            L.colv[tl] = act ? norm2(acc) : 0.0;
            lds_sync();
            for (int o = 0; o < 2 * chn; ++o) nn += L.colv[o];
          }
          if (!isfinite(nn) || !(nn > 0.0)) status |= GMPS_ST_NAN;
          const double nr = sqrt(nn);
          if (diff) drift = fmax(drift, fabs(nr - 1.0));
          // site 0 now holds the norm: to its edge slot in FP64, to its site slot as stored
          const cd outd = (diff ? 1.0 / nr : 1.0) * acc;
          const cx<S> out = store_cast<S>(outd, rs_state, sr);
          lds_sync();
          if (real && act) {
            slot[s * D + jj] = out;
            edges[s * D + jj] = outd;
          }
          if (tl == 0) L.bond[0] = 1;
          team_sync_global();
        }
      }
    }
  }

  // ------------------------------------------------------------------ write back
  if (real) {
    for (int l = tl; l < kBondStride; l += TW) P.bonds[(int64_t)me * kBondStride + l] = L.bond[l];
    if (tl == 0) {
      I->k_done += k;
      I->flops64 += f64;
      I->flops32 += f32;
      I->drift = fmax(I->drift, drift);
      I->trunc_w = fmax(I->trunc_w, truncw);
      if (drift > 1e-3) status |= GMPS_ST_DRIFT;
      if (truncw > 1e-8) status |= GMPS_ST_TRUNC;
      I->status |= status;
    }
  }
  team_sync_global();
}

// Persistent kernel of one team class W: a workgroup takes bundles from the class's queue
// until it is empty.
// Persistent kernel of the pre-contracted reflections for team class W.
template <class S, int W>
__global__ __launch_bounds__(kWide[W].TW < 64 ? 64 : kWide[W].TW) void grover_team_pc_kernel(IterParams P) {
  extern __shared__ __align__(16) char lds[];
  __shared__ unsigned int next_bundle;
  for (;;) {
    if (threadIdx.x == 0) next_bundle = atomicAdd(&P.queue->next, 1u);
    lds_sync();
    const unsigned int bi = next_bundle;
    lds_sync();
    if ((int)bi >= P.queue->nbundles) break;
    run_team_pc<S, kWide[W].CM, kWide[W].TW>(P, P.bundles + bi, lds);
  }
}

// Launch and occupancy of class W, defined in the class's own translation unit.
template <int W>
hipError_t launch_team_w(bool mixed, const IterParams& P, int grid, size_t lds, hipStream_t st);
template <int W>
hipError_t occupancy_team_w(bool mixed, size_t lds, int* blocks_per_cu);

#define GMPS_TEAM_CLASS(W)                                                                           \
  template <>                                                                                        \
  hipError_t launch_team_w<W>(bool mixed, const IterParams& P, int grid, size_t lds, hipStream_t st) { \
    constexpr int nt = kWide[W].TW < 64 ? 64 : kWide[W].TW;                                           \
    if (mixed)                                                                                       \
      grover_team_kernel<float, W><<<grid, nt, lds, st>>>(P);                                         \
    else                                                                                             \
      grover_team_kernel<double, W><<<grid, nt, lds, st>>>(P);                                        \
    return hipGetLastError();                                                                        \
  }                                                                                                  \
  template <>                                                                                        \
  hipError_t occupancy_team_w<W>(bool mixed, size_t lds, int* blocks_per_cu) {                      \
    constexpr int nt = kWide[W].TW < 64 ? 64 : kWide[W].TW;                                           \
    return mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_team_kernel<float, W>, nt, lds) \
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_team_kernel<double, W>, nt, lds); \
  }

// The pre-contracted kernels of a class (classes with bond caps up to 17).
template <int W>
hipError_t launch_team_pc_w(bool mixed, const IterParams& P, int grid, size_t lds, hipStream_t st);
template <int W>
hipError_t occupancy_team_pc_w(bool mixed, size_t lds, int* blocks_per_cu);

// Instantiated for FP64 storage only: gmps_create refuses pre-contraction on the mixed path.
#define GMPS_TEAM_PC_CLASS(W)                                                                        \
  template <>                                                                                        \
  hipError_t launch_team_pc_w<W>(bool mixed, const IterParams& P, int grid, size_t lds, hipStream_t st) { \
    constexpr int nt = kWide[W].TW < 64 ? 64 : kWide[W].TW;                                           \
    if (mixed) return hipErrorInvalidValue;                                                          \
    grover_team_pc_kernel<double, W><<<grid, nt, lds, st>>>(P);                                       \
    return hipGetLastError();                                                                        \
  }                                                                                                  \
  template <>                                                                                        \
  hipError_t occupancy_team_pc_w<W>(bool mixed, size_t lds, int* blocks_per_cu) {                   \
    constexpr int nt = kWide[W].TW < 64 ? 64 : kWide[W].TW;                                           \
    if (mixed) return hipErrorInvalidValue;                                                          \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_team_pc_kernel<double, W>, nt, lds); \
  }

// The gate-level circuit kernels of a class (FP64 storage, classes with bond caps up to 17).
template <int W>
hipError_t launch_team_circ_w(const IterParams& P, int grid, size_t lds, hipStream_t st);
template <int W>
hipError_t occupancy_team_circ_w(size_t lds, int* blocks_per_cu);

#define GMPS_TEAM_CIRC_CLASS(W)                                                                      \
  template <>                                                                                        \
  hipError_t launch_team_circ_w<W>(const IterParams& P, int grid, size_t lds, hipStream_t st) {      \
    constexpr int nt = kWide[W].TW < 64 ? 64 : kWide[W].TW;                                           \
    grover_team_circ_kernel<double, W><<<grid, nt, lds, st>>>(P);                                     \
    return hipGetLastError();                                                                        \
  }                                                                                                  \
  template <>                                                                                        \
  hipError_t occupancy_team_circ_w<W>(size_t lds, int* blocks_per_cu) {                             \
    constexpr int nt = kWide[W].TW < 64 ? 64 : kWide[W].TW;                                           \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_team_circ_kernel<double, W>, nt, lds); \
  }

}  // namespace gmps
