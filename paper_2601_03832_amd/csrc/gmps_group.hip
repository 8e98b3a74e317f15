// Lane-group iterate kernel of libgmps: iterative Grover search on matrix product states
// (gfx950), for bond caps up to 6.
//
// Layout. One wave (64 lanes) takes one bundle of instances from a persistent queue;
// each instance owns a group of G consecutive lanes. Inside a group a tile is held row
// per lane in registers: lane l keeps row l of the current QR tile (rows (a, s) of the
// reshaped site tensor) or of the current SVD tile. Column sums (inner products over
// rows) are butterfly reductions across the group, so every lane of a group ends with
// bit-identical sums and takes the same branch.
//
// One reflection c0*I + c1*(P_0 x ... x P_{n-1}) (the oracle for one marked x, or the
// diffusion of Eq. (4) with P = |+><+|) is applied as a bond-2 MPO whose site blocks are
// built while the site is staged, then recompressed (Section III-B):
//   QR sweep  i = 0..n-1 : X = R_{i-1} * MPO(A_i) reshaped (2r, D), Householder QR,
//                          Q stays in the site slot, R moves on (the last site keeps X).
//   SVD sweep i = n-1..1 : M = Q_i * (U Sigma)_{i+1} reshaped (r, 2 chi'), one-sided
//                          Jacobi SVD, keep sigma >= tol * sigma_max (at most the cap),
//                          V^dagger stays, U Sigma moves left.
//   site 0               : Q_0 * (U Sigma)_1, renormalised after the diffusion.
// The storage / contraction type S is double (FP64 path) or float (complex64 site tensors
// and contractions). The factorisation type C (QR, SVD, norms) is double on the FP64 and
// mixed paths and float on the all-FP32 path.
#include <hip/hip_runtime.h>

#include "gmps_device.h"

namespace gmps {

// ------------------------------------------------------------------------------- QR
// Householder QR of an m x c tile X held row per lane (row gl in x[], m <= G, c <= NC;
// rows >= m and columns >= c are zero), stopped at the numerical rank: before step j > 0
// the squared norm T_j of the trailing block X[j:, j:] is compared with rank2 * ||X||^2,
// and the factorisation ends when it falls below, or after KMAX steps. Returns the rank k
// kept; lanes gl < k then hold row gl of R (k x c, in pivoted column order) in x[] and
// q[] holds row gl of the thin Q (m x k), so X P = Q R + E with ||E||^2 = T_k
// (*dropped = T_k/||X||^2), where column perm[t] of X sits in position t.
// A tile after a bond-2 MPO has its columns in the order [A block (npiv) | P A block]. The
// A block has full rank and is eliminated in its own order; the projector block adds one
// direction (rank chi + 1 in all), which need not lie in the block's first column, so from
// step npiv on the remaining column with the largest residual norm is pivoted in first.
// Below `zero` a squared norm counts as zero. In FP32 the squares of entries near 1e-20 are
// denormals, which v_rsq_f32 / v_rcp_f32 flush to zero (an infinite estimate, and NaN after
// the Newton step), so the FP32 instantiation treats squared norms below 1e-30 as zero.
template <class C>
struct QrLimits;
template <>
struct QrLimits<double> {
  static constexpr double zero = 0.0;
};
template <>
struct QrLimits<float> {
  static constexpr float zero = 1e-30f;
};

template <class C, int G, int NC, int KMAX>
__device__ __forceinline__ int householder_qr_rank(cx<C> (&x)[NC], cx<C> (&q)[KMAX], int (&perm)[NC], int gl, int m,
                                                   int c, int npiv, C rank2, double* dropped) {
  using T = cx<C>;
  const int kmax = min(min(m, c), KMAX);
  T hv[KMAX];
  C tau[KMAX];
#pragma unroll
  for (int k = 0; k < NC; ++k) perm[k] = k;
  C t0 = 0;
#pragma unroll
  for (int k = 0; k < NC; ++k) t0 += norm2(x[k]);
  t0 = gsum<G>(gl < m ? t0 : 0.0);
  int kr = kmax;
  bool done = false;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    hv[j] = czero<C>();
    tau[j] = 0;
    if (j > 0 && !done && j < kmax) {
      C tj = 0;
#pragma unroll
      for (int k = j; k < NC; ++k) tj += norm2(x[k]);
      tj = gsum<G>((gl >= j && gl < m) ? tj : C(0));
      if (tj <= rank2 * t0) {
        done = true;
        kr = j;
      }
    }
    if (!done && j < kmax && j >= npiv) {
      // pivot: the remaining column with the largest norm below row j
      C best = -1;
      int p = j;
#pragma unroll
      for (int k = j; k < NC; ++k) {
        if (k < c) {
          const C nk = gsum<G>((gl >= j && gl < m) ? norm2(x[k]) : C(0));
          if (nk > best) {
            best = nk;
            p = k;
          }
        }
      }
#pragma unroll
      for (int k = j + 1; k < NC; ++k) {
        if (k == p) {
          const T t = x[j];
          x[j] = x[k];
          x[k] = t;
          const int pt = perm[j];
          perm[j] = perm[k];
          perm[k] = pt;
        }
      }
    }
    if (!done && j < kmax) {
      const T xj = x[j];
      const C sub = gsum<G>((gl > j && gl < m) ? norm2(xj) : C(0));
      const T alpha = gbcast<G>(xj, gl, j);
      const C a2 = norm2(alpha);
      const bool refl = sub > QrLimits<C>::zero;
      const bool anz = a2 > QrLimits<C>::zero;
      const C ra = anz ? rsqrt_acc(a2) : C(0);
      const C aa = a2 * ra;                               // |alpha|
      const C n2 = a2 + sub;
      const C nrm = refl ? n2 * rsqrt_acc(n2) : aa;       // norm of column j from the diagonal down
      const T ph = anz ? T{alpha.re * ra, alpha.im * ra} : T{C(1), C(0)};
      const T beta = {-ph.re * nrm, -ph.im * nrm};
      const C t = refl ? rcp_acc(nrm * (nrm + aa)) : C(0);
      T v = (gl == j) ? alpha - beta : ((gl > j && gl < m) ? xj : czero<C>());
      if (!refl) v = czero<C>();
      T w[NC];
#pragma unroll
      for (int k = j + 1; k < NC; ++k)
        if (k < c) w[k] = gsum<G>(cmulc(v, x[k]));
#pragma unroll
      for (int k = j + 1; k < NC; ++k)
        if (k < c) {
          const T tw = t * w[k];
          x[k] = x[k] - v * tw;
        }
      if (refl) x[j] = (gl == j) ? beta : ((gl > j) ? czero<C>() : xj);
      hv[j] = v;
      tau[j] = t;
    }
  }
  C tk = 0;
#pragma unroll
  for (int k = 0; k < NC; ++k) tk += (k >= kr) ? norm2(x[k]) : C(0);
  tk = gsum<G>((gl >= kr && gl < m) ? tk : C(0));
  *dropped = t0 > 0 ? (double)(tk / t0) : 0.0;
  // thin Q = H_0 ... H_{kr-1} [I; 0], applied right to left
#pragma unroll
  for (int k = 0; k < KMAX; ++k) q[k] = {(gl == k && k < kr) ? C(1) : C(0), C(0)};
#pragma unroll
  for (int j = KMAX - 1; j >= 0; --j) {
    if (j < kr && tau[j] != 0) {
      T w[KMAX];
#pragma unroll
      for (int k = j; k < KMAX; ++k)
        if (k < kr) w[k] = gsum<G>(cmulc(hv[j], q[k]));
#pragma unroll
      for (int k = j; k < KMAX; ++k)
        if (k < kr) {
          const T tw = tau[j] * w[k];
          q[k] = q[k] - hv[j] * tw;
        }
    }
  }
  return kr;
}

// ---------------------------------------------------------------------------- Jacobi SVD
// One-sided (Hestenes) Jacobi on the first NC columns of a tile held row per lane in a[]
// over a lane group of W lanes (rows beyond the tile are zero), accumulating V (NC x NC,
// row gl in v[]). For a pair (i, j) with gamma = a_i^H a_j and phi = arg(gamma), the rotation
//   a_i' = c a_i - s e^{-i phi} a_j,   a_j' = s e^{i phi} a_i + c a_j,
// with t = s/c the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = (|a_j|^2 - |a_i|^2)/(2|gamma|),
// makes the pair orthogonal and moves t|gamma| of squared norm from a_i to a_j; the norms are
// tracked that way within a sweep and recomputed at the start of the next.
// A pair is skipped when it is already orthogonal to tol2 (relative, squared) or when one
// of its columns lies at the rounding-noise floor of the tile (skip2 * largest squared
// norm): such a column is dropped by the truncation, and leaving it unrotated changes the
// kept part by no more than its own norm. Convergence is quadratic, so a sweep whose
// largest relative off-diagonal was below 1e-10 leaves ~1e-20 behind and ends the iteration.
// The all-FP32 instantiation stops at a relative off-diagonal of 1e-5 instead (its rounding
// floor is near 1e-7), and its guards against underflow and overflow are FP32 ones.
template <class C>
struct JacobiLimits;
template <>
struct JacobiLimits<double> {
  static constexpr double stop = 1e-20, tiny = 1e-300, huge = 1e300;
};
template <>
struct JacobiLimits<float> {
  static constexpr float stop = 1e-10f, tiny = 1e-36f, huge = 1e30f;
};

template <class C, int W, int NC, int NCM>
__device__ __forceinline__ int jacobi_fixed(cx<C> (&a)[NCM], cx<C> (&v)[NCM], C tol2, C skip2,
                                            int max_sweeps) {
  using T = cx<C>;
  using Lim = JacobiLimits<C>;
  int sweeps = 0;
  bool more = true;
  while (more && sweeps < max_sweeps) {
    ++sweeps;
    C nrm[NC];
    C amax = 0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      nrm[k] = gsum<W>(norm2(a[k]));
      amax = fmax(amax, nrm[k]);
    }
    const C floor2 = skip2 * amax;
    more = false;
#pragma unroll
    for (int r = 0; r < NC - 1; ++r) {
      T ga[NC / 2];
#pragma unroll
      for (int p = 0; p < NC / 2; ++p) {
        const int i = cmin(circ_a(NC, r, p), circ_b(NC, r, p));
        const int j = cmax(circ_a(NC, r, p), circ_b(NC, r, p));
        ga[p] = gsum<W>(cmulc(a[i], a[j]));
      }
#pragma unroll
      for (int p = 0; p < NC / 2; ++p) {
        const int i = cmin(circ_a(NC, r, p), circ_b(NC, r, p));
        const int j = cmax(circ_a(NC, r, p), circ_b(NC, r, p));
        const C g2 = norm2(ga[p]);
        const C ab = nrm[i] * nrm[j];
        if (g2 > tol2 * ab && fmin(nrm[i], nrm[j]) > floor2 && g2 > Lim::tiny) {
          more |= g2 > Lim::stop * ab;
          const C rg = rsqrt_acc(g2);                          // 1/|gamma|
          const C zeta = (nrm[j] - nrm[i]) * (C(0.5) * rg);
          const C az = fabs(zeta);
          const C u = fmin(fma(zeta, zeta, C(1)), Lim::huge);
          const C den = az + u * rsq_raw(u);                   // |zeta| + sqrt(1 + zeta^2)
          C t = rcp_raw(den);
          t = fma(t, fma(-den, t, C(1)), t);
          t = copysign(t, zeta);
          const C cs = rsqrt_acc(fma(t, t, C(1)));
          const C sn = cs * t;
          const T se = {sn * ga[p].re * rg, sn * ga[p].im * rg};  // s e^{i phi}
          rot2(a[i], a[j], cs, se);
          rot2(v[i], v[j], cs, se);
          const C tg = t * (g2 * rg);
          nrm[i] -= tg;
          nrm[j] += tg;
        }
      }
    }
  }
  return sweeps;
}

// Dispatches on the runtime (even) column count c <= NCM so that every round of the
// round-robin schedule is full.
// v[] must hold row gl of the starting unitary (the identity, or a warm start whose
// product with the tile is already in a[]).
template <class C, int W, int NCM>
__device__ __forceinline__ int jacobi_svd(cx<C> (&a)[NCM], cx<C> (&v)[NCM], int gl, int c, C tol2,
                                          C skip2, int max_sweeps) {
  switch (c) {
    case 2: return jacobi_fixed<C, W, 2, NCM>(a, v, tol2, skip2, max_sweeps);
    case 4: if constexpr (NCM >= 4) return jacobi_fixed<C, W, 4, NCM>(a, v, tol2, skip2, max_sweeps); break;
    case 6: if constexpr (NCM >= 6) return jacobi_fixed<C, W, 6, NCM>(a, v, tol2, skip2, max_sweeps); break;
    case 8: if constexpr (NCM >= 8) return jacobi_fixed<C, W, 8, NCM>(a, v, tol2, skip2, max_sweeps); break;
    case 10: if constexpr (NCM >= 10) return jacobi_fixed<C, W, 10, NCM>(a, v, tol2, skip2, max_sweeps); break;
    case 12: if constexpr (NCM >= 12) return jacobi_fixed<C, W, 12, NCM>(a, v, tol2, skip2, max_sweeps); break;
    default: break;
  }
  return 0;
}

// ---------------------------------------------------------------------------- per-group LDS
template <class S, class C, int CM>
struct GroupLds {
  static constexpr int D = 2 * CM;
  cx<C> X[2 * D][D];        // staged QR tile (rows (a, s)) or SVD tile (rows a)
  cx<C> R[D][D];            // R of the previous QR step
  cx<C> Y[D][CM];           // U Sigma of the previous SVD step
  cx<S> A[CM][2][CM];       // compressed site tensor, zero padded
  cx<C> U[CM + 2][CM + 2];  // warm-start unitary
  cx<C> UG[CM + 2][CM + 2]; // U^H U of the warm start
  int32_t bond[kBondStride];
  int32_t rdim[kBondStride];
};

// ----------------------------------------------------------------------- prefetched loads
// Site tensors are read one site ahead of their use: the loads for site i+1 (QR sweep) or
// i-1 (SVD sweep) are issued into registers while site i is being factorised, so the
// global-memory latency overlaps the arithmetic. The slot being prefetched is never written
// by the current step.

template <class S, int CM, int KQ>
struct QPrefetch {
  cx<S> v[2][KQ];
  __device__ __forceinline__ void load(const cx<S>* slot, int gl, int ri, int rn) {
    constexpr int D = 2 * CM;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int b = 0; b < KQ; ++b) {
        // unconditional load from a row inside the slot, masked afterwards (see APrefetch)
        const int gr = gl < D ? gl : D - 1;
        const cx<S> val = slot[gr * 2 * D + s * D + b];
        v[s][b] = (gl < ri && b < rn) ? val : czero<S>();
      }
  }
};

template <int KJ, int G>
struct WPrefetch {
  static constexpr int NE = (KJ * KJ + G - 1) / G;
  cd v[NE];
  int r;
  __device__ __forceinline__ void load(const WarmRec* w, int gl, int ncj) {
    r = w ? w->r : 0;
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = gl + t * G;
      const int ra = e / KJ, ca = e % KJ;
      v[t] = (w && e < KJ * KJ && ra < ncj && ca < ncj)
                 ? cd{w->u[2 * (ra * kWarmStride + ca)], w->u[2 * (ra * kWarmStride + ca) + 1]}
                 : cd{0.0, 0.0};
    }
  }
};

// ------------------------------------------------------------------------------ one bundle
template <class S, class C, int CM, int G, int WS>
__device__ void run_bundle(const IterParams& P, const Bundle* bdp, char* lds_base) {
  using T = cx<C>;
  constexpr int D = 2 * CM;
  constexpr int SLOT = slot_elems(CM);
  constexpr bool kMixed = sizeof(S) == sizeof(float);
  constexpr bool kF32 = sizeof(C) == sizeof(float);  // factorisations in FP32
  constexpr int KQ = CM + 1;                 // rank of a tile after the bond-2 MPO, at most
  constexpr int KJ = (KQ + 1) & ~1;          // Jacobi columns (even)
  static_assert(G >= 2 * KQ, "a lane group must hold a QR tile's rows");
  static_assert(WS >= D && WS >= KJ && WS <= G, "the SVD lanes must hold M^H's rows and J's rows");
  const int lane = threadIdx.x;
  const int grp = lane / G;
  const int gl = lane % G;
  const bool real = grp < bdp->count;
  // inst[] is indexed per lane: read it from memory, not from a register copy
  const int me = bdp->inst[real ? grp : 0];
  GroupLds<S, C, CM>& L = reinterpret_cast<GroupLds<S, C, CM>*>(lds_base)[grp];
  InstDev* I = P.inst + me;
  const int n = I->n;
  const int M = I->M;
  const int cap = I->cap < CM ? I->cap : CM;
  const int64_t k = bdp->k;
  cx<S>* arena = reinterpret_cast<cx<S>*>(P.arena) + I->site_off;
  const uint64_t* W = P.marked + I->marked_off;
  const C tol2 = (C)(P.trunc_tol * P.trunc_tol);
  const C rank2 = (C)(P.rank_tol * P.rank_tol);
  const bool sr = P.stoch_round != 0;
  WarmRec* warm = P.warm ? reinterpret_cast<WarmRec*>(reinterpret_cast<char*>(P.warm) + I->warm_off) : nullptr;
  // read once: a global load inside the sweeps would be waited for at its use
  const uint64_t k_done0 = (uint64_t)I->k_done;
  uint64_t rs_state = mix64(((uint64_t)me << 32) ^ (k_done0 * 0x9E3779B97F4A7C15ull) ^ (uint64_t)gl);

  for (int l = gl; l < kBondStride; l += G) L.bond[l] = P.bonds[(int64_t)me * kBondStride + l];
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
        const cx<S> a0 = arena[0], a1 = arena[D];
        cx<S> o = czero<S>();
        if (gl < 2) {
          const cx<S> pa = proj_apply<S>(a0, a1, gl, diff, xb);
          const cx<S> as = sel(a0, a1, gl);
          o = {(S)c0 * as.re + (S)c1 * pa.re, (S)c0 * as.im + (S)c1 * pa.im};
        }
        const C nn = gsum<G>(gl < 2 ? norm2(cvt<C>(o)) : C(0));
        if (diff) {
          const C nr = sqrt(nn);
          drift = fmax(drift, fabs((double)nr - 1.0));
          if (!(nn > 0) || !isfinite(nn)) status |= GMPS_ST_NAN;
          o = cvt<S>((C(1) / nr) * cvt<C>(o));
        }
        lds_sync();
        if (real && gl < 2) arena[gl * D] = o;
        lds_sync();
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
        if (gl == 0) {
          L.R[0][0] = {C(1), C(0)};
          L.rdim[0] = 1;
        }
        APrefetch<S, CM, G> apre;
        apre.load(arena, gl, L.bond[0], L.bond[1]);
        lds_sync();
        for (int i = 0; i < n; ++i) {
          const int chl = L.bond[i], chr = L.bond[i + 1];
          const bool first = (i == 0), last = (i == n - 1);
          const int xb = diff ? 0 : (int)((xw >> (n - 1 - i)) & 1ull);
          const int Dl = first ? 1 : 2 * chl;
          const int Dr = last ? 1 : 2 * chr;
          cx<S>* slot = arena + (int64_t)i * SLOT;
          apre.stage(&L.A[0][0][0], gl);
          if (i + 1 < n) apre.load(arena + (int64_t)(i + 1) * SLOT, gl, L.bond[i + 1], L.bond[i + 2]);
          lds_sync();
          if (gl < 2 * D) {
            const int a = gl >> 1, s = gl & 1;
            const bool rowok = a < r;
            if (!last) {
#pragma unroll
              for (int beta = 0; beta < 2; ++beta) {
#pragma unroll
                for (int b = 0; b < CM; ++b) {
                  if (b < chr) {
                    cx<S> acc = czero<S>();
                    if (rowok) {
                      if (first) {
                        const cx<S> a0 = L.A[0][0][b], a1 = L.A[0][1][b];
                        acc = beta == 0 ? sel(a0, a1, s) : proj_apply<S>(a0, a1, s, diff, xb);
                      } else {
#pragma unroll
                        for (int ap = 0; ap < CM; ++ap)
                          if (ap < chl) {
                            const cx<S> a0 = L.A[ap][0][b], a1 = L.A[ap][1][b];
                            const cx<S> wa = beta == 0 ? sel(a0, a1, s) : proj_apply<S>(a0, a1, s, diff, xb);
                            acc = cfma(acc, cvt<S>(L.R[a][beta * chl + ap]), wa);
                          }
                      }
                    }
                    L.X[gl][beta * chr + b] = cvt<C>(acc);
                  }
                }
              }
              for (int col = Dr; col < D; ++col) L.X[gl][col] = czero<C>();
            } else {
              cx<S> acc = czero<S>();
              if (rowok) {
#pragma unroll
                for (int al = 0; al < 2; ++al) {
                  const S cal = (S)(al == 0 ? c0 : c1);
#pragma unroll
                  for (int ap = 0; ap < CM; ++ap)
                    if (ap < chl) {
                      const cx<S> a0 = L.A[ap][0][0], a1 = L.A[ap][1][0];
                      const cx<S> wa = al == 0 ? sel(a0, a1, s) : proj_apply<S>(a0, a1, s, diff, xb);
                      acc = cfma(acc, cvt<S>(L.R[a][al * chl + ap]), cal * wa);
                    }
                }
              }
              L.X[gl][0] = cvt<C>(acc);
            }
          }
          const double macs = (double)r * Dl * 2.0 * Dr;
          if (kMixed) f32 += 8.0 * macs; else f64 += 8.0 * macs;
          lds_sync();
          if (last) {
            if (real && gl < 2 * r) {
              const int a = gl >> 1, s = gl & 1;
              slot[a * 2 * D + s * D] = store_cast<S>(L.X[gl][0], rs_state, sr);
            }
            if (gl == 0) {
              L.rdim[n - 1] = r;
              L.rdim[n] = 1;
            }
            lds_sync();
            break;
          }
          T xr[D], q[KQ];
#pragma unroll
          for (int col = 0; col < D; ++col) xr[col] = (gl < 2 * D) ? L.X[gl][col] : czero<C>();
          const int m = 2 * r;
          double qdrop = 0.0;
          int perm[D];
          const int kr = householder_qr_rank<C, G, D, KQ>(xr, q, perm, gl, m, Dr, last ? Dr : chr, rank2, &qdrop);
          truncw = fmax(truncw, qdrop);
          {
            const double mm = m, cc = Dr, kk = kr;
            const double fl = 8.0 * (2.0 * mm * cc * kk - (mm + cc) * kk * kk + 2.0 * kk * kk * kk / 3.0) +
                              8.0 * (2.0 * mm * kk * kk - 2.0 * kk * kk * kk / 3.0);
            if (kF32) f32 += fl; else f64 += fl;
          }
          if (real && gl < m) {
            const int a = gl >> 1, s = gl & 1;
#pragma unroll
            for (int col = 0; col < KQ; ++col)
              if (col < kr) slot[a * 2 * D + s * D + col] = store_cast<S>(q[col], rs_state, sr);
          }
          if (gl < kr) {
            // R P^T: column t of the pivoted R belongs to column perm[t] of the tile
#pragma unroll
            for (int col = 0; col < D; ++col) L.R[gl][perm[col]] = col < gl ? czero<C>() : xr[col];
          }
          if (gl == 0) L.rdim[i + 1] = kr;
          r = kr;
          lds_sync();
        }

        // ---------------------------------------------- truncated-SVD sweep
        // At site i the tile is M = Q_i (U Sigma)_{i+1} reshaped (r_i, 2 chi'). Jacobi runs on
        // the r_i columns of M^H (rows (s, j) on lanes): M^H J = V Sigma with J = U, so
        // V^H = Sigma^{-1} (M^H J)^H stays in site i and U Sigma = J Sigma moves left.
        if (gl == 0) L.Y[0][0] = {C(1), C(0)};
        QPrefetch<S, CM, KQ> qpre;
        WPrefetch<KJ, G> wpre;
        qpre.load(arena + (int64_t)(n - 1) * SLOT, gl, L.rdim[n - 1], L.rdim[n]);
        wpre.load(warm ? warm + ((int64_t)j * n + (n - 1)) : nullptr, gl, (L.rdim[n - 1] + 1) & ~1);
        lds_sync();
        for (int i = n - 1; i >= 1; --i) {
          const int ri = L.rdim[i], rn = L.rdim[i + 1];
          const int chn = L.bond[i + 1];
          const int c = 2 * chn;
          cx<S>* slot = arena + (int64_t)i * SLOT;
          const QPrefetch<S, CM, KQ> qcur = qpre;
          const WPrefetch<KJ, G> wcur = wpre;
          if (i - 1 >= 1) {
            qpre.load(arena + (int64_t)(i - 1) * SLOT, gl, L.rdim[i - 1], L.rdim[i]);
            wpre.load(warm ? warm + ((int64_t)j * n + (i - 1)) : nullptr, gl, (L.rdim[i - 1] + 1) & ~1);
          }
          if (gl < ri) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
              cx<S> qrow[KQ];
#pragma unroll
              for (int b = 0; b < KQ; ++b) qrow[b] = qcur.v[s][b];
#pragma unroll
              for (int jj = 0; jj < CM; ++jj)
                if (jj < chn) {
                  cx<S> acc = czero<S>();
#pragma unroll
                  for (int b = 0; b < KQ; ++b)
                    if (b < rn) acc = cfma(acc, qrow[b], cvt<S>(L.Y[b][jj]));
                  L.X[gl][s * chn + jj] = cvt<C>(acc);
                }
            }
          }
          {
            const double macs = (double)ri * 2.0 * rn * chn;
            if (kMixed) f32 += 8.0 * macs; else f64 += 8.0 * macs;
          }
          lds_sync();
          T mh[KJ], u[KJ];
#pragma unroll
          for (int a = 0; a < KJ; ++a) mh[a] = (gl < c && a < ri) ? conj(L.X[a][gl]) : czero<C>();
          const int ncj = (ri + 1) & ~1;
          // warm start: the unitary from this (reflection, site) in the previous iteration
          WarmRec* wrec = warm ? warm + ((int64_t)j * n + i) : nullptr;
          const bool use_warm = wrec && wcur.r == ncj;
          // the stored unitary is a product of exact rotations, so its unitarity drifts by
          // ~1e-16 per use; one Newton-Schulz step every 64 iterations keeps it below ~1e-13
          const bool renorm_warm = use_warm && ((k_done0 + (uint64_t)it) & 63ull) == 0ull;
          if (use_warm) {
#pragma unroll
            for (int t = 0; t < WPrefetch<KJ, G>::NE; ++t) {
              const int e = gl + t * G;
              const int ra = e / KJ, ca = e % KJ;
              if (e < KJ * KJ && ra < ncj && ca < ncj) L.U[ra][ca] = cvt<C>(wcur.v[t]);
            }
          }
          lds_sync();
          if (renorm_warm) {
            // one Newton-Schulz polar step U <- U (3I - U^H U) / 2 removes the unitarity
            // error the stored product picked up (error e -> O(e^2))
            if (gl < ncj) {
#pragma unroll
              for (int cc = 0; cc < KJ; ++cc)
                if (cc < ncj) {
                  T g = czero<C>();
#pragma unroll
                  for (int a = 0; a < KJ; ++a)
                    if (a < ncj) g = g + cmulc(L.U[a][gl], L.U[a][cc]);
                  L.UG[gl][cc] = g;
                }
            }
          }
          lds_sync();
          if (renorm_warm) {
            T un[KJ];
            if (gl < ncj) {
#pragma unroll
              for (int cc = 0; cc < KJ; ++cc) {
                T acc = czero<C>();
#pragma unroll
                for (int b = 0; b < KJ; ++b)
                  if (b < ncj && cc < ncj) acc = cfma(acc, L.U[gl][b], L.UG[b][cc]);
                un[cc] = cc < ncj ? C(1.5) * L.U[gl][cc] - C(0.5) * acc : czero<C>();
              }
            }
            lds_sync();
            if (gl < ncj) {
#pragma unroll
              for (int cc = 0; cc < KJ; ++cc)
                if (cc < ncj) L.U[gl][cc] = un[cc];
            }
          } else {
            lds_sync();
          }
          lds_sync();
          if (use_warm) {
            T t[KJ];
#pragma unroll
            for (int b = 0; b < KJ; ++b) {
              T acc = czero<C>();
#pragma unroll
              for (int a = 0; a < KJ; ++a)
                if (a < ncj && b < ncj) acc = cfma(acc, mh[a], L.U[a][b]);
              t[b] = acc;
            }
#pragma unroll
            for (int b = 0; b < KJ; ++b) {
              mh[b] = t[b];
              u[b] = (gl < ncj && b < ncj) ? L.U[gl][b] : T{(gl == b && b < ncj) ? C(1) : C(0), C(0)};
            }
          } else {
#pragma unroll
            for (int b = 0; b < KJ; ++b) u[b] = {(gl == b && b < ncj) ? C(1) : C(0), C(0)};
          }
          int sweeps = 0;
          if (gl < WS)
            sweeps = jacobi_svd<C, WS, KJ>(mh, u, gl, ncj, (C)kJacobiTol2, (C)(P.skip_tol * P.skip_tol), P.max_sweeps);
          else {
#pragma unroll
            for (int a = 0; a < KJ; ++a) u[a] = czero<C>();
          }
          sweeps = (int)gsum<G>(gl == 0 ? (double)sweeps : 0.0);
          {
            const double fl = (double)sweeps * ri * (ri - 1) / 2.0 * 56.0 * c;
            if (kF32) f32 += fl; else f64 += fl;
          }
          C sg[KJ];
          C smax = 0, stot = 0;
          // every column below ncj can carry weight (a warm start mixes the pad column in)
#pragma unroll
          for (int col = 0; col < KJ; ++col) {
            sg[col] = col < ncj ? gsum<G>(gl < c ? norm2(mh[col]) : C(0)) : C(0);
            smax = fmax(smax, sg[col]);
            stot += sg[col];
          }
          int above = 0;
#pragma unroll
          for (int col = 0; col < KJ; ++col)
            above += (col < ncj && sg[col] > QrLimits<C>::zero && sg[col] >= tol2 * smax) ? 1 : 0;
          int chi_new = above < cap ? above : cap;
          if (chi_new < 1) chi_new = 1;
          // keep the chi_new largest columns; kept columns stay in their index order (so the
          // bond basis, and the next warm start, does not jump when Schmidt values are
          // degenerate), dropped ones follow
          C dropped = 0;
          int rank[KJ];
          bool keep[KJ];
#pragma unroll
          for (int col = 0; col < KJ; ++col) {
            int rk = 0;
#pragma unroll
            for (int o = 0; o < KJ; ++o) rk += (sg[o] > sg[col] || (sg[o] == sg[col] && o < col)) ? 1 : 0;
            keep[col] = rk < chi_new;
            if (!keep[col]) dropped += sg[col];
          }
          {
            int nk = 0, nd = 0;
#pragma unroll
            for (int col = 0; col < KJ; ++col) {
              rank[col] = keep[col] ? nk : chi_new + nd;
              nk += keep[col] ? 1 : 0;
              nd += keep[col] ? 0 : 1;
            }
          }
          if (stot > 0) truncw = fmax(truncw, (double)(dropped / stot));
          if (!isfinite(stot)) status |= GMPS_ST_NAN;
          if (wrec && real) {
            // keep J with its columns in singular-value order for the next iteration
            if (gl < ncj) {
#pragma unroll
              for (int col = 0; col < KJ; ++col)
                if (col < ncj) {
                  const int rk = rank[col];
                  wrec->u[2 * (gl * kWarmStride + rk)] = u[col].re;
                  wrec->u[2 * (gl * kWarmStride + rk) + 1] = u[col].im;
                }
            }
            if (gl == 0) wrec->r = ncj;
          }
          lds_sync();
#pragma unroll
          for (int col = 0; col < KJ; ++col) {
            if (rank[col] < chi_new) {
              const int rk = rank[col];
              const C sig2 = sg[col];
              const C rs = rsqrt_acc(sig2);  // 1/sigma
              if (real && gl < c) {
                const int s = gl >= chn ? 1 : 0;
                const int jp = gl - s * chn;
                slot[rk * 2 * D + s * D + jp] = store_cast<S>(rs * conj(mh[col]), rs_state, sr);
              }
              if (gl < ri) L.Y[gl][rk] = (sig2 * rs) * u[col];
            }
          }
          if (gl == 0) L.bond[i] = chi_new;
          lds_sync();
        }
        // ---------------------------------------------- site 0 (holds the norm)
        {
          const int rn = L.rdim[1], chn = L.bond[1];
          cx<S>* slot = arena;
          cx<S> acc = czero<S>();
          const bool act = gl < 2 * chn;
          const int s = gl >= chn ? 1 : 0;
          const int jj = gl - s * chn;
          if (act) {
#pragma unroll
            for (int b = 0; b < KQ; ++b)
              if (b < rn) acc = cfma(acc, slot[s * D + b], cvt<S>(L.Y[b][jj]));
          }
          const double macs = 2.0 * rn * chn;
          if (kMixed) f32 += 8.0 * macs; else f64 += 8.0 * macs;
          const C nn = gsum<G>(act ? norm2(cvt<C>(acc)) : C(0));
          if (!isfinite(nn) || !(nn > 0)) status |= GMPS_ST_NAN;
          const C nr = sqrt(nn);
          if (diff) drift = fmax(drift, fabs((double)nr - 1.0));
          const cx<S> out = store_cast<S>((diff ? C(1) / nr : C(1)) * cvt<C>(acc), rs_state, sr);
          lds_sync();
          if (real && act) slot[s * D + jj] = out;
          if (gl == 0) L.bond[0] = 1;
          lds_sync();
        }
      }
    }
  }

  // ------------------------------------------------------------------ write back
  if (real) {
    for (int l = gl; l < kBondStride; l += G) P.bonds[(int64_t)me * kBondStride + l] = L.bond[l];
    if (gl == 0) {
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
  lds_sync();
}

template <class S, class C>
__global__ __launch_bounds__(64) void grover_group_kernel(IterParams P) {
  extern __shared__ __align__(16) char lds[];
  for (;;) {
    unsigned int bi = 0;
    if (threadIdx.x == 0) bi = atomicAdd(&P.queue->next, 1u);
    bi = __shfl(bi, 0);
    if ((int)bi >= P.queue->nbundles) break;
    const Bundle* bd = P.bundles + bi;
    switch (bd->cls) {
      case 0: run_bundle<S, C, 2, 8, 4>(P, bd, lds); break;
      case 1: run_bundle<S, C, 3, 8, 8>(P, bd, lds); break;
      case 2: run_bundle<S, C, 4, 16, 8>(P, bd, lds); break;
      case 3: run_bundle<S, C, 5, 16, 16>(P, bd, lds); break;
      case 4: run_bundle<S, C, 6, 16, 16>(P, bd, lds); break;
      default: break;
    }
  }
}

// ------------------------------------------------------------------------- launch wrappers
// mode: 0 FP64, 1 mixed (complex64 storage, FP64 factorisations), 2 all-FP32
hipError_t launch_group(int mode, const IterParams& P, int grid, size_t lds, hipStream_t st) {
  if (mode == 2)
    grover_group_kernel<float, float><<<grid, 64, lds, st>>>(P);
  else if (mode == 1)
    grover_group_kernel<float, double><<<grid, 64, lds, st>>>(P);
  else
    grover_group_kernel<double, double><<<grid, 64, lds, st>>>(P);
  return hipGetLastError();
}

hipError_t group_occupancy(int mode, size_t lds, int* blocks_per_cu) {
  if (mode == 2)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_group_kernel<float, float>, 64, lds);
  if (mode == 1)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_group_kernel<float, double>, 64, lds);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_group_kernel<double, double>, 64, lds);
}

template <int CM>
size_t group_lds_cls(int mode) {
  if (mode == 2) return sizeof(GroupLds<float, float, CM>);
  if (mode == 1) return sizeof(GroupLds<float, double, CM>);
  return sizeof(GroupLds<double, double, CM>);
}

size_t group_lds_bytes(int mode, int cls) {
  switch (cls) {
    case 0: return group_lds_cls<2>(mode);
    case 1: return group_lds_cls<3>(mode);
    case 2: return group_lds_cls<4>(mode);
    case 3: return group_lds_cls<5>(mode);
    case 4: return group_lds_cls<6>(mode);
  }
  return 0;
}

}  // namespace gmps
