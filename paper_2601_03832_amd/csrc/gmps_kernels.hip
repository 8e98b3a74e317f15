// HIP kernels of libgmps: iterative Grover search on matrix product states (gfx950).
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
// QR, SVD and norms are FP64. The storage / contraction type S is double (FP64 path) or
// float (mixed path: complex64 site tensors and contractions).
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
template <class S>
__device__ __forceinline__ cx<S> down(cd a) { return {(S)a.re, (S)a.im}; }
template <class S>
__device__ __forceinline__ cd up(cx<S> a) { return {(double)a.re, (double)a.im}; }
template <class S>
__device__ __forceinline__ cx<S> czero() { return {(S)0, (S)0}; }

// ------------------------------------------------------------------------ group collectives
template <int G>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int m = 1; m < G; m <<= 1) v += __shfl_xor(v, m, G);
  return v;
}
template <int G>
__device__ __forceinline__ cd gsum(cd v) { return {gsum<G>(v.re), gsum<G>(v.im)}; }
template <int G>
__device__ __forceinline__ cd gbcast(cd v, int src) { return {__shfl(v.re, src, G), __shfl(v.im, src, G)}; }

// Round-robin (circle method) pairing of NC columns: round r pairs NC-1 with r and
// (r+p) with (r-p) mod (NC-1); after NC-1 rounds every pair has met once.
__host__ __device__ constexpr int circ_a(int NC, int r, int p) { return p == 0 ? NC - 1 : (r + p) % (NC - 1); }
__host__ __device__ constexpr int circ_b(int NC, int r, int p) {
  return p == 0 ? r : (r - p + (NC - 1)) % (NC - 1);
}
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int cmax(int a, int b) { return a < b ? b : a; }

// ------------------------------------------------------------------------------- QR
// Householder QR of an m x c tile (row gl of the tile in x[], m <= G, c <= NC; rows >= m
// and columns >= c are zero). On exit lanes gl < min(m, c) hold row gl of R in x[] and
// q[] holds row gl of the thin Q (m x min(m, c)).
template <int G, int NC>
__device__ __forceinline__ void householder_qr(cd (&x)[NC], cd (&q)[NC], int gl, int m, int c) {
  const int kr = m < c ? m : c;
  cd hv[NC];
  double tau[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    hv[j] = {0.0, 0.0};
    tau[j] = 0.0;
    if (j < kr) {
      const cd xj = x[j];
      const double sub = gsum<G>((gl > j && gl < m) ? norm2(xj) : 0.0);
      const cd alpha = gbcast<G>(xj, j);
      const double aa = sqrt(norm2(alpha));
      const double nrm = sqrt(aa * aa + sub);
      const bool refl = sub > 0.0;
      const cd ph = aa > 0.0 ? cd{alpha.re / aa, alpha.im / aa} : cd{1.0, 0.0};
      const cd beta = {-ph.re * nrm, -ph.im * nrm};
      const double t = refl ? 1.0 / (nrm * (nrm + aa)) : 0.0;
      cd v = (gl == j) ? alpha - beta : ((gl > j && gl < m) ? xj : cd{0.0, 0.0});
      if (!refl) v = {0.0, 0.0};
      cd w[NC];
#pragma unroll
      for (int k = j + 1; k < NC; ++k)
        if (k < c) w[k] = gsum<G>(cmulc(v, x[k]));
#pragma unroll
      for (int k = j + 1; k < NC; ++k)
        if (k < c) {
          const cd tw = t * w[k];
          x[k] = x[k] - v * tw;
        }
      if (refl) x[j] = (gl == j) ? beta : ((gl > j) ? cd{0.0, 0.0} : xj);
      hv[j] = v;
      tau[j] = t;
    }
  }
  // thin Q = H_0 H_1 ... H_{kr-1} [I; 0], applied right to left
#pragma unroll
  for (int k = 0; k < NC; ++k) q[k] = {(gl == k && k < kr) ? 1.0 : 0.0, 0.0};
#pragma unroll
  for (int j = NC - 1; j >= 0; --j) {
    if (j < kr && tau[j] != 0.0) {
      cd w[NC];
#pragma unroll
      for (int k = j; k < NC; ++k)
        if (k < kr) w[k] = gsum<G>(cmulc(hv[j], q[k]));
#pragma unroll
      for (int k = j; k < NC; ++k)
        if (k < kr) {
          const cd tw = tau[j] * w[k];
          q[k] = q[k] - hv[j] * tw;
        }
    }
  }
}

// ---------------------------------------------------------------------------- Jacobi SVD
// One-sided (Hestenes) Jacobi on the columns of a rows x c tile held row per lane in a[]
// (columns >= c are zero). Accumulates V (c x c, row gl in v[]). On exit the columns of
// a[] are U*Sigma (mutually orthogonal) and tile = (U Sigma) V^dagger. Returns sweeps run.
template <int G, int NC>
__device__ __forceinline__ int jacobi_svd(cd (&a)[NC], cd (&v)[NC], int gl, int c, double tol,
                                          int max_sweeps) {
#pragma unroll
  for (int k = 0; k < NC; ++k) v[k] = {(gl == k && k < c) ? 1.0 : 0.0, 0.0};
  int sweeps = 0;
  while (sweeps < max_sweeps) {
    ++sweeps;
    double off = 0.0;
#pragma unroll
    for (int r = 0; r < NC - 1; ++r) {
      double al[NC / 2], be[NC / 2];
      cd ga[NC / 2];
#pragma unroll
      for (int p = 0; p < NC / 2; ++p) {
        const int i = cmin(circ_a(NC, r, p), circ_b(NC, r, p));
        const int j = cmax(circ_a(NC, r, p), circ_b(NC, r, p));
        if (j < c) {
          al[p] = gsum<G>(norm2(a[i]));
          be[p] = gsum<G>(norm2(a[j]));
          ga[p] = gsum<G>(cmulc(a[i], a[j]));
        }
      }
#pragma unroll
      for (int p = 0; p < NC / 2; ++p) {
        const int i = cmin(circ_a(NC, r, p), circ_b(NC, r, p));
        const int j = cmax(circ_a(NC, r, p), circ_b(NC, r, p));
        if (j < c) {
          const double g = sqrt(norm2(ga[p]));
          const double ab = sqrt(al[p] * be[p]);
          if (g > tol * ab && g > 1e-300) {
            const double zeta = (be[p] - al[p]) / (2.0 * g);
            const double az = fabs(zeta);
            const double t = az > 1e150 ? 0.5 / zeta : copysign(1.0, zeta) / (az + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + t * t);
            const double sn = cs * t;
            const cd e = {ga[p].re / g, ga[p].im / g};
            const cd se = sn * e;          // s e^{i phi}
            const cd sec = conj(se);       // s e^{-i phi}
            const cd ai = a[i], aj = a[j];
            a[i] = cs * ai - sec * aj;
            a[j] = se * ai + cs * aj;
            const cd vi = v[i], vj = v[j];
            v[i] = cs * vi - sec * vj;
            v[j] = se * vi + cs * vj;
            off = fmax(off, g / ab);
          }
        }
      }
    }
    if (!(off > tol)) break;
  }
  return sweeps;
}

// ---------------------------------------------------------------------------- per-group LDS
template <class S, int CM>
struct GroupLds {
  static constexpr int D = 2 * CM;
  cd X[2 * D][D];           // staged QR tile (rows (a, s)) or SVD tile (rows a)
  cd R[D][D];               // R of the previous QR step
  cd Y[D][CM];              // U Sigma of the previous SVD step
  cx<S> A[CM][2][CM];       // compressed site tensor, zero padded
  int32_t bond[kBondStride];
  int32_t rdim[kBondStride];
};

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

constexpr double kJacobiTol = 1e-15;

// ------------------------------------------------------------------------------ one bundle
template <class S, int CM, int G>
__device__ void run_bundle(const IterParams& P, const Bundle& bd, char* lds_base) {
  constexpr int D = 2 * CM;
  constexpr int SLOT = slot_elems(CM);
  constexpr bool kMixed = sizeof(S) == sizeof(float);
  static_assert(G >= 2 * D, "a lane group must hold a QR tile's rows");
  const int lane = threadIdx.x;
  const int grp = lane / G;
  const int gl = lane % G;
  const bool real = grp < bd.count;
  const int me = bd.inst[real ? grp : 0];
  GroupLds<S, CM>& L = reinterpret_cast<GroupLds<S, CM>*>(lds_base)[grp];
  InstDev* I = P.inst + me;
  const int n = I->n;
  const int M = I->M;
  const int cap = I->cap < CM ? I->cap : CM;
  const int64_t k = bd.k;
  cx<S>* arena = reinterpret_cast<cx<S>*>(P.arena) + I->site_off;
  const uint64_t* W = P.marked + I->marked_off;
  const double tol2 = P.trunc_tol * P.trunc_tol;

  for (int l = gl; l < kBondStride; l += G) L.bond[l] = P.bonds[(int64_t)me * kBondStride + l];
  __syncthreads();

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
        double nn = gsum<G>(gl < 2 ? norm2(up(o)) : 0.0);
        if (diff) {
          const double nr = sqrt(nn);
          drift = fmax(drift, fabs(nr - 1.0));
          if (!(nn > 0.0) || !isfinite(nn)) status |= GMPS_ST_NAN;
          o = down<S>((1.0 / nr) * up(o));
        }
        __syncthreads();
        if (real && gl < 2) arena[gl * D] = o;
        __syncthreads();
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
          L.R[0][0] = {1.0, 0.0};
          L.rdim[0] = 1;
        }
        __syncthreads();
        for (int i = 0; i < n; ++i) {
          const int chl = L.bond[i], chr = L.bond[i + 1];
          const bool first = (i == 0), last = (i == n - 1);
          const int xb = diff ? 0 : (int)((xw >> (n - 1 - i)) & 1ull);
          const int Dl = first ? 1 : 2 * chl;
          const int Dr = last ? 1 : 2 * chr;
          cx<S>* slot = arena + (int64_t)i * SLOT;
          for (int e = gl; e < CM * 2 * CM; e += G) {
            const int a = e / (2 * CM), s = (e / CM) & 1, b = e % CM;
            cx<S> val = czero<S>();
            if (a < chl && b < chr) val = slot[a * 2 * D + s * D + b];
            (&L.A[0][0][0])[e] = val;
          }
          __syncthreads();
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
                            acc = cfma(acc, down<S>(L.R[a][beta * chl + ap]), wa);
                          }
                      }
                    }
                    L.X[gl][beta * chr + b] = up(acc);
                  }
                }
              }
              for (int col = Dr; col < D; ++col) L.X[gl][col] = {0.0, 0.0};
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
                      acc = cfma(acc, down<S>(L.R[a][al * chl + ap]), cal * wa);
                    }
                }
              }
              L.X[gl][0] = up(acc);
            }
          }
          const double macs = (double)r * Dl * 2.0 * Dr;
          if (kMixed) f32 += 8.0 * macs; else f64 += 8.0 * macs;
          __syncthreads();
          if (last) {
            if (real && gl < 2 * r) {
              const int a = gl >> 1, s = gl & 1;
              slot[a * 2 * D + s * D] = down<S>(L.X[gl][0]);
            }
            if (gl == 0) {
              L.rdim[n - 1] = r;
              L.rdim[n] = 1;
            }
            __syncthreads();
            break;
          }
          cd xr[D], q[D];
#pragma unroll
          for (int col = 0; col < D; ++col) xr[col] = (gl < 2 * D) ? L.X[gl][col] : cd{0.0, 0.0};
          const int m = 2 * r;
          householder_qr<G, D>(xr, q, gl, m, Dr);
          const int kr = m < Dr ? m : Dr;
          {
            const double mm = m, cc = Dr;
            f64 += mm >= cc ? 8.0 * (2.0 * mm * cc * cc - 2.0 * cc * cc * cc / 3.0)
                            : 8.0 * (2.0 * cc * mm * mm - 2.0 * mm * mm * mm / 3.0);
          }
          if (real && gl < m) {
            const int a = gl >> 1, s = gl & 1;
#pragma unroll
            for (int col = 0; col < D; ++col)
              if (col < kr) slot[a * 2 * D + s * D + col] = down<S>(q[col]);
          }
          if (gl < kr) {
#pragma unroll
            for (int col = 0; col < D; ++col) L.R[gl][col] = col < gl ? cd{0.0, 0.0} : xr[col];
          }
          if (gl == 0) L.rdim[i + 1] = kr;
          r = kr;
          __syncthreads();
        }

        // ---------------------------------------------- truncated-SVD sweep
        if (gl == 0) L.Y[0][0] = {1.0, 0.0};
        __syncthreads();
        for (int i = n - 1; i >= 1; --i) {
          const int ri = L.rdim[i], rn = L.rdim[i + 1];
          const int chn = L.bond[i + 1];
          const int c = 2 * chn;
          cx<S>* slot = arena + (int64_t)i * SLOT;
          if (gl < D) {
            const bool rowok = gl < ri;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
              cx<S> qrow[D];
#pragma unroll
              for (int b = 0; b < D; ++b)
                qrow[b] = (rowok && b < rn) ? slot[gl * 2 * D + s * D + b] : czero<S>();
#pragma unroll
              for (int jj = 0; jj < CM; ++jj)
                if (jj < chn) {
                  cx<S> acc = czero<S>();
#pragma unroll
                  for (int b = 0; b < D; ++b)
                    if (b < rn) acc = cfma(acc, qrow[b], down<S>(L.Y[b][jj]));
                  L.X[gl][s * chn + jj] = up(acc);
                }
            }
            for (int col = c; col < D; ++col) L.X[gl][col] = {0.0, 0.0};
          }
          {
            const double macs = (double)ri * 2.0 * rn * chn;
            if (kMixed) f32 += 8.0 * macs; else f64 += 8.0 * macs;
          }
          __syncthreads();
          cd mrow[D], vrow[D];
#pragma unroll
          for (int col = 0; col < D; ++col) mrow[col] = (gl < D) ? L.X[gl][col] : cd{0.0, 0.0};
          const int sweeps = jacobi_svd<G, D>(mrow, vrow, gl, c, kJacobiTol, P.max_sweeps);
          f64 += (double)sweeps * c * (c - 1) / 2.0 * 56.0 * ri;
          double sg[D];
          double smax = 0.0, stot = 0.0;
#pragma unroll
          for (int col = 0; col < D; ++col) {
            sg[col] = col < c ? gsum<G>(gl < ri ? norm2(mrow[col]) : 0.0) : 0.0;
            smax = fmax(smax, sg[col]);
            stot += sg[col];
          }
          int above = 0;
#pragma unroll
          for (int col = 0; col < D; ++col) above += (col < c && sg[col] > 0.0 && sg[col] >= tol2 * smax) ? 1 : 0;
          int chi_new = above < cap ? above : cap;
          if (chi_new < 1) chi_new = 1;
          double dropped = 0.0;
          int rank[D];
#pragma unroll
          for (int col = 0; col < D; ++col) {
            int rk = 0;
#pragma unroll
            for (int o = 0; o < D; ++o) rk += (sg[o] > sg[col] || (sg[o] == sg[col] && o < col)) ? 1 : 0;
            rank[col] = rk;
            if (rk >= chi_new) dropped += sg[col];
          }
          if (stot > 0.0) truncw = fmax(truncw, dropped / stot);
          if (!isfinite(stot)) status |= GMPS_ST_NAN;
          __syncthreads();
#pragma unroll
          for (int col = 0; col < D; ++col) {
            if (rank[col] < chi_new) {
              const int rk = rank[col];
              if (real && gl < c) {
                const int s = gl >= chn ? 1 : 0;
                const int jp = gl - s * chn;
                slot[rk * 2 * D + s * D + jp] = down<S>(conj(vrow[col]));
              }
              if (gl < ri) L.Y[gl][rk] = mrow[col];
            }
          }
          if (gl == 0) L.bond[i] = chi_new;
          __syncthreads();
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
            for (int b = 0; b < D; ++b)
              if (b < rn) acc = cfma(acc, slot[s * D + b], down<S>(L.Y[b][jj]));
          }
          const double macs = 2.0 * rn * chn;
          if (kMixed) f32 += 8.0 * macs; else f64 += 8.0 * macs;
          const double nn = gsum<G>(act ? norm2(up(acc)) : 0.0);
          if (!isfinite(nn) || !(nn > 0.0)) status |= GMPS_ST_NAN;
          if (diff) {
            const double nr = sqrt(nn);
            drift = fmax(drift, fabs(nr - 1.0));
            acc = down<S>((1.0 / nr) * up(acc));
          }
          __syncthreads();
          if (real && act) slot[s * D + jj] = acc;
          if (gl == 0) L.bond[0] = 1;
          __syncthreads();
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
  __syncthreads();
}

template <class S>
__global__ __launch_bounds__(64) void grover_kernel(IterParams P) {
  extern __shared__ __align__(16) char lds[];
  for (;;) {
    unsigned int bi = 0;
    if (threadIdx.x == 0) bi = atomicAdd(&P.queue->next, 1u);
    bi = __shfl(bi, 0);
    if ((int)bi >= P.queue->nbundles) break;
    const Bundle bd = P.bundles[bi];
    switch (bd.cls) {
      case 0: run_bundle<S, 2, 8>(P, bd, lds); break;
      case 1: run_bundle<S, 3, 16>(P, bd, lds); break;
      case 2: run_bundle<S, 4, 16>(P, bd, lds); break;
      case 3: run_bundle<S, 6, 32>(P, bd, lds); break;
      default: break;
    }
  }
}

__global__ void queue_reset_kernel(QueueState* q) {
  if (threadIdx.x == 0 && blockIdx.x == 0) q->next = 0u;
}

// a2: every instance <- |+>^n with all bonds 1.
template <class S>
__global__ void init_uniform_kernel(InstDev* inst, int B, const int64_t* site_start, int32_t* bonds,
                                    void* arena_v, int64_t total_sites) {
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
  const int CM = kClasses[I.cls].CM;
  const int D = 2 * CM;
  cx<S>* slot = reinterpret_cast<cx<S>*>(arena_v) + I.site_off + (int64_t)i * slot_elems(CM);
  const S h = (S)0.70710678118654752440;
  slot[0] = {h, (S)0};
  slot[D] = {h, (S)0};
  bonds[(int64_t)lo * kBondStride + i] = 1;
  if (i == I.n - 1) bonds[(int64_t)lo * kBondStride + I.n] = 1;
  if (i == 0) {
    I.k_done = 0;
    I.status = 0;
    I.drift = 0.0;
    I.trunc_w = 0.0;
    I.flops64 = 0.0;
    I.flops32 = 0.0;
  }
}

// -------------------------------------------------------------------------- read-out kernels
constexpr int kMaxChi = 8;

template <class S>
__device__ cd amplitude_of(const InstDev& I, const int32_t* bond, const cx<S>* base, uint64_t x) {
  const int CM = kClasses[I.cls].CM;
  const int D = 2 * CM;
  const int n = I.n;
  cd v[kMaxChi];
  v[0] = {1.0, 0.0};
  int chl = 1;
  for (int i = 0; i < n; ++i) {
    const int chr = bond[i + 1];
    const int s = (int)((x >> (n - 1 - i)) & 1ull);
    const cx<S>* slot = base + (int64_t)i * slot_elems(CM);
    cd w[kMaxChi];
    for (int b = 0; b < chr; ++b) {
      cd acc = {0.0, 0.0};
      for (int a = 0; a < chl; ++a) acc = cfma(acc, v[a], up(slot[a * 2 * D + s * D + b]));
      w[b] = acc;
    }
    for (int b = 0; b < chr; ++b) v[b] = w[b];
    chl = chr;
  }
  return v[0];
}

template <class S>
__device__ double norm2_of(const InstDev& I, const int32_t* bond, const cx<S>* base) {
  // <psi|psi> by left transfer matrices E <- sum_s A_s^dagger E A_s
  const int CM = kClasses[I.cls].CM;
  const int D = 2 * CM;
  cd E[kMaxChi][kMaxChi], T[kMaxChi][kMaxChi];
  E[0][0] = {1.0, 0.0};
  int chl = 1;
  for (int i = 0; i < I.n; ++i) {
    const int chr = bond[i + 1];
    const cx<S>* slot = base + (int64_t)i * slot_elems(CM);
    for (int b = 0; b < chr; ++b)
      for (int bb = 0; bb < chr; ++bb) {
        cd acc = {0.0, 0.0};
        for (int s = 0; s < 2; ++s)
          for (int a = 0; a < chl; ++a) {
            cd ea = {0.0, 0.0};
            for (int aa = 0; aa < chl; ++aa) ea = cfma(ea, E[a][aa], up(slot[aa * 2 * D + s * D + bb]));
            acc = acc + cmulc(up(slot[a * 2 * D + s * D + b]), ea);
          }
        T[b][bb] = acc;
      }
    for (int b = 0; b < chr; ++b)
      for (int bb = 0; bb < chr; ++bb) E[b][bb] = T[b][bb];
    chl = chr;
  }
  return E[0][0].re;
}

template <class S>
__global__ void marked_prob_kernel(InstDev* inst, const uint64_t* marked, const int32_t* bonds,
                                   const void* arena_v, int B, double* out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  InstDev& I = inst[b];
  const cx<S>* base = reinterpret_cast<const cx<S>*>(arena_v) + I.site_off;
  const int32_t* bond = bonds + (int64_t)b * kBondStride;
  const double nn = norm2_of<S>(I, bond, base);
  double acc = 0.0;
  for (int j = 0; j < I.M; ++j) acc += norm2(amplitude_of<S>(I, bond, base, marked[I.marked_off + j]));
  const double p = acc / nn;
  if (!isfinite(p)) I.status |= GMPS_ST_NAN;
  out[b] = p;
}

template <class S>
__global__ void amplitude_kernel(const InstDev* inst, int which, const int32_t* bonds, const void* arena_v,
                                 const uint64_t* xs, int64_t cnt, double* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const InstDev& I = inst[which];
  const cx<S>* base = reinterpret_cast<const cx<S>*>(arena_v) + I.site_off;
  const cd a = amplitude_of<S>(I, bonds + (int64_t)which * kBondStride, base, xs[t]);
  out[2 * t] = a.re;
  out[2 * t + 1] = a.im;
}

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

template <class S>
__global__ void sample_kernel(const InstDev* inst, const uint64_t* marked, const int32_t* bonds,
                              const void* arena_v, int B, const int64_t* shot_off, uint64_t seed,
                              uint64_t* bits, unsigned long long* hits) {
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
  const int CM = kClasses[I.cls].CM;
  const int D = 2 * CM;
  const int n = I.n;
  const cx<S>* base = reinterpret_cast<const cx<S>*>(arena_v) + I.site_off;
  const int32_t* bond = bonds + (int64_t)lo * kBondStride;
  cd v[kMaxChi];
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
      philox4x64_10(words, seed, (uint64_t)lo);
    }
    const double u = (double)(words[i & 3] >> 11) * (1.0 / 9007199254740992.0);
    const int chr = bond[i + 1];
    const cx<S>* slot = base + (int64_t)i * slot_elems(CM);
    cd w0[kMaxChi], w1[kMaxChi];
    double q0 = 0.0, q1 = 0.0;
    for (int b = 0; b < chr; ++b) {
      cd a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
      for (int a = 0; a < chl; ++a) {
        a0 = cfma(a0, v[a], up(slot[a * 2 * D + b]));
        a1 = cfma(a1, v[a], up(slot[a * 2 * D + D + b]));
      }
      w0[b] = a0;
      w1[b] = a1;
      q0 += norm2(a0);
      q1 += norm2(a1);
    }
    const double p0 = q0 / (q0 + q1);
    const bool zero = u < p0;
    const double sc = 1.0 / sqrt(zero ? q0 : q1);
    for (int b = 0; b < chr; ++b) v[b] = sc * (zero ? w0[b] : w1[b]);
    if (!zero) x |= 1ull << (n - 1 - i);
    chl = chr;
  }
  bits[t] = x;
  for (int j = 0; j < I.M; ++j)
    if (marked[I.marked_off + j] == x) {
      atomicAdd(hits + lo, 1ull);
      break;
    }
}

// ------------------------------------------------------------------------- launch wrappers
template <class S>
static hipError_t launch_iterate_t(const IterParams& P, int grid, size_t lds, hipStream_t st) {
  queue_reset_kernel<<<1, 64, 0, st>>>(P.queue);
  grover_kernel<S><<<grid, 64, lds, st>>>(P);
  return hipGetLastError();
}

hipError_t launch_iterate(bool mixed, const IterParams& P, int grid, size_t lds, hipStream_t st) {
  return mixed ? launch_iterate_t<float>(P, grid, lds, st) : launch_iterate_t<double>(P, grid, lds, st);
}

hipError_t iterate_occupancy(bool mixed, size_t lds, int* blocks_per_cu) {
  return mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_kernel<float>, 64, lds)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_kernel<double>, 64, lds);
}

size_t group_lds_bytes(bool mixed, int cls) {
  switch (cls) {
    case 0: return mixed ? sizeof(GroupLds<float, 2>) : sizeof(GroupLds<double, 2>);
    case 1: return mixed ? sizeof(GroupLds<float, 3>) : sizeof(GroupLds<double, 3>);
    case 2: return mixed ? sizeof(GroupLds<float, 4>) : sizeof(GroupLds<double, 4>);
    case 3: return mixed ? sizeof(GroupLds<float, 6>) : sizeof(GroupLds<double, 6>);
  }
  return 0;
}

hipError_t launch_init(bool mixed, InstDev* inst, int B, const int64_t* site_start, int32_t* bonds, void* arena,
                       int64_t total_sites, hipStream_t st) {
  const int blk = 256;
  const int grid = (int)((total_sites + blk - 1) / blk);
  if (grid == 0) return hipSuccess;
  if (mixed)
    init_uniform_kernel<float><<<grid, blk, 0, st>>>(inst, B, site_start, bonds, arena, total_sites);
  else
    init_uniform_kernel<double><<<grid, blk, 0, st>>>(inst, B, site_start, bonds, arena, total_sites);
  return hipGetLastError();
}

hipError_t launch_prob(bool mixed, InstDev* inst, const uint64_t* marked, const int32_t* bonds, const void* arena,
                       int B, double* out, hipStream_t st) {
  const int blk = 64;
  const int grid = (B + blk - 1) / blk;
  if (mixed)
    marked_prob_kernel<float><<<grid, blk, 0, st>>>(inst, marked, bonds, arena, B, out);
  else
    marked_prob_kernel<double><<<grid, blk, 0, st>>>(inst, marked, bonds, arena, B, out);
  return hipGetLastError();
}

hipError_t launch_amplitudes(bool mixed, const InstDev* inst, int which, const int32_t* bonds, const void* arena,
                             const uint64_t* xs, int64_t cnt, double* out, hipStream_t st) {
  const int blk = 64;
  const int grid = (int)((cnt + blk - 1) / blk);
  if (grid == 0) return hipSuccess;
  if (mixed)
    amplitude_kernel<float><<<grid, blk, 0, st>>>(inst, which, bonds, arena, xs, cnt, out);
  else
    amplitude_kernel<double><<<grid, blk, 0, st>>>(inst, which, bonds, arena, xs, cnt, out);
  return hipGetLastError();
}

hipError_t launch_sample(bool mixed, const InstDev* inst, const uint64_t* marked, const int32_t* bonds,
                         const void* arena, int B, const int64_t* shot_off, int64_t total, uint64_t seed,
                         uint64_t* bits, unsigned long long* hits, hipStream_t st) {
  const int blk = 64;
  const int grid = (int)((total + blk - 1) / blk);
  if (grid == 0) return hipSuccess;
  if (mixed)
    sample_kernel<float><<<grid, blk, 0, st>>>(inst, marked, bonds, arena, B, shot_off, seed, bits, hits);
  else
    sample_kernel<double><<<grid, blk, 0, st>>>(inst, marked, bonds, arena, B, shot_off, seed, bits, hits);
  return hipGetLastError();
}

}  // namespace gmps
