// Pipelined reflections for the team classes whose teams fit one wave (bond caps 2, 3, 5
// and 8), in the per-projector MPO form (Section III-B) and in the pre-contracted form.
//
// Each reflection is a canonicalisation sweep (MPO applied, rank-stopped QR) followed by a
// truncation sweep (one-sided Jacobi SVD) in the opposite direction. Reflections alternate
// directions: reflection j canonicalises left to right when j is even and right to left when
// j is odd, so the truncation sweep of reflection j and the canonicalisation sweep of
// reflection j+1 run in the same direction, and the second can follow the first one site
// behind. A workgroup holds a bundle of 64/TW instances with equal (n, M, k) on two waves:
// team t of wave 0 runs instance t's truncation sweeps, team t of wave 1 its canonicalisation
// sweeps, in lock step ticks of one site. Every final site tensor
// the truncation wave produces is handed to the canonicalisation wave through LDS. Both waves
// take exactly one workgroup barrier per tick and none inside a step.
//
// Mirrored steps: right-to-left canonicalisation takes the LQ factorisation of the MPO-applied
// tile as the QR of its conjugate transpose, the site keeps Q^H (right-orthonormal) and the
// carry is R^H; left-to-right truncation runs the Jacobi on the columns of M (the bond being
// truncated), keeps U = M J / Sigma and carries Sigma J^H to the right. After a call the chain
// is right-canonical with the norm in site 0, as the read-out kernels expect: a call whose last
// truncation ran left to right ends with one right-to-left canonicalisation of the identity.
//
// Storage precision (S = float: GMPS_MIXED). All arithmetic is FP64. The bulk sites are stored
// as complex64 and each rounding is compensated: a stored isometry Q~ = Q + d changes the state
// by d times the rest of the chain, and the part of d inside the span of Q's columns (rows, for
// a right-orthonormal site) is undone to first order by the carry that moves on,
// R' = R - (Q^H d) R (for kept rows v_q of a truncation, Y' = Y - Y Z with Z[p][q] = <v_q | d_p>).
// The part outside that span is orthogonal to every state whose support at this bond lies in
// it, as the Grover states' supports do away from the chain's ends: it cannot rotate the state
// within their span, and it reaches the marked probability only at second order. The edge
// sites (within ceil(log2(M+1)) of either end, where a bond of 2^i cannot hold that support,
// and the norm-carrying end site) stay in complex FP64 in edge slots, and the hand-over between
// the waves is FP64 too. With plain rounding every stored tile moves the rotation angle by
// O(2^-24), and the moves add up over the k (M+1) 2n stores of a run.
#pragma once
#include "gmps_team.h"

namespace gmps {

template <class S, int CM>
struct PipeLds {
  using T = TeamShape<CM, 64>;
  cd W[2][CM][2][CM];            // canonicalisation: staged MPO blocks [c0 A | c1 P A]
  cd R[T::KQ][T::D];             // canonicalisation carry: R (to the right) or R~ = L^H (left)
  cd V[T::KQ][T::PQ * T::RQ];    // Householder vectors, then the columns of Q
  double tau[T::KQ];
  cd ZQ[T::KQ][T::KQ];           // canonicalisation: Q^H d of the stored Q~ = Q + d
  cd Q[T::KQ][2][T::KQ];         // truncation: staged site of the canonicalised chain
  cd Y[T::KQ][CM];               // truncation carry, [canonical bond][kept bond]
  cd WB[CM][2 * CM];             // truncation: the kept vectors, by position
  cd ZT[CM][CM];                 // truncation: Z[p][q] = <v_q | d_p>
  cd H[2][CM][2][CM];            // final site tensors handed over (as stored), by tick parity
  int32_t bond[kBondStride];     // bonds of the chain the truncation wave produces
  int32_t rdim[2][kBondStride];  // bonds of the canonicalised chain, by reflection parity
};

// Pre-contracted reflections on the pipelined kernel (instantiated for FP64 storage: on
// complex64 storage the rotation angle drifts, faster with n). Reflection j maps psi to
// c0 psi + c1 sum_t <p_t|psi> p_t, an MPS of bond chi + T whose sites are diag(A_i, e_t(i)),
// e_t(i) the one-site factor of the product state p_t (a marked bit, or |+>). The
// canonicalisation wave runs one site behind the truncation wave that produces psi, so the
// overlaps are complete only at its last site. The term columns therefore enter the sweep
// with predicted weights c1 <p_t|psi>: the reflections are exact, so the overlaps of the next
// reflection's terms follow from this one's, <q|psi'> = c0 <q|psi> + c1 sum_t <p_t|psi> <q|p_t>
// (<w|w'> = [w = w'], <+|w> = 2^(-n/2)). The wave contracts the overlaps of psi with both
// reflections' terms as it stages each site, and at the last site rescales each term column
// from its predicted to its measured coefficient, which takes in the truncation and rounding
// of the previous step. Columns with physical weights keep the rank-stopped QR from measuring
// them against the rounding noise of psi's small Schmidt directions. The first reflection of a
// call takes its overlaps from a pass over the input chain.
template <int CM>
struct PipeOv {
  cd OV[2][CM + 1][CM];  // overlap rows: a row vector (left to right) or column, by step parity
  cd om[2][CM + 1];      // first-site weights of the term columns, by reflection parity
};

template <class S, int CM, int TW, bool PC = false>
__device__ void run_pipe(const IterParams& P, const Bundle* bdp, char* lds_base) {
  using T = TeamShape<CM, TW>;
  constexpr int TEAMS = 64 / TW;
  constexpr int D = T::D, KQ = T::KQ;
  constexpr int PQ = T::PQ, RQ = T::RQ, PJ = T::PJ, RJ = T::RJ, RU = T::RU;
  constexpr int SLOT = slot_elems(CM);
  constexpr int NE = (CM * CM + TW - 1) / TW;  // (CM x CM) box elements per lane
  constexpr bool kMixed = sizeof(S) == sizeof(float);
  const int wave = threadIdx.x / 64;  // 0: truncation, 1: canonicalisation
  const int lane = threadIdx.x % 64;
  const int team = lane / TW;
  const int tl = lane % TW;             // lane within the team
  const int base = lane - tl;           // the team's first lane in its wave
  const int qc = tl / PQ, qh = tl % PQ;  // QR layout
  const int jc = tl / PJ, jh = tl % PJ;  // Jacobi layout
  const bool real = team < bdp->count;
  // inst[] is indexed per lane: read it from memory, not from a register copy
  const int me = bdp->inst[real ? team : 0];
  PipeLds<S, CM>& L = reinterpret_cast<PipeLds<S, CM>*>(lds_base)[team];
  PipeOv<CM>& X = reinterpret_cast<PipeOv<CM>*>(lds_base + (64 / TW) * sizeof(PipeLds<S, CM>))[team];
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
  const uint64_t* Wm = P.marked + I->marked_off;
  const bool sr = P.stoch_round != 0;
  uint64_t rs_state = mix64(((uint64_t)me << 32) ^ ((uint64_t)I->k_done * 0x9E3779B97F4A7C15ull) ^ (uint64_t)threadIdx.x);
  const double tol2 = P.trunc_tol * P.trunc_tol;
  const double rank2 = P.rank_tol * P.rank_tol;
  const double skip2 = P.skip_tol * P.skip_tol;

  for (int l = wave * TW + tl; l < kBondStride; l += 2 * TW) L.bond[l] = P.bonds[(int64_t)me * kBondStride + l];
  team_sync_global();

  double f64 = 0.0, f32 = 0.0, drift = 0.0, truncw = 0.0;
  int status = 0;
  // pre-contracted: the M oracle terms in one reflection when the host says so (lossless cap,
  // M within the class), else one reflection per marked index; the diffusion comes last
  const bool whole = PC && I->whole != 0;
  const int nrefl = whole ? 2 : M + 1;
  const int64_t J = k * nrefl;  // reflections of this call
  int opar = 0;                 // pre-contracted: parity of the current term weights

  // ---------------------------------------------------------------- pre-contracted terms
  // Overlap rows u of reflection jr: with the whole oracle in one reflection the M marked
  // states and |+> (row M); else row 0 is this reflection's term, row 1 the next one's. A
  // row's kind is its marked index, or -1 for |+>.
  auto ov_rows = [&](bool ident) -> int { return ident ? 0 : (whole ? M + 1 : 2); };
  auto row_kind = [&](int jr, int u) -> int {
    if (whole) return u < M ? u : -1;
    const int j = u == 0 ? jr : (jr + 1) % nrefl;
    return j == nrefl - 1 ? -1 : j;
  };
  auto this_row = [&](int jr, int t) -> int { return whole ? (jr == nrefl - 1 ? M : t) : 0; };
  auto next_row = [&](int jr, int t) -> int { return whole ? (jr == nrefl - 1 ? t : M) : 1; };
  auto terms_of = [&](int jr) -> int { return (whole && jr != nrefl - 1) ? M : 1; };
  auto efac = [&](int kind, int i, int s) -> double {
    if (kind < 0) return kInvSqrt2;
    return (int)((Wm[kind] >> (n - 1 - i)) & 1ull) == s ? 1.0 : 0.0;
  };
  auto gram = [&](int ka, int kb) -> double {
    if (ka < 0 && kb < 0) return 1.0;
    if (ka < 0 || kb < 0) return exp2(-0.5 * n);
    return Wm[ka] == Wm[kb] ? 1.0 : 0.0;
  };
  // stage site i as A itself into W[0] and advance the overlap rows through it
  auto stage_ov = [&](int jr, bool ident, bool lr, int i, const cd (*h)[2][CM]) {
    const int chl = L.bond[i], chr = L.bond[i + 1];
    const bool first = lr ? (i == 0) : (i == n - 1);
    const cx<S>* slot = arena + (int64_t)i * SLOT;
    const cd* es = eslot(i);
    const int U = ov_rows(ident);
    if (first && tl < U) X.OV[0][tl][0] = {1.0, 0.0};
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tl + t * TW;
      if (e < CM * CM) {
        const int a = e / CM, b = e % CM;
        cd a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
        if (a < chl && b < chr) {
          if (h) {
            a0 = h[a][0][b];
            a1 = h[a][1][b];
          } else if (es) {
            a0 = es[a * 2 * D + b];
            a1 = es[a * 2 * D + D + b];
          } else {
            a0 = up(slot[a * 2 * D + b]);
            a1 = up(slot[a * 2 * D + D + b]);
          }
        }
        L.W[0][a][0][b] = a0;
        L.W[0][a][1][b] = a1;
      }
    }
    wave_sync();
    if (U > 0) {
      // <p_u| A_0 .. A_i: left to right a row over the right bond of site i, right to left a
      // column over its left bond
      const int step = lr ? i : n - 1 - i;
      const cd(*vin)[CM] = X.OV[step & 1];
      cd(*vout)[CM] = X.OV[(step + 1) & 1];
      const int nin = lr ? chl : chr, nout = lr ? chr : chl;
      for (int el = tl; el < U * CM; el += TW) {
        const int u = el / CM, o = el % CM;
        if (o < nout) {
          const int kind = row_kind(jr, u);
          const double e0 = efac(kind, i, 0), e1 = efac(kind, i, 1);
          cd acc = {0.0, 0.0};
          for (int v = 0; v < CM; ++v)
            if (v < nin) {
              const cd w0 = lr ? L.W[0][v][0][o] : L.W[0][o][0][v];
              const cd w1 = lr ? L.W[0][v][1][o] : L.W[0][o][1][v];
              acc = cfma(acc, vin[u][v], cd{e0 * w0.re + e1 * w1.re, e0 * w0.im + e1 * w1.im});
            }
          vout[u][o] = acc;
        }
      }
      f64 += 8.0 * (double)U * nin * nout;
      wave_sync();
    }
  };

  // ---------------------------------------------------------------- canonicalisation step
  // Reflection jr (0..nrefl-1, the last one the diffusion) at site i, direction lr; the site
  // tensor comes from the handover buffer h (null: from its arena slot). rdo: the ranks it
  // produces.
  auto canon_step = [&](int jr, bool ident, bool lr, int i, const cd (*h)[2][CM], int32_t* rdo) {
    const bool diff = (jr == nrefl - 1);
    const int xb = (diff || ident) ? 0 : (int)((Wm[jr] >> (n - 1 - i)) & 1ull);
    const double c0 = ident ? 1.0 : (diff ? -1.0 : 1.0);
    const double c1 = ident ? 0.0 : (diff ? 2.0 : -2.0);
    const int chl = L.bond[i], chr = L.bond[i + 1];
    const bool mpo_last = (i == n - 1);  // the MPO's coefficients sit on the last site
    const bool first = lr ? (i == 0) : (i == n - 1);
    const bool last = lr ? (i == n - 1) : (i == 0);
    cx<S>* slot = arena + (int64_t)i * SLOT;
    cd* es = eslot(i);
    const int T = (!PC || ident) ? 0 : terms_of(jr);  // pre-contracted: product terms
    const int step = lr ? i : n - 1 - i;               // position in the sweep
    if (first && tl == 0) {
      rdo[lr ? 0 : n] = 1;
      L.R[0][0] = {1.0, 0.0};
      if constexpr (PC) {
        // the term blocks enter with their predicted weights (R~ = L^H right to left)
        for (int t = 0; t < T; ++t) L.R[0][1 + t] = lr ? X.om[opar][t] : conj(X.om[opar][t]);
      } else {
        L.R[0][1] = {1.0, 0.0};
      }
    }
    if constexpr (PC) {
      stage_ov(jr, ident, lr, i, h);
    } else {
      // stage [c0 A | c1 P A] (coefficients on the last site only): the site as the truncation
      // wave handed it over, else from its edge slot (complex FP64) or its site slot
      const double s0 = mpo_last ? c0 : 1.0, s1 = mpo_last ? c1 : 1.0;
#pragma unroll
      for (int t = 0; t < NE; ++t) {
        const int e = tl + t * TW;
        if (e < CM * CM) {
          const int a = e / CM, b = e % CM;
          const bool ok = a < chl && b < chr;
          cd a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
          if (ok) {
            if (h) {
              a0 = h[a][0][b];
              a1 = h[a][1][b];
            } else if (es) {
              a0 = es[a * 2 * D + b];
              a1 = es[a * 2 * D + D + b];
            } else {
              a0 = up(slot[a * 2 * D + b]);
              a1 = up(slot[a * 2 * D + D + b]);
            }
          }
          L.W[0][a][0][b] = s0 * a0;
          L.W[0][a][1][b] = s0 * a1;
          L.W[1][a][0][b] = s1 * proj_apply<double>(a0, a1, 0, diff, xb);
          L.W[1][a][1][b] = s1 * proj_apply<double>(a0, a1, 1, diff, xb);
        }
      }
      wave_sync();
    }
    const int r = first ? 1 : rdo[lr ? i : i + 1];
    cd x[RQ];
    int Dr;  // columns of the QR tile
    if constexpr (PC) {
      // the tile of the site diag(A_i, e_1(i), .., e_T(i)) after the carry: left to right
      // X[(a, s)][b] = sum R[a][a'] A[a'][s][b] and X[(a, s)][chr + t] = R[a][chl + t] e_t[s];
      // right to left the conjugate-transposed tile of the mirrored product (as in the MPO form
      // below). At the sweep's last site the columns sum into one: c0 on the A block, and on
      // term t the measured coefficient c1 <p_t|psi> over the predicted weight it carries.
      const int nA = lr ? chr : chl;  // A-block columns
      const int nS = lr ? chl : chr;  // bond summed over
      Dr = last ? 1 : nA + T;
#pragma unroll
      for (int e = 0; e < RQ; ++e) {
        const int row = qh + PQ * e;
        const int a = row >> 1, s = row & 1;
        cd acc = {0.0, 0.0};
        if (row < 2 * r && qc < Dr) {
          if (last || qc < nA) {
            const int col = last ? 0 : qc;
#pragma unroll
            for (int u = 0; u < CM; ++u)
              if (u < nS) acc = lr ? cfma(acc, L.R[a][u], L.W[0][u][s][col]) : cfma(acc, conj(L.W[0][col][s][u]), L.R[a][u]);
            if (last) {
              acc = c0 * acc;
              for (int t = 0; t < T; ++t) {
                const cd g = cdiv(c1 * X.OV[(step + 1) & 1][this_row(jr, t)][0], X.om[opar][t]);
                const double ev = efac(row_kind(jr, this_row(jr, t)), i, s);
                const cd cw = {ev * g.re, ev * g.im};
                acc = lr ? cfma(acc, L.R[a][nS + t], cw) : cfma(acc, conj(cw), L.R[a][nS + t]);
              }
            }
          } else {
            const int t = qc - nA;
            acc = efac(row_kind(jr, this_row(jr, t)), i, s) * L.R[a][nS + t];
          }
        }
        x[e] = (!lr && last) ? conj(acc) : acc;
      }
    } else if (lr) {
      // X = R_{i-1} * MPO(A_i): rows (a, s) = 2a + s, columns (beta, b)
      Dr = last ? 1 : 2 * chr;
      const int beta = (!last && qc >= chr) ? 1 : 0;
      const int bcol = qc - beta * chr;
#pragma unroll
      for (int e = 0; e < RQ; ++e) {
        const int row = qh + PQ * e;
        const int a = row >> 1, s = row & 1;
        cd acc = {0.0, 0.0};
        if (row < 2 * r && qc < Dr) {
#pragma unroll
          for (int bl = 0; bl < 2; ++bl) {
            if (last || bl == beta) {
#pragma unroll
              for (int ap = 0; ap < CM; ++ap)
                if (ap < chl) acc = cfma(acc, L.R[a][bl * chl + ap], L.W[bl][ap][s][bcol]);
            }
          }
        }
        x[e] = acc;
      }
    } else {
      // X'^H, X' = MPO(A_i) * L_{i+1} with L = R~^H: rows (c, s) = 2c + s, columns
      // (alpha, a); X'^H[(c,s)][(alpha,a)] = sum_b conj(W_alpha[a][s][b]) R~[c][alpha chr + b]
      Dr = last ? 1 : 2 * chl;
      const int alpha = (!last && qc >= chl) ? 1 : 0;
      const int acol = qc - alpha * chl;
#pragma unroll
      for (int e = 0; e < RQ; ++e) {
        const int row = qh + PQ * e;
        const int c = row >> 1, s = row & 1;
        cd acc = {0.0, 0.0};
        if (row < 2 * r && qc < Dr) {
#pragma unroll
          for (int al = 0; al < 2; ++al) {
            if (last || al == alpha) {
#pragma unroll
              for (int bp = 0; bp < CM; ++bp)
                if (bp < chr) acc = cfma(acc, conj(L.W[al][last ? 0 : acol][s][bp]), L.R[c][al * chr + bp]);
            }
          }
        }
        // the left boundary keeps X' itself (one row): conjugate back
        x[e] = last ? conj(acc) : acc;
      }
    }
    if constexpr (PC)
      f64 += 8.0 * (double)r * (first ? 1 : (lr ? chl : chr)) * 2.0 * (last ? 1 : (lr ? chr : chl));
    else
      f64 += 8.0 * (double)r * (first ? 1 : 2 * (lr ? chl : chr)) * 2.0 * Dr;
    if (last) {
      // the boundary site holds the norm: its tile goes to its edge slot and, as stored, to its
      // site slot (left to right the column (a, s) of site n-1, right to left the row (s, c) of
      // site 0)
      if (real && qc == 0) {
#pragma unroll
        for (int e = 0; e < RQ; ++e) {
          const int row = qh + PQ * e;
          if (row < 2 * r) {
            const int off = (lr ? (row >> 1) * 2 * D : 0) + (row & 1) * D + (lr ? 0 : (row >> 1));
            slot[off] = store_cast<S>(x[e], rs_state, sr);
            es[off] = x[e];
          }
        }
      }
      // the rank next to the boundary (r) was read from rdo above and stays; only the
      // boundary's own entry is written (a rewrite of r would race with that read)
      if (tl == 0) rdo[lr ? n : 0] = 1;
      wave_sync();
      if constexpr (PC) {
        if (!ident) {
          // predicted weights of the next reflection's terms
          const int jn = (jr + 1) % nrefl;
          const double c1n = jn == nrefl - 1 ? 2.0 : -2.0;
          const cd(*fin)[CM] = X.OV[(step + 1) & 1];
          if (tl < terms_of(jn)) {
            const int qr = next_row(jr, tl), qk = row_kind(jr, qr);
            cd pr = c0 * fin[qr][0];
            for (int t = 0; t < T; ++t) {
              const int pt = this_row(jr, t);
              pr = pr + (c1 * gram(qk, row_kind(jr, pt))) * fin[pt][0];
            }
            cd w = c1n * pr;
            // a vanishing prediction: a tiny finite weight (the column then carries nothing)
            if (fabs(w.re) + fabs(w.im) < 1e-150) w = {1e-150, 0.0};
            X.om[opar ^ 1][tl] = w;
          }
          opar ^= 1;
          wave_sync();
        }
      }
      return;
    }
    const int m = 2 * r;
    cd q[RQ];
    double qdrop = 0.0;
    const int npiv = lr ? chr : chl;
    const int kr = team_qr_wave<TW, PQ, RQ, KQ, true>(x, q, base, qc, qh, m, Dr, npiv, rank2, &qdrop, L.V, L.tau);
    truncw = fmax(truncw, qdrop);
    {
      const double mm = m, cc = Dr, kk = kr;
      f64 += 8.0 * (2.0 * mm * cc * kk - (mm + cc) * kk * kk + 2.0 * kk * kk * kk / 3.0) +
             8.0 * (2.0 * mm * kk * kk - 2.0 * kk * kk * kk / 3.0);
    }
    // the stored Q~ (stochastic rounding on the mixed path unless round_mode asks for nearest)
    cx<S> qs[RQ];
#pragma unroll
    for (int e = 0; e < RQ; ++e) qs[e] = store_cast<S>(q[e], rs_state, sr);
    if (real && qc < kr) {
#pragma unroll
      for (int e = 0; e < RQ; ++e) {
        const int row = qh + PQ * e;
        if (row < m) {
          // right to left site i keeps Q^H: [k][s][c] = conj(Q[(c, s)][k])
          const int off = lr ? (row >> 1) * 2 * D + (row & 1) * D + qc : qc * 2 * D + (row & 1) * D + (row >> 1);
          slot[off] = lr ? qs[e] : conj(qs[e]);
          if (es) es[off] = lr ? q[e] : conj(q[e]);
        }
      }
    }
    if (qc < Dr) {
#pragma unroll
      for (int e = 0; e < RQ; ++e) {
        const int row = qh + PQ * e;
        if (row < kr) L.R[row][qc] = x[e];
      }
    }
    if (kMixed && !es) {
      // compensation of the stored Q~ = Q + d: R <- R - (Q^H d) R. Column b of Z = Q^H d is
      // formed in slot b from the columns of Q (through V, free once Q is formed); row a of
      // the correction then reads Z and R from LDS.
      cd dq[RQ];
#pragma unroll
      for (int e = 0; e < RQ; ++e) dq[e] = up(qs[e]) - q[e];
      wave_sync();
      if (qc < kr) {
#pragma unroll
        for (int e = 0; e < RQ; ++e) L.V[qc][qh + PQ * e] = q[e];
      }
      wave_sync();
      for (int a = 0; a < kr; ++a) {
        cd z = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < RQ; ++e) z = z + cmulc(L.V[a][qh + PQ * e], dq[e]);
        z = gsum<PQ>(z);
        if (qh == 0 && qc < kr) L.ZQ[a][qc] = z;
      }
      wave_sync();
      cd corr[RQ];
#pragma unroll
      for (int e = 0; e < RQ; ++e) {
        const int row = qh + PQ * e;
        cd cz = {0.0, 0.0};
        if (qc < Dr && row < kr)
          for (int b = 0; b < kr; ++b) cz = cfma(cz, L.ZQ[row][b], L.R[b][qc]);
        corr[e] = cz;
      }
      wave_sync();
      if (qc < Dr) {
#pragma unroll
        for (int e = 0; e < RQ; ++e) {
          const int row = qh + PQ * e;
          if (row < kr) L.R[row][qc] = x[e] - corr[e];
        }
      }
      f64 += 8.0 * ((double)kr * kr * m + (double)kr * kr * Dr);
    }
    if (tl == 0) rdo[lr ? i + 1 : i] = kr;
    wave_sync();
  };

  // the truncation wave loads the next canonicalised site one tick ahead: that slot is final
  // for the whole stage (the canonicalisation wave rewrites it two ticks later)
  TeamQPre<S, KQ, CM, TW> qpre;

  // ---------------------------------------------------------------- truncation step
  // Reflection jr at site i, direction lr (the opposite of its canonicalisation); rdi: the
  // canonicalised chain's bonds. Writes the final site i to h and, when no canonicalisation
  // follows in the stage (keep_slot), to its slot; a following canonicalisation rewrites the
  // slot from h.
  auto trunc_step = [&](int jr, bool lr, int i, const int32_t* rdi, cd (*h)[2][CM], bool keep_slot) {
    const bool wr = real && keep_slot;
    const bool diff = (jr == nrefl - 1);
    const bool first = lr ? (i == 0) : (i == n - 1);
    const bool edge = lr ? (i == n - 1) : (i == 0);  // absorbs the carry, holds the norm
    cx<S>* slot = arena + (int64_t)i * SLOT;
    cd* es = eslot(i);
    const int ri = rdi[i], rn = rdi[i + 1];
    if (first && tl == 0) L.Y[0][0] = {1.0, 0.0};
    // stage the canonicalised site (ri, 2, rn), then load the next one: an edge site (the first
    // one holds the norm) from its edge slot, a bulk site from the prefetch of its site slot
    if (es) {
      for (int e = tl; e < KQ * 2 * KQ; e += TW) {
        const int a = e / (2 * KQ), s = (e / KQ) & 1, b = e % KQ;
        (&L.Q[0][0][0])[e] = (a < ri && b < rn) ? es[a * 2 * D + s * D + b] : cd{0.0, 0.0};
      }
    } else {
      qpre.stage(&L.Q[0][0][0], tl);
    }
    if (!edge) {
      const int nx = lr ? i + 1 : i - 1;
      if (!eslot(nx)) qpre.load(arena + (int64_t)nx * SLOT, tl, rdi[nx], rdi[nx + 1]);
    }
    wave_sync();
    if (edge) {
      // right to left: site 0 = Q_0 Y, (1, 2, chn); left to right: site n-1 = Y^T Q, (chp, 2, 1)
      const int chc = lr ? L.bond[i] : L.bond[1];  // kept bond of the carry
      const int cr = lr ? ri : rn;                 // canonical bond of the carry
      const bool act = tl < 2 * chc;
      const int s = tl >= chc ? 1 : 0;
      const int jj = tl - s * chc;
      cd acc = {0.0, 0.0};
      if (act) {
#pragma unroll
        for (int b = 0; b < KQ; ++b)
          if (b < cr) acc = lr ? cfma(acc, L.Y[b][jj], L.Q[b][s][0]) : cfma(acc, L.Q[0][s][b], L.Y[b][jj]);
      }
      f64 += 8.0 * 2.0 * cr * chc;
      const double nn = tsum<TW>(act ? norm2(acc) : 0.0);
      if (!isfinite(nn) || !(nn > 0.0)) status |= GMPS_ST_NAN;
      const double nr = sqrt(nn);
      if (diff) drift = fmax(drift, fabs(nr - 1.0));
      // the new norm-carrying end site: in FP64 to the canonicalisation wave and, when no
      // canonicalisation follows in this stage, to its edge slot (and as stored to its site slot)
      const cd out = (diff ? 1.0 / nr : 1.0) * acc;
      if (act) {
        const int off = lr ? (jj * 2 * D + s * D) : (s * D + jj);
        if (lr) h[jj][s][0] = out; else h[0][s][jj] = out;
        if (wr) {
          slot[off] = store_cast<S>(out, rs_state, sr);
          es[off] = out;
        }
      }
      if (tl == 0) L.bond[lr ? n : 0] = 1;
      wave_sync();
      return;
    }
    // tile: right to left, the columns of M^H, M = Q_i (U Sigma)_{i+1}, rows (s, jj) of the
    // kept bond chn to the right; left to right, the columns of M = (Sigma J^H)_{i-1} Q_i,
    // rows (s, jj) of the kept bond to the left
    const int chn = lr ? L.bond[i] : L.bond[i + 1];
    const int c = 2 * chn;
    const int ncol = lr ? rn : ri;
    const int ncj = (ncol + 1) & ~1;
    const int cr = lr ? ri : rn;  // canonical bond summed over
    cd a[RJ];
#pragma unroll
    for (int e = 0; e < RJ; ++e) {
      const int row = jh + PJ * e;
      const int s = row >= chn ? 1 : 0;
      const int jj = row - s * chn;
      cd acc = {0.0, 0.0};
      if (jc < ncol && row < c) {
#pragma unroll
        for (int b = 0; b < KQ; ++b)
          if (b < cr) acc = lr ? cfma(acc, L.Y[b][jj], L.Q[b][s][jc]) : cfma(acc, L.Q[jc][s][b], L.Y[b][jj]);
      }
      a[e] = lr ? acc : conj(acc);
    }
    f64 += 8.0 * (double)ncol * 2.0 * cr * chn;
    wave_sync();  // every read of Y is done before it is rewritten below
    cd uu[RU];
#pragma unroll
    for (int e = 0; e < RU; ++e) uu[e] = {(jh + PJ * e == jc && jc < ncj) ? 1.0 : 0.0, 0.0};
    // the mixed path stores every site in complex64 (relative 6e-8): a sweep whose rotations all
    // had cosines below 1e-4 of the column norms leaves, once applied, off-diagonals of order
    // 1e-8 (the cyclic sweep converges quadratically) and ends the Jacobi
    const int sweeps = team_jacobi_wave<TW, PJ, RJ, RU>(a, uu, base, jc, jh, ncj, kJacobiTol2, skip2, P.max_sweeps,
                                                         kMixed ? 1e-8 : 1e-20);
    f64 += (double)sweeps * ncol * (ncol - 1) / 2.0 * 56.0 * c;
    const bool colok = jc < ncj;
    double sg = 0.0;
#pragma unroll
    for (int e = 0; e < RJ; ++e) sg += norm2(a[e]);
    sg = gsum<PJ>(sg);
    const double mine = colok ? sg : 0.0;
    const double smax = tmax<TW>(mine);
    const double stot = tsum<TW>(jh == 0 ? mine : 0.0);
    const int above = (int)tsum<TW>((jh == 0 && mine > 0.0 && mine >= tol2 * smax) ? 1.0 : 0.0);
    int rk = 0;
    for (int o = 0; o < ncj; ++o) {
      const double v = shfl_f64(mine, base + o * PJ);
      rk += (v > sg || (v == sg && o < jc)) ? 1 : 0;
    }
    int chi_new = above < cap ? above : cap;
    if (chi_new < 1) chi_new = 1;
    const bool keep = colok && rk < chi_new;
    const uint64_t kept = tballot<TW>(jh == 0 && keep, base);
    const int pos = __popcll(kept & ((1ull << (base + jc * PJ)) - 1ull));
    const double dropped = tsum<TW>((jh == 0 && colok && !keep) ? sg : 0.0);
    if (stot > 0.0) truncw = fmax(truncw, dropped / stot);
    if (!isfinite(stot)) status |= GMPS_ST_NAN;
    const double rs = keep ? rsqrt_acc(sg) : 0.0;  // 1/sigma
    cd wv[RJ];  // this slot's kept vector: right to left a row of V^H, left to right a column of U
    cx<S> vs[RJ];  // ... as stored
#pragma unroll
    for (int e = 0; e < RJ; ++e) {
      wv[e] = lr ? rs * a[e] : rs * conj(a[e]);
      vs[e] = store_cast<S>(wv[e], rs_state, sr);
    }
    if (keep) {
#pragma unroll
      for (int e = 0; e < RJ; ++e) {
        const int row = jh + PJ * e;
        if (row < c) {
          const int s = row >= chn ? 1 : 0;
          const int jp = row - s * chn;
          // right to left: V^H[pos][s][jp] = conj(a) / sigma; left to right: U[jp][s][pos] = a / sigma;
          // an edge site keeps it in FP64, a bulk site as stored
          const int off = lr ? jp * 2 * D + s * D + pos : pos * 2 * D + s * D + jp;
          const cd hv = es ? wv[e] : up(vs[e]);
          if (wr) {
            slot[off] = vs[e];
            if (es) es[off] = wv[e];
          }
          if (lr) h[jp][s][pos] = hv; else h[pos][s][jp] = hv;
        }
      }
    }
    // right to left: carry J Sigma [row][pos]; left to right: (Sigma J^H)^T [row][pos]
    cd yv[RU];
#pragma unroll
    for (int e = 0; e < RU; ++e) yv[e] = (sg * rs) * (lr ? conj(uu[e]) : uu[e]);
    if (kMixed && !es) {
      // compensation of the stored vectors v~_p = v_p + d_p: Y <- Y - Y Z, Z[p][q] = <v_q | d_p>;
      // the kept vectors go through LDS, row p of Z is formed in the slot of position p
      if (keep) {
#pragma unroll
        for (int e = 0; e < RJ; ++e) {
          const int row = jh + PJ * e;
          if (row < c) L.WB[pos][row] = wv[e];
        }
#pragma unroll
        for (int e = 0; e < RU; ++e) {
          const int row = jh + PJ * e;
          if (row < ncol) L.Y[row][pos] = yv[e];
        }
      }
      wave_sync();
      for (int q = 0; q < chi_new; ++q) {
        cd z = {0.0, 0.0};
#pragma unroll
        for (int e = 0; e < RJ; ++e) {
          const int row = jh + PJ * e;
          if (row < c) z = z + cmulc(L.WB[q][row], up(vs[e]) - wv[e]);
        }
        z = gsum<PJ>(z);
        if (keep && jh == 0) L.ZT[pos][q] = z;
      }
      wave_sync();
#pragma unroll
      for (int e = 0; e < RU; ++e) {
        const int row = jh + PJ * e;
        cd cz = {0.0, 0.0};
        if (keep && row < ncol)
          for (int p = 0; p < chi_new; ++p) cz = cfma(cz, L.Y[row][p], L.ZT[p][pos]);
        yv[e] = yv[e] - cz;
      }
      wave_sync();
      f64 += 8.0 * ((double)chi_new * chi_new * c + (double)chi_new * chi_new * ncol);
    }
    if (keep) {
#pragma unroll
      for (int e = 0; e < RU; ++e) {
        const int row = jh + PJ * e;
        if (row < ncol) L.Y[row][pos] = yv[e];
      }
    }
    if (tl == 0) L.bond[lr ? i + 1 : i] = chi_new;
    wave_sync();
  };

  // ---------------------------------------------------------------- schedule
  // Tick t of a stage: the truncation wave takes its t-th site, the canonicalisation wave
  // its (t-1)-th, so a site reaches the second sweep the tick after the first finished it.
  // Stages: canonicalisation of reflection 0 alone; then truncation j with canonicalisation
  // j+1, j = 0..J-2; then truncation J-1 alone, followed by a right-to-left canonicalisation
  // of the identity if that truncation ran left to right. Both waves take n+1 barriers per
  // stage. Within a stage the waves exchange through LDS only (hand-over buffers, bonds and
  // ranks; the truncation wave leaves the arena to the canonicalisation wave, which rewrites
  // each slot anyway), so the intermediate barriers order LDS only; the last one of a stage
  // also orders the arena, which the next stage reads.
  if constexpr (PC) {
    // the first reflection's weights from its overlaps with the input chain
    if (wave == 1 && J > 0) {
      for (int i = 0; i < n; ++i) stage_ov(0, false, true, i, nullptr);
      const double c1f = nrefl == 1 ? 2.0 : -2.0;
      if (tl < terms_of(0)) {
        cd w = c1f * X.OV[n & 1][this_row(0, tl)][0];
        if (fabs(w.re) + fabs(w.im) < 1e-150) w = {1e-150, 0.0};
        X.om[0][tl] = w;
      }
      wave_sync();
    }
  }
  const int64_t nstage = J == 0 ? 0 : J + 1;
  const bool fix = J > 0 && ((J - 1) & 1) == 1;  // last truncation ran left to right
  for (int64_t stg = 0; stg < nstage + (fix ? 1 : 0); ++stg) {
    const int64_t jt = stg - 1;   // reflection whose truncation runs (-1: none)
    const int64_t jc2 = stg;      // reflection whose canonicalisation runs
    const bool extra = stg == nstage;
    const bool do_t = !extra && jt >= 0;
    const bool do_c = extra || jc2 < J;
    // directions: canonicalisation of reflection j left to right iff j even; its truncation
    // the other way
    const bool lr_c = extra ? false : ((jc2 & 1) == 0);
    const bool lr_t = (jt & 1) == 1;
    for (int tick = 0; tick <= n; ++tick) {
      if (wave == 0) {
        if (do_t && tick < n) {
          const int i = lr_t ? tick : n - 1 - tick;
          trunc_step((int)(jt % nrefl), lr_t, i, L.rdim[jt & 1], L.H[tick & 1], !do_c);
        }
      } else {
        if (do_c && tick >= 1) {
          const int i = lr_c ? tick - 1 : n - tick;
          // follows the truncation wave (handover of the previous tick) when it runs,
          // else reads the arena
          const cd(*h)[2][CM] = do_t ? L.H[(tick - 1) & 1] : nullptr;
          canon_step(extra ? 0 : (int)(jc2 % nrefl), extra, lr_c, i, h, L.rdim[extra ? 0 : (jc2 & 1)]);
        }
      }
      if (tick < n) lds_sync(); else team_sync_global();
    }
    if (extra) {
      // the identity's canonicalisation only re-gauges: its ranks are the bonds
      for (int l = wave * TW + tl; l <= n; l += 2 * TW) L.bond[l] = L.rdim[0][l];
      team_sync_global();
    }
  }

  // ------------------------------------------------------------------ write back
  // the two waves' counters are summed through the status slots of the instance record
  if (real) {
    for (int l = wave * TW + tl; l < kBondStride; l += 2 * TW) P.bonds[(int64_t)me * kBondStride + l] = L.bond[l];
  }
  __shared__ double red[TEAMS][2][4];
  __shared__ int redst[TEAMS][2];
  if (tl == 0) {
    red[team][wave][0] = f64;
    red[team][wave][1] = f32;
    red[team][wave][2] = drift;
    red[team][wave][3] = truncw;
    redst[team][wave] = status;
  }
  team_sync_global();
  if (real && wave == 0 && tl == 0) {
    const double d = fmax(red[team][0][2], red[team][1][2]);
    const double tw = fmax(red[team][0][3], red[team][1][3]);
    int st = redst[team][0] | redst[team][1];
    I->k_done += k;
    I->flops64 += red[team][0][0] + red[team][1][0];
    I->flops32 += red[team][0][1] + red[team][1][1];
    I->drift = fmax(I->drift, d);
    I->trunc_w = fmax(I->trunc_w, tw);
    if (d > 1e-3) st |= GMPS_ST_DRIFT;
    if (tw > 1e-8) st |= GMPS_ST_TRUNC;
    I->status |= st;
  }
  team_sync_global();
}

// Persistent kernel of the pipelined reflections for team class W (a bundle per workgroup of
// two waves).
template <class S, int W, bool PC = false>
__global__ __launch_bounds__(128) void grover_pipe_kernel(IterParams P) {
  extern __shared__ __align__(16) char lds[];
  __shared__ unsigned int next_bundle;
  for (;;) {
    if (threadIdx.x == 0) next_bundle = atomicAdd(&P.queue->next, 1u);
    lds_sync();
    const unsigned int bi = next_bundle;
    lds_sync();
    if ((int)bi >= P.queue->nbundles) break;
    run_pipe<S, kWide[W].CM, kWide[W].TW, PC>(P, P.bundles + bi, lds);
  }
}

template <int W>
hipError_t launch_pipe_w(bool mixed, bool pc, const IterParams& P, int grid, size_t lds, hipStream_t st);
template <int W>
hipError_t occupancy_pipe_w(bool mixed, bool pc, size_t lds, int* blocks_per_cu);

#define GMPS_PIPE_CLASS(W)                                                                           \
  template <>                                                                                        \
  hipError_t launch_pipe_w<W>(bool mixed, bool pc, const IterParams& P, int grid, size_t lds, hipStream_t st) { \
    if (pc && mixed) {                                                                               \
      return hipErrorInvalidValue;                                                                   \
    } else if (pc) {                                                                                 \
      grover_pipe_kernel<double, W, true><<<grid, 128, lds, st>>>(P);                                 \
    } else if (mixed) {                                                                              \
      grover_pipe_kernel<float, W><<<grid, 128, lds, st>>>(P);                                        \
    } else {                                                                                         \
      grover_pipe_kernel<double, W><<<grid, 128, lds, st>>>(P);                                       \
    }                                                                                                \
    return hipGetLastError();                                                                        \
  }                                                                                                  \
  template <>                                                                                        \
  hipError_t occupancy_pipe_w<W>(bool mixed, bool pc, size_t lds, int* blocks_per_cu) {             \
    if (pc)                                                                                          \
      return mixed ? hipErrorInvalidValue                                                            \
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_pipe_kernel<double, W, true>, 128, lds); \
    return mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_pipe_kernel<float, W>, 128, lds) \
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, grover_pipe_kernel<double, W>, 128, lds); \
  }

}  // namespace gmps
