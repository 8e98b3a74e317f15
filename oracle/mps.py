"""FP64 matrix-product-state oracle of the iterative Grover method (Sections II-III).

The state is a chain of site tensors A_i of shape (left bond, 2, right bond)
(Section III-B: memory O(n chi^2)). The iterative method (Section III-A, Fig. 1(C))
feeds the stored MPS back through one Grover gate G = D O per iteration (Eq. (3)).
Each reflection c0*I + c1*(P_0 x P_1 x ... x P_{n-1}) is applied as a bond-2 matrix
product operator:

* oracle, one marked x:   I - 2|x><x|          -> c0 = 1,  c1 = -2, P_i = |x_i><x_i|
* diffusion (Eq. (4)):    2|s><s| - I          -> c0 = -1, c1 = 2,  P_i = |+><+|
  (H^n (2|0><0| - I) H^n with the Hadamard frame folded into the projector).

Per site the operator reads [I, P] (first), diag(I, P) (middle), [c0 I; c1 P] (last),
so every bond doubles. The MPS is then recompressed (Section III-B: local update,
then truncation of small singular values up to chi_max):

1. QR left-canonicalisation sweep, site 0 -> n-2: reshape (left*2, right), Q stays,
   R moves into the next site.
2. Truncated-SVD sweep, site n-1 -> 1: reshape (left, 2*right), keep the singular
   values with sigma_j >= tol * sigma_0, at most chi_cap; V^dagger stays, U*Sigma moves
   into the previous site. The chain ends right-canonical with the norm in site 0.
3. After the diffusion of each iteration, site 0 is divided by the norm.

numpy's LAPACK QR and SVD are the factorisation steps. Bit convention: site i holds
bit (n-1-i) of a basis index.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox

P0 = np.array([[1.0, 0.0], [0.0, 0.0]], dtype=np.complex128)
P1 = np.array([[0.0, 0.0], [0.0, 1.0]], dtype=np.complex128)
PPLUS = np.full((2, 2), 0.5, dtype=np.complex128)

DEFAULT_TOL = 1e-12


def bit(x: int, n: int, i: int) -> int:
    return (int(x) >> (n - 1 - i)) & 1


class GroverMPS:
    """One Grover instance held as an MPS in complex128."""

    def __init__(self, n: int, marked, chi_cap: int, tol: float = DEFAULT_TOL):
        self.n = int(n)
        self.marked = [int(x) for x in marked]
        self.chi_cap = int(chi_cap)
        self.tol = float(tol)
        self.k_done = 0
        self.discarded = 0.0          # largest discarded weight sum_{j dropped} sigma_j^2 / sum sigma^2
        self.norm_drift = 0.0         # largest |norm - 1| seen before a renormalisation
        self.init_uniform()

    # --- a2: |s> = |+>^n (Eq. (2)) -------------------------------------------------
    def init_uniform(self):
        h = 1.0 / math.sqrt(2.0)
        self.A = [np.full((1, 2, 1), h, dtype=np.complex128) for _ in range(self.n)]
        self.k_done = 0

    # --- a3/a6: a reflection as a bond-2 MPO ------------------------------------------
    def apply_reflection_mpo(self, projs, c0: float, c1: float):
        n = self.n
        out = []
        for i, A in enumerate(self.A):
            PA = np.einsum("st,atb->asb", projs[i], A)
            l, _, r = A.shape
            if n == 1:
                B = c0 * A + c1 * PA
            elif i == 0:
                B = np.concatenate([A, PA], axis=2)
            elif i == n - 1:
                B = np.concatenate([c0 * A, c1 * PA], axis=0)
            else:
                B = np.zeros((2 * l, 2, 2 * r), dtype=np.complex128)
                B[:l, :, :r] = A
                B[l:, :, r:] = PA
            out.append(B)
        self.A = out

    # --- a4: QR left-canonicalisation sweep ---------------------------------------------
    def qr_sweep(self):
        R = np.ones((1, 1), dtype=np.complex128)
        for i in range(self.n - 1):
            X = np.tensordot(R, self.A[i], axes=(1, 0))
            r, _, D = X.shape
            Q, R = np.linalg.qr(X.reshape(r * 2, D), mode="reduced")
            self.A[i] = Q.reshape(r, 2, Q.shape[1])
        self.A[-1] = np.tensordot(R, self.A[-1], axes=(1, 0))

    # --- a5: truncated-SVD sweep --------------------------------------------------------
    def svd_sweep(self):
        for i in range(self.n - 1, 0, -1):
            l, _, r = self.A[i].shape
            U, S, Vh = np.linalg.svd(self.A[i].reshape(l, 2 * r), full_matrices=False)
            keep = int(np.count_nonzero(S >= self.tol * S[0])) if S[0] > 0 else 1
            keep = max(1, min(keep, self.chi_cap))
            tot = float(np.sum(S * S))
            if tot > 0:
                self.discarded = max(self.discarded, float(np.sum(S[keep:] ** 2)) / tot)
            self.A[i] = Vh[:keep].reshape(keep, 2, r)
            self.A[i - 1] = np.tensordot(self.A[i - 1], U[:, :keep] * S[:keep], axes=(2, 0))

    def reflect(self, projs, c0, c1):
        """One multi-controlled-Z reflection: MPO, QR sweep, truncated-SVD sweep."""
        self.apply_reflection_mpo(projs, c0, c1)
        self.qr_sweep()
        self.svd_sweep()

    # --- a7: renormalisation --------------------------------------------------------------
    def renormalise(self):
        nrm = float(np.linalg.norm(self.A[0]))
        self.norm_drift = max(self.norm_drift, abs(nrm - 1.0))
        self.A[0] = self.A[0] / nrm

    # --- one Grover iterate G = D O (Eq. (3)) ---------------------------------------------
    def iterate(self, k: int = 1):
        n = self.n
        for _ in range(k):
            for x in self.marked:
                self.reflect([P1 if bit(x, n, i) else P0 for i in range(n)], 1.0, -2.0)
            self.reflect([PPLUS] * n, -1.0, 2.0)
            self.renormalise()
            self.k_done += 1

    # --- read-out -------------------------------------------------------------------------
    def bond_dims(self):
        return [1] + [A.shape[2] for A in self.A[:-1]] + [1]

    def amplitude(self, x: int) -> complex:
        v = np.ones((1,), dtype=np.complex128)
        for i in range(self.n):
            v = v @ self.A[i][:, bit(x, self.n, i), :]
        return complex(v[0])

    def norm2(self) -> float:
        E = np.ones((1, 1), dtype=np.complex128)
        for A in self.A:
            E = sum(A[:, s, :].conj().T @ E @ A[:, s, :] for s in range(2))
        return float(E[0, 0].real)

    def marked_prob(self) -> float:
        """sum_{x in W} |<x|psi>|^2 / <psi|psi> (Eq. (6))."""
        return sum(abs(self.amplitude(x)) ** 2 for x in self.marked) / self.norm2()

    def statevector(self) -> np.ndarray:
        psi = self.A[0].reshape(2, -1)
        for A in self.A[1:]:
            l, _, r = A.shape
            psi = (psi @ A.reshape(l, 2 * r)).reshape(-1, r)
        return psi.reshape(-1)

    def schmidt_values(self, cut: int) -> np.ndarray:
        """Singular values at bond `cut` (1..n-1); the chain must be right-canonical."""
        T = self.A[0]
        for A in self.A[1:cut]:
            T = np.tensordot(T, A, axes=(T.ndim - 1, 0))
        left = T.reshape(-1, T.shape[-1])
        Ql, Rl = np.linalg.qr(left)
        return np.linalg.svd(Rl, compute_uv=False)

    # --- a9: perfect sampling -----------------------------------------------------------------
    def sample(self, shots: int, seed: int, inst: int = 0):
        """Site-by-site sampling on the right-canonical chain with the shared Philox stream.
        Returns (bits, p0_at_each_decision) so tests can check near-tie decisions."""
        n = self.n
        bits = np.zeros(shots, dtype=np.uint64)
        p0s = np.zeros((shots, n))
        us = np.zeros((shots, n))
        for sh in range(shots):
            v = np.ones((1,), dtype=np.complex128)
            x = 0
            for i in range(n):
                w0 = v @ self.A[i][:, 0, :]
                w1 = v @ self.A[i][:, 1, :]
                q0 = float(np.vdot(w0, w0).real)
                q1 = float(np.vdot(w1, w1).real)
                p0 = q0 / (q0 + q1)
                u = philox.uniform(seed, inst, sh, i)
                p0s[sh, i] = p0
                us[sh, i] = u
                if u < p0:
                    v = w0 / math.sqrt(q0)
                else:
                    v = w1 / math.sqrt(q1)
                    x |= 1 << (n - 1 - i)
            bits[sh] = x
        return bits, p0s, us


def run(n: int, marked, k: int, chi_cap: int, tol: float = DEFAULT_TOL) -> GroverMPS:
    m = GroverMPS(n, marked, chi_cap, tol)
    m.iterate(k)
    return m
