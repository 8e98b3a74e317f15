"""Statevector oracles (Sections II and III-B of the paper).

* :func:`grover_sv` -- the plain definition of the iterative method (Section III-A,
  Fig. 1(C)): the state is fed back through G = D O each iteration, with the oracle
  O = I - 2 sum_{x in W} |x><x| and the diffusion D = 2|s><s| - I = H^n (2|0><0| - I) H^n
  (Eqs. (3)-(4)). O flips the marked amplitudes; D maps psi to 2 mean(psi) - psi.
* :func:`grover_gates` -- the same iteration as the gate list of Fig. 1(A): H layer,
  X on the zero bits of x, multi-controlled Z, X again (oracle); H, X on all qubits,
  multi-controlled Z, X, H (diffusion). That circuit equals -G (it realises
  I - 2|s><s| for the diffusion), so after k iterations it gives (-1)^k G^k|s>.
* :func:`dense_grover_unitary` -- G as an explicit 2^n x 2^n matrix from Kronecker
  products of H, X and the multi-controlled Z (n <= 8), for the decomposition check.

Qubit q of the circuit acts on bit (n-1-q) of the basis index (most significant first).
"""
from __future__ import annotations

import numpy as np


def uniform_state(n: int) -> np.ndarray:
    """|s> = N^{-1/2} sum_x |x> (Eq. (2))."""
    return np.full(1 << n, 1.0 / np.sqrt(float(1 << n)), dtype=np.float64)


def grover_sv(n: int, marked, k: int, psi: np.ndarray | None = None) -> np.ndarray:
    """k iterations of psi <- D O psi on the full statevector, FP64 (Eqs. (3)-(4))."""
    idx = np.asarray(marked, dtype=np.int64)
    psi = uniform_state(n) if psi is None else psi.astype(np.complex128 if np.iscomplexobj(psi) else np.float64)
    for _ in range(k):
        psi[idx] *= -1.0                      # O = I - 2 sum_{x in W} |x><x|
        psi = 2.0 * psi.mean() - psi          # D = 2|s><s| - I
    return psi


def _apply_h(psi: np.ndarray, n: int, q: int) -> np.ndarray:
    t = psi.reshape((1 << q), 2, (1 << (n - 1 - q)))
    a, b = t[:, 0, :].copy(), t[:, 1, :].copy()
    s = 1.0 / np.sqrt(2.0)
    t[:, 0, :] = s * (a + b)
    t[:, 1, :] = s * (a - b)
    return t.reshape(-1)


def _apply_x(psi: np.ndarray, n: int, q: int) -> np.ndarray:
    t = psi.reshape((1 << q), 2, (1 << (n - 1 - q)))
    return t[:, ::-1, :].reshape(-1).copy()


def _apply_mcz(psi: np.ndarray) -> np.ndarray:
    out = psi.copy()
    out[-1] *= -1.0                           # Z on |1...1>, all other qubits as controls
    return out


def grover_gates(n: int, marked, k: int) -> np.ndarray:
    """k iterations of the Fig. 1(A) gate list on the statevector (single marked item per
    X-conjugated MCZ; M oracle blocks for M marked items)."""
    psi = np.zeros(1 << n, dtype=np.float64)
    psi[0] = 1.0
    for q in range(n):
        psi = _apply_h(psi, n, q)
    for _ in range(k):
        for x in marked:
            x = int(x)
            zeros = [q for q in range(n) if not (x >> (n - 1 - q)) & 1]
            for q in zeros:
                psi = _apply_x(psi, n, q)
            psi = _apply_mcz(psi)
            for q in zeros:
                psi = _apply_x(psi, n, q)
        for q in range(n):
            psi = _apply_h(psi, n, q)
        for q in range(n):
            psi = _apply_x(psi, n, q)
        psi = _apply_mcz(psi)
        for q in range(n):
            psi = _apply_x(psi, n, q)
        for q in range(n):
            psi = _apply_h(psi, n, q)
    return psi


def dense_grover_unitary(n: int, marked) -> np.ndarray:
    """The circuit of Fig. 1(A) as a dense matrix, built from Kronecker products (n <= 8)."""
    if n > 8:
        raise ValueError("dense unitary only for n <= 8")
    I2 = np.eye(2)
    H = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    X = np.array([[0.0, 1.0], [1.0, 0.0]])

    def layer(ops):
        out = np.array([[1.0]])
        for op in ops:
            out = np.kron(out, op)
        return out

    N = 1 << n
    mcz = np.eye(N)
    mcz[N - 1, N - 1] = -1.0
    Hn = layer([H] * n)
    Xn = layer([X] * n)
    oracle = np.eye(N)
    for x in marked:
        x = int(x)
        Xx = layer([I2 if (x >> (n - 1 - q)) & 1 else X for q in range(n)])
        oracle = Xx @ mcz @ Xx @ oracle
    diffusion = Hn @ Xn @ mcz @ Xn @ Hn
    return diffusion @ oracle
