"""The team kernels' one-sided Jacobi on its own, in every team class's shape (the in-wave variant
for teams of up to 64 lanes, the LDS variant for the three- and four-wave classes), through the
test probe in tests/gpu_probes (built by __graft_entry__.build()).

The truncated SVD of Eq. (4)'s sweep rests on it: the kept left factor is J, the singular values
are the column norms of M^H J. Checked per tile, against what the mathematics fixes:

* J unitary: every 2x2 rotation is unitary to a few ulps, and a tile takes at most
  16 sweeps x (ncj - 1) rounds, so ||J^H J - I||_max <= 1e-12 holds with a wide margin;
* M^H J as returned equals M^H times the returned J (relative Frobenius error <= 1e-12);
* the column norms of M^H J are numpy's singular values of M (to 1e-12 of the largest);
* the returned columns are orthogonal: the sweeps stop once no pair of columns above the skip
  floor (1e-30 of the largest squared norm) had a relative squared overlap above 1e-20, so
  |<a_p, a_q>| <= 1e-10 |a_p| |a_q| for such pairs, and every tile stops before the 16-sweep cap.

The inputs include the cases that stress the pairwise exchange: exactly degenerate singular values
(as a Grover state's Schmidt spectrum has when marked strings share no prefix), near-identity
columns, rank-deficient and wide tiles, graded column norms and a zero column. Both members of a
pair must derive the same rotation to the bit; when they did not, J lost unitarity by up to 1e-7
on such tiles while the rotated columns still matched M^H J.
"""
import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "gpu_probes", "libjacobi_probe.so")
LD, TILE, SWEEPS = 64, 64 * 64, 16
CLASSES = [(0, 2), (1, 3), (2, 5), (3, 8), (4, 17), (5, 32)]  # (class id, bond cap)
KINDS = ("random", "degenerate", "near_identity", "rank_deficient", "wide", "graded", "zero_column")


def load():
    if not os.path.exists(LIB):
        pytest.fail("%s is not built: run __graft_entry__.build() first" % LIB)
    lib = ctypes.CDLL(LIB)
    lib.gmps_probe_jacobi_shape.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.gmps_probe_team_jacobi.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    return lib


def make_tile(rng, kind, kj, maxrows):
    """(rows, ncj, M^H as a rows x ncj complex array)."""
    ncj = 2 * int(rng.integers(1, kj // 2 + 1))
    rows = int(rng.integers(1, maxrows + 1))
    g = lambda r, c: rng.standard_normal((r, c)) + 1j * rng.standard_normal((r, c))
    if kind == "wide":
        rows = int(rng.integers(1, max(2, ncj)))
        ncj = max(ncj, 2)
    elif kind in ("degenerate", "near_identity"):
        rows = int(rng.integers(ncj, maxrows + 1)) if ncj <= maxrows else maxrows
    a = g(rows, ncj)
    if kind == "degenerate":
        # a repeated singular value: orthonormal columns scaled by (3, 1, 1, ..., 1), mixed by a
        # random unitary on the right so that every pair starts far from orthogonal
        q, _ = np.linalg.qr(g(rows, min(rows, ncj)))
        s = np.ones(q.shape[1])
        s[0] = 3.0
        v, _ = np.linalg.qr(g(ncj, ncj))
        a = (q * s) @ v[: q.shape[1], :]
    elif kind == "near_identity":
        a = np.eye(rows, ncj) + 1e-9 * a
    elif kind == "rank_deficient":
        a[:, 1:] = a[:, :1] * (0.5 + np.arange(1, ncj)) + 1e-14 * a[:, 1:]
    elif kind == "graded":
        a = a * 10.0 ** (-rng.integers(0, 15, size=ncj).astype(float))
    elif kind == "zero_column":
        a[:, -1] = 0.0
    return rows, ncj, a


def run_class(torch, lib, w, cap, count, seed):
    kj, maxrows = ctypes.c_int(), ctypes.c_int()
    assert lib.gmps_probe_jacobi_shape(w, ctypes.byref(kj), ctypes.byref(maxrows)) == 0
    kj, maxrows = kj.value, maxrows.value
    rng = np.random.default_rng(seed)
    host = np.zeros((count, LD, LD), dtype=np.complex128)
    dims = np.zeros((count, 2), dtype=np.int32)
    tiles = []
    for t in range(count):
        kind = KINDS[t % len(KINDS)]
        rows, ncj, a = make_tile(rng, kind, kj, maxrows)
        assert 1 <= rows <= maxrows and 2 <= ncj <= kj and ncj % 2 == 0
        host[t, :rows, :ncj] = a
        dims[t] = (rows, ncj)
        tiles.append((kind, rows, ncj, a))
    dev = torch.device("cuda:0")
    d_a = torch.from_numpy(host).to(dev)
    d_dims = torch.from_numpy(dims).to(dev)
    d_aj = torch.zeros_like(d_a)
    d_j = torch.zeros_like(d_a)
    d_sw = torch.zeros(count, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    print("case: team Jacobi probe, class %d (bond cap %d), %d tiles, seed %d" % (w, cap, count, seed), flush=True)
    rc = lib.gmps_probe_team_jacobi(w, d_a.data_ptr(), d_dims.data_ptr(), d_aj.data_ptr(), d_j.data_ptr(),
                                    d_sw.data_ptr(), count, SWEEPS)
    assert rc == 0, rc
    aj, jm, sw = d_aj.cpu().numpy(), d_j.cpu().numpy(), d_sw.cpu().numpy()
    worst = {"unitary": 0.0, "reconstruct": 0.0, "sigma": 0.0, "offdiag": 0.0, "sweeps": int(sw.max())}
    for t, (kind, rows, n, a) in enumerate(tiles):
        u = jm[t, :n, :n]
        b = aj[t, :rows, :n]
        un = np.abs(u.conj().T @ u - np.eye(n)).max()
        rec = np.linalg.norm(a @ u - b) / max(np.linalg.norm(a), 1e-300)
        sv = np.sort(np.linalg.svd(a, compute_uv=False))[::-1]
        cn = np.sort(np.linalg.norm(b, axis=0))[::-1]
        k = len(sv)
        sig = np.abs(cn[:k] - sv).max() / max(sv[0], 1e-300) if sv[0] > 0 else cn.max()
        sig = max(sig, (cn[k:].max() / max(sv[0], 1e-300)) if n > k and sv[0] > 0 else 0.0)
        nr = np.linalg.norm(b, axis=0) ** 2
        off = 0.0
        live = np.nonzero(nr > 1e-30 * nr.max())[0] if nr.max() > 0 else []
        for i in range(len(live)):
            for j in range(i + 1, len(live)):
                p, q = live[i], live[j]
                off = max(off, abs(np.vdot(b[:, p], b[:, q])) / np.sqrt(nr[p] * nr[q]))
        worst["unitary"] = max(worst["unitary"], un)
        worst["reconstruct"] = max(worst["reconstruct"], rec)
        worst["sigma"] = max(worst["sigma"], sig)
        worst["offdiag"] = max(worst["offdiag"], off)
        assert un <= 1e-12, (w, t, kind, rows, n, int(sw[t]), un)
        assert rec <= 1e-12, (w, t, kind, rows, n, rec)
        assert sig <= 1e-12, (w, t, kind, rows, n, sig)
        assert off <= 1e-10, (w, t, kind, rows, n, off)
        assert sw[t] < SWEEPS, (w, t, kind, rows, n, int(sw[t]))
    print("  worst: %s" % ", ".join("%s %.3g" % kv for kv in worst.items()), flush=True)


@pytest.mark.parametrize("w,cap", CLASSES, ids=["bond%d" % c for _, c in CLASSES])
def test_team_jacobi_properties(gpu, w, cap):
    import torch
    run_class(torch, load(), w, cap, 700 if cap <= 8 else 210, 9000 + w)
