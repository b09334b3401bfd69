"""Right-preconditioned flexible GMRES (Saad and Schultz; Section 3 of the paper).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Arnoldi with modified Gram-Schmidt, complex Givens rotations for the
Hessenberg least-squares problem, x0 = 0, no restart.  The preconditioned
directions z_j = M v_j are stored (flexible form), so the same loop serves a
fixed preconditioner, the identity (unpreconditioned GMRES) or a changing one.
Stops when the rotated residual estimate falls to tol * ||b||.
"""
from __future__ import annotations

import numpy as np


def givens(a: complex, b: complex):
    """(c, s, r) with [[c, s], [-conj(s), c]] [a, b]^T = [r, 0]^T, c real."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b)
    t = np.hypot(abs(a), abs(b))
    phase = a / abs(a)
    return abs(a) / t, phase * np.conj(b) / t, phase * t


def fgmres(apply_A, b: np.ndarray, apply_M=None, tol: float = 1e-10, max_iter: int = 200):
    """Solve A x = b.  Returns (x, iterations, residual_history)."""
    shape = b.shape
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    beta = np.linalg.norm(b)
    hist = [1.0]
    if beta == 0:
        return np.zeros(shape, dtype=np.complex128), 0, hist
    V = [b / beta]
    Z = []
    H = np.zeros((max_iter + 1, max_iter), dtype=np.complex128)
    cs = np.zeros(max_iter)
    sn = np.zeros(max_iter, dtype=np.complex128)
    g = np.zeros(max_iter + 1, dtype=np.complex128)
    g[0] = beta
    k = 0
    for j in range(max_iter):
        z = V[j] if apply_M is None else np.asarray(apply_M(V[j].reshape(shape))).reshape(-1)
        Z.append(z)
        w = np.asarray(apply_A(z.reshape(shape)), dtype=np.complex128).reshape(-1)
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j] if H[j + 1, j] != 0 else w)
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        cs[j], sn[j], H[j, j] = givens(H[j, j], H[j + 1, j])
        H[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]) / beta)
        if abs(g[j + 1]) <= tol * beta:
            break
    y = np.zeros(k, dtype=np.complex128)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    x = np.zeros_like(b)
    for i in range(k):
        x = x + y[i] * Z[i]
    return x.reshape(shape), k, hist
