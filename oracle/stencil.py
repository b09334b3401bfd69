"""The sparsifying operator Q, the matrix C and the sparse P = Q + C q.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2.2 (conditions on Q, definition of C and P) and Section 2.3
(neighbourhood gamma, the leaf set partition into cells/faces/edges/vertices,
T_S = G(S, gamma^c) G(beta, gamma^c)^+ via an explicit pseudoinverse,
Q(S, gamma(S)) = [I  -T_S] with columns ordered (S, beta(S))).

Sets are labelled by a boolean mask over the d axes and a leaf-box anchor
a in [0, n/b)^d.  With b = 1 every set is a single point, whose
neighbourhood is mu(j) = gamma({j}) (the point pattern Section 2.3 weighs
against the set pattern): only the all-True mask has points then.  Axis i of the set is pinned to the grid line a_i b when
mask[i] is set and runs over the open interval a_i b + 1 .. a_i b + b - 1
otherwise.  So the all-False mask is a cell, the all-True mask a vertex, one
True axis an edge (2D) or a face (3D), two True axes an edge (3D).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import spectral


def set_masks(d: int):
    """All 2^d set types (orientation-resolved), cells first, vertex last."""
    return [tuple(bool(x) for x in m) for m in itertools.product((0, 1), repeat=d)]


def set_kind(mask) -> str:
    pinned = sum(mask)
    d = len(mask)
    if pinned == 0:
        return "cell"
    if pinned == d:
        return "vertex"
    if d == 3 and pinned == 1:
        return "face"
    return "edge"


def set_points(n: int, b: int, mask, anchor) -> np.ndarray:
    """Multi-indices of the set, shape (|S|, d), in lexicographic order."""
    ranges = []
    for i, pinned in enumerate(mask):
        base = anchor[i] * b
        ranges.append([base] if pinned else list(range(base + 1, base + b)))
    pts = np.array(list(itertools.product(*ranges)), dtype=np.int64).reshape(-1, len(mask))
    return pts % n


def ravel(points: np.ndarray, n: int) -> np.ndarray:
    """C-order global index of multi-indices (last axis fastest)."""
    idx = np.zeros(points.shape[0], dtype=np.int64)
    for i in range(points.shape[1]):
        idx = idx * n + points[:, i]
    return idx


def gamma(points: np.ndarray, n: int) -> np.ndarray:
    """gamma(S) = { i : exists j in S with ||j - i||_inf <= 1 }, distance mod n (Section 2.3).

    Written straight from the definition: the union of the 3^d neighbours of
    every point, returned as sorted unique C-order indices.
    """
    d = points.shape[1]
    out = []
    for delta in itertools.product((-1, 0, 1), repeat=d):
        out.append(ravel((points + np.array(delta)) % n, n))
    return np.unique(np.concatenate(out))


def set_geometry(n: int, d: int, b: int, mask, anchor=None):
    """(S, beta) as C-order global indices; S lexicographic, beta sorted.

    The column order of Q(S, gamma(S)) is (S, beta(S)) (Section 2.3).
    """
    if anchor is None:
        anchor = (0,) * d
    S = ravel(set_points(n, b, mask, anchor), n)
    g = gamma(set_points(n, b, mask, anchor), n)
    beta = np.setdiff1d(g, S, assume_unique=True)
    return S, beta


def unravel(idx: np.ndarray, n: int, d: int) -> np.ndarray:
    out = np.zeros((idx.shape[0], d), dtype=np.int64)
    rem = idx.copy()
    for i in range(d - 1, -1, -1):
        out[:, i] = rem % n
        rem //= n
    return out


def green_block(g: np.ndarray, rows: np.ndarray, cols: np.ndarray, n: int, d: int) -> np.ndarray:
    """G(rows, cols) with G[i, j] = g[(i - j) mod n] (eq. G)."""
    r = unravel(rows, n, d)
    c = unravel(cols, n, d)
    diff = (r[:, None, :] - c[None, :, :]) % n
    return g[tuple(diff[..., i] for i in range(d))]


def stencil_T(g: np.ndarray, n: int, d: int, b: int, mask, anchor=None, chunk: int = 16384):
    """T_S = G(S, gamma(S)^c) G(beta(S), gamma(S)^c)^+ (Section 2.3, eq. Qc).

    The pseudoinverse is the SVD one with MATLAB's default cutoff
    (singular values below max(size) * sigma_max * eps are dropped).
    Returns (T, S, beta).
    """
    S, beta = set_geometry(n, d, b, mask, anchor)
    gam = np.concatenate([S, beta])
    outside = np.setdiff1d(np.arange(n ** d), gam)
    A = green_block(g, beta, outside, n, d)
    pinvA = np.linalg.pinv(A, rcond=max(A.shape) * np.finfo(np.float64).eps)
    del A
    T = np.zeros((S.size, beta.size), dtype=np.complex128)
    for lo in range(0, outside.size, chunk):
        cols = outside[lo:lo + chunk]
        T += green_block(g, S, cols, n, d) @ pinvA[lo:lo + chunk]
    return T, S, beta


def stencil_C(g: np.ndarray, n: int, d: int, T: np.ndarray, S: np.ndarray, beta: np.ndarray):
    """C(S, gamma(S)) = Q(S, gamma(S)) G(gamma(S), gamma(S)) (Section 2.3)."""
    gam = np.concatenate([S, beta])
    Qblk = np.concatenate([np.eye(S.size), -T], axis=1)
    return Qblk @ green_block(g, gam, gam, n, d)


class Stencils:
    """T_S and C_S for every set type, computed once per type at anchor 0.

    The paper notes that T_S (hence C_S) is the same for every translate of
    a set, so one computation per type suffices (Section 2.3).
    """

    def __init__(self, n: int, d: int, b: int, s: float):
        if n % b or (n // b) < 2:
            raise ValueError("b must divide n with at least two leaf boxes per axis")
        self.n, self.d, self.b, self.s = n, d, b, s
        self.g = spectral.green_kernel(n, d, s)
        # (with b = 1 only the vertex mask, a single point, is not empty)
        self.masks = [m for m in set_masks(d) if b > 1 or all(m)]
        self.T, self.C, self.S0, self.beta0 = {}, {}, {}, {}
        for mask in self.masks:
            T, S, beta = stencil_T(self.g, n, d, b, mask)
            self.T[mask] = T
            self.C[mask] = stencil_C(self.g, n, d, T, S, beta)
            self.S0[mask], self.beta0[mask] = S, beta

    def instances(self, mask):
        """(rows, cols) global indices for every translate of the set type.

        rows: (m^d, |S|), cols: (m^d, |S| + |beta|) in the (S, beta) order.
        """
        n, d, b = self.n, self.d, self.b
        m = n // b
        rows, cols = [], []
        base = np.concatenate([self.S0[mask], self.beta0[mask]])
        base_pts = unravel(base, n, d)
        for anchor in itertools.product(range(m), repeat=d):
            shift = np.array(anchor, dtype=np.int64) * b
            pts = (base_pts + shift) % n
            gidx = ravel(pts, n)
            rows.append(gidx[: self.S0[mask].size])
            cols.append(gidx)
        return np.array(rows), np.array(cols)

    def _assemble(self, value_fn):
        N = self.n ** self.d
        R, Cc, V = [], [], []
        for mask in self.masks:
            rows, cols = self.instances(mask)
            vals = value_fn(mask, cols)           # (inst, |S|, |gamma|)
            R.append(np.broadcast_to(rows[:, :, None], vals.shape).reshape(-1))
            Cc.append(np.broadcast_to(cols[:, None, :], vals.shape).reshape(-1))
            V.append(vals.reshape(-1))
        M = sp.coo_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(Cc))),
                          shape=(N, N)).tocsr()
        return M

    def Q_matrix(self):
        """Sparse Q: Q(S, gamma(S)) = [I  -T_S] for every set S (Section 2.3)."""
        def fn(mask, cols):
            blk = np.concatenate([np.eye(self.S0[mask].size), -self.T[mask]], axis=1)
            return np.broadcast_to(blk, (cols.shape[0],) + blk.shape)
        return self._assemble(fn)

    def P_matrix(self, q: np.ndarray):
        """Sparse P = Q + C q (Section 2.2), same pattern as Q."""
        qf = np.asarray(q, dtype=np.float64).reshape(-1)

        def fn(mask, cols):
            blk = np.concatenate([np.eye(self.S0[mask].size), -self.T[mask]], axis=1)
            return blk[None] + self.C[mask][None] * qf[cols][:, None, :]
        return self._assemble(fn)


def apply_Q(st: Stencils, r: np.ndarray) -> np.ndarray:
    """Q r for a grid function r, written per set: (Q r)_S = r_S - T_S r_beta(S)."""
    flat = np.asarray(r, dtype=np.complex128).reshape(-1)
    out = np.empty_like(flat)
    for mask in st.masks:
        rows, cols = st.instances(mask)
        nS = rows.shape[1]
        out[rows] = flat[rows] - flat[cols[:, nS:]] @ st.T[mask].T
    return out.reshape(r.shape)
