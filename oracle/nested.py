"""Nested-dissection block elimination of the sparse P (Section 2.3, Figure 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The domain is cut into boxes of width b h (the leaves); the interior points
of every box are eliminated by a Schur complement, boxes are merged (four at
a time in 2D, eight in 3D for the "octree" ordering of Figure 1; or two at a
time along alternating axes for the "binary" ordering), and the process
repeats until one box (the whole periodic domain) remains, whose remaining
points are eliminated last.

This is plain block Gaussian elimination on the current reduced sparse
matrix.  The neighbours of each box's pivots are read off that matrix's
nonzero pattern rather than assumed from geometry, and each pivot block is
factorised by LAPACK's LU with partial pivoting (pivots restricted to the
box's own fully-summed rows).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def octree_shapes(n: int, d: int, b: int):
    """Box widths per level for Figure 1's ordering: b, 2b, 4b, ..., n."""
    shapes, w = [], b
    while w < n:
        shapes.append((w,) * d)
        w *= 2
    if w != n:
        raise ValueError("n / b must be a power of two")
    shapes.append((n,) * d)
    return shapes


def binary_shapes(n: int, d: int, b: int):
    """Box widths per level when boxes merge two at a time, axes in turn."""
    if (n // b) & (n // b - 1):
        raise ValueError("n / b must be a power of two")
    shape = [b] * d
    shapes = [tuple(shape)]
    axis = 0
    while any(w < n for w in shape):
        while shape[axis] >= n:
            axis = (axis + 1) % d
        shape[axis] *= 2
        shapes.append(tuple(shape))
        axis = (axis + 1) % d
    return shapes


def nd_levels(n: int, d: int, b: int, ordering: str = "octree"):
    """Pivot sets (C-order indices) of every box, level by level, leaves first."""
    shapes = octree_shapes(n, d, b) if ordering == "octree" else binary_shapes(n, d, b)
    N = n ** d
    coords = np.stack(np.unravel_index(np.arange(N), (n,) * d), axis=1)
    alive = np.ones(N, dtype=bool)
    levels = []
    for shape in shapes:
        interior = alive.copy()
        box = np.zeros(N, dtype=np.int64)
        for i, w in enumerate(shape):
            if w < n:
                interior &= (coords[:, i] % w) != 0
            box = box * (n // w) + coords[:, i] // w
        idx = np.nonzero(interior)[0]
        order = np.argsort(box[idx], kind="stable")
        idx = idx[order]
        bid = box[idx]
        cuts = np.nonzero(np.diff(bid))[0] + 1
        groups = [g for g in np.split(idx, cuts) if g.size]
        levels.append(groups)
        alive[idx] = False
    if alive.any():
        raise AssertionError("ordering left points uneliminated")
    return levels


class NDFactor:
    """Block LU of P in nested-dissection order.

    ``fronts`` holds, in elimination order, tuples
    (piv, nbr, lu_piv_block, P_piv_nbr, P_nbr_piv) of the reduced matrix at
    the time the box was eliminated.
    """

    def __init__(self, P: sp.spmatrix, levels):
        N = P.shape[0]
        S = sp.csr_matrix(P, dtype=np.complex128)
        alive = np.ones(N, dtype=bool)
        self.fronts = []
        self.shapes = []
        for groups in levels:
            Scsc = S.tocsc()
            R, C, V = [], [], []
            for piv in groups:
                rowblk = S[piv]
                colblk = Scsc[:, piv]
                nz = np.union1d(rowblk.indices, colblk.indices)
                nz = nz[alive[nz]]
                nbr = np.setdiff1d(nz, piv, assume_unique=False)
                A11 = rowblk[:, piv].toarray()
                A12 = rowblk[:, nbr].toarray()
                A21 = colblk[nbr].toarray()
                lu = sla.lu_factor(A11, check_finite=True)
                upd = -A21 @ sla.lu_solve(lu, A12)
                self.fronts.append((piv, nbr, lu, A12, A21))
                self.shapes.append((piv.size + nbr.size, piv.size))
                R.append(np.repeat(nbr, nbr.size))
                C.append(np.tile(nbr, nbr.size))
                V.append(upd.reshape(-1))
            for piv in groups:
                alive[piv] = False
            if R:
                S = S + sp.coo_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))),
                                      shape=(N, N)).tocsr()

    def solve(self, y: np.ndarray) -> np.ndarray:
        """x = P^{-1} y by forward elimination then back substitution."""
        shape = y.shape
        x = np.array(y, dtype=np.complex128).reshape(shape[0], -1) if y.ndim > 1 else \
            np.array(y, dtype=np.complex128).reshape(-1, 1)
        for piv, nbr, lu, A12, A21 in self.fronts:
            x[nbr] -= A21 @ sla.lu_solve(lu, x[piv])
        for piv, nbr, lu, A12, A21 in reversed(self.fronts):
            x[piv] = sla.lu_solve(lu, x[piv] - A12 @ x[nbr])
        return x.reshape(shape)

    def factor_entries(self) -> int:
        """Number of stored factor entries: sum of p^2 + 2 p (F - p)."""
        return int(sum(p * p + 2 * p * (F - p) for F, p in self.shapes))
