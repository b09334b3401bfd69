"""End-to-end oracle: setup and preconditioned solve (Sections 2.2-2.3, 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import gmres, nested, spectral, stencil


@dataclasses.dataclass
class OracleSetup:
    n: int
    d: int
    b: int
    s: float
    q: np.ndarray
    shift_moves: int
    stencils: stencil.Stencils
    P: object
    factor: nested.NDFactor


def coefficients(kind: str, n: int, d: int, coeff, omega=0.0, ell=1.0, energy=0.0):
    """(s, q, number of shift perturbations) for either equation (eq. Dsq, Section 2.2)."""
    if kind == "helmholtz":
        s, q = spectral.split_helmholtz(omega, coeff)
    elif kind == "schrodinger":
        s, q = spectral.split_schrodinger(ell, energy, coeff)
    else:
        raise ValueError(kind)
    s, q, moves = spectral.perturb_shift(n, d, s, q)
    return s, q, moves


def setup(kind: str, n: int, d: int, b: int, coeff, omega=0.0, ell=1.0, energy=0.0,
          ordering: str = "octree", pattern: str = "sets") -> OracleSetup:
    """pattern "sets": the stencils of the leaf boxes' cells, edges, faces and
    vertices (Section 2.3); "points": every point with its own neighbourhood
    mu(j) = gamma({j}).  The nested dissection uses leaf boxes of width b in
    both cases."""
    s, q, moves = coefficients(kind, n, d, coeff, omega, ell, energy)
    st = stencil.Stencils(n, d, b if pattern == "sets" else 1, s)
    P = st.P_matrix(q)
    fac = nested.NDFactor(P, nested.nd_levels(n, d, b, ordering))
    return OracleSetup(n=n, d=d, b=b, s=s, q=q, shift_moves=moves, stencils=st, P=P, factor=fac)


def setup_workload(W, ordering: str = "octree", pattern: str = "sets") -> OracleSetup:
    return setup(W.kind, W.n, W.d, W.b, W.coeff, W.omega, W.ell, W.energy, ordering, pattern)


def precondition(o: OracleSetup, r: np.ndarray) -> np.ndarray:
    """z = P^{-1} Q r, the sparsifying preconditioner (Section 2.2)."""
    return o.factor.solve(stencil.apply_Q(o.stencils, r).reshape(-1)).reshape(r.shape)


def rhs_transform(o: OracleSetup, f: np.ndarray) -> np.ndarray:
    """g = G f (Section 2.2)."""
    return spectral.apply_green(f, o.d, o.s)


def solve(o: OracleSetup, f: np.ndarray, tol: float = 1e-10, max_iter: int = 300,
          preconditioned: bool = True):
    """Solve (I + G q) u = G f by FGMRES; returns (u, iterations, history)."""
    g = rhs_transform(o, f)
    A = lambda z: spectral.apply_integral(z, o.d, o.s, o.q)
    M = (lambda r: precondition(o, r)) if preconditioned else None
    return gmres.fgmres(A, g, M, tol=tol, max_iter=max_iter)


def dense_solution(kind: str, n: int, d: int, coeff, f, omega=0.0, ell=1.0, energy=0.0):
    """Ground truth u* of (L - s + q) u = f by a dense solve (eq. Lsq); N <= ~4096."""
    s, q, _ = coefficients(kind, n, d, coeff, omega, ell, energy)
    A = spectral.dense_differential(n, d, s, q)
    return np.linalg.solve(A, np.asarray(f, dtype=np.complex128).reshape(-1)).reshape(f.shape)


def differential_residual(o: OracleSetup, u: np.ndarray, f: np.ndarray) -> float:
    """||f - (L - s + q) u|| / ||f||."""
    r = f - spectral.apply_differential(u, o.d, o.s, o.q)
    return float(np.linalg.norm(r) / np.linalg.norm(f))
