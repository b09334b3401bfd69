"""Pins for the oracle's nested-dissection elimination of P (Section 2.3, Figure 1).

P^{-1} from the box-by-box Schur elimination is checked against LAPACK's dense
LU and SuperLU on the assembled sparse P, and the front sizes it discovers
from P's nonzero pattern against the counts that follow from the leaf box
geometry the paper describes ((b-1)^d interior and (b+1)^d closure points).
"""
import collections

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import nested, pipeline, spectral, stencil


def build_P(n, d, b, waves, seed=0):
    W = workloads.small(n, d, b, waves=waves, instance=seed)
    s, q, _ = pipeline.coefficients(W.kind, n, d, W.coeff, W.omega)
    st = stencil.Stencils(n, d, b, s)
    return st.P_matrix(q)


@pytest.mark.parametrize("d,n,b,waves,ordering", [
    (2, 16, 4, 2.0, "octree"), (2, 32, 8, 4.0, "octree"), (2, 32, 4, 4.0, "binary"),
    (2, 16, 8, 2.0, "octree"), (3, 8, 2, 1.0, "octree"), (3, 8, 2, 1.0, "binary"),
    (3, 12, 3, 1.5, "binary")])
def test_nd_solve_equals_dense_solve(d, n, b, waves, ordering):
    P = build_P(n, d, b, waves)
    fac = nested.NDFactor(P, nested.nd_levels(n, d, b, ordering))
    rng = np.random.default_rng(4)
    y = rng.standard_normal((n ** d, 3)) + 1j * rng.standard_normal((n ** d, 3))
    x_ref = np.linalg.solve(P.toarray(), y)
    x = fac.solve(y)
    assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)


def test_nd_solve_equals_superlu_on_parity_grid():
    W = workloads.parity_2d()
    o = pipeline.setup_workload(W)
    rng = np.random.default_rng(5)
    y = rng.standard_normal(W.n ** 2) + 1j * rng.standard_normal(W.n ** 2)
    x_ref = spla.splu(o.P.tocsc()).solve(y)
    assert np.linalg.norm(o.factor.solve(y) - x_ref) <= 1e-10 * np.linalg.norm(x_ref)


def test_front_sizes_follow_box_geometry():
    """Leaves: (F, p) = ((b+1)^2, (b-1)^2); level boxes of width w eliminate their
    interior cross (p = 2w - 3) against their boundary ring (4w points); the last
    front holds the two periodic grid lines of each axis (4n - 4 points)."""
    W = workloads.parity_2d()                    # n = 64, b = 8
    o = pipeline.setup_workload(W)
    got = collections.Counter(o.factor.shapes)
    n, b = W.n, W.b
    expect = collections.Counter({((b + 1) ** 2, (b - 1) ** 2): (n // b) ** 2})
    w = 2 * b
    while w < n:
        expect[(2 * w - 3 + 4 * w, 2 * w - 3)] = (n // w) ** 2
        w *= 2
    expect[(4 * n - 4, 4 * n - 4)] = 1
    assert got == expect
    assert o.factor.factor_entries() == sum(
        cnt * (p * p + 2 * p * (F - p)) for (F, p), cnt in expect.items())


def test_orderings_cover_every_point_once():
    for d, n, b in [(2, 32, 4), (3, 16, 4)]:
        for ordering in ("octree", "binary"):
            levels = nested.nd_levels(n, d, b, ordering)
            allpts = np.concatenate([g for lev in levels for g in lev])
            assert np.array_equal(np.sort(allpts), np.arange(n ** d))
            assert levels[0][0].size == (b - 1) ** d
    # Binary bisection in 3D ends with the two planes of the first cut.
    levels = nested.nd_levels(16, 3, 4, "binary")
    assert len(levels[-1]) == 1 and levels[-1][0].size == 2 * 16 * 16
