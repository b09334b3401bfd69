"""Pins for the oracle's GMRES solve of (I + G q) u = G f (Sections 2.2 and 3).

The solve is tied to a dense LAPACK solve of eq. (Lsq), to closed forms for a
constant medium, to the symmetry of the real operator (reciprocity), to the
independence of u from b, the ordering and the shift, and loosely to the
iteration counts the paper prints for its 2D Helmholtz examples.
"""
import math
import os
import shlex

import numpy as np
import pytest

import workloads
from oracle import gmres, pipeline, spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_givens_zeroes_second_component():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s, r = gmres.givens(a, b)
        assert abs(c * a + s * b - r) < 1e-14 and abs(-np.conj(s) * a + c * b) < 1e-14
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-14


def test_gmres_matches_lapack_on_random_system():
    rng = np.random.default_rng(1)
    n = 40
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist = gmres.fgmres(lambda v: A @ v, b, tol=1e-13, max_iter=n)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    assert it <= n and hist[-1] <= 1e-13
    M = np.linalg.inv(A + 0.1 * rng.standard_normal((n, n)))
    x2, it2, _ = gmres.fgmres(lambda v: A @ v, b, lambda v: M @ v, tol=1e-13, max_iter=n)
    np.testing.assert_allclose(x2, x, rtol=1e-10, atol=1e-12)
    assert it2 < it


@pytest.fixture(scope="module")
def parity():
    W = workloads.parity_2d()
    o = pipeline.setup_workload(W)
    f = W.rhs[0]
    u_star = pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, f, W.omega)
    return W, o, f, u_star


def test_preconditioned_and_plain_gmres_reach_dense_solution(parity):
    W, o, f, u_star = parity
    for prec in (True, False):
        u, it, hist = pipeline.solve(o, f, tol=1e-12, max_iter=400, preconditioned=prec)
        assert np.linalg.norm(u - u_star) <= 1e-9 * np.linalg.norm(u_star)
    u, it, _ = pipeline.solve(o, f, tol=1e-10)
    u0, it0, _ = pipeline.solve(o, f, tol=1e-10, preconditioned=False, max_iter=400)
    assert it <= 12 and it0 >= 2 * it


def test_real_data_gives_real_solution(parity):
    W, o, f, u_star = parity
    u, _, _ = pipeline.solve(o, f, tol=1e-12)
    assert np.abs(u.imag).max() <= 1e-10 * np.abs(u).max()


def test_reciprocity(parity):
    """L - s + q is real symmetric, so u_{delta_a}(x_b) = u_{delta_b}(x_a)."""
    W, o, _, _ = parity
    a, b = (5, 40), (33, 9)
    ua, _, _ = pipeline.solve(o, workloads.grid_delta(W.n, 2, a), tol=1e-12)
    ub, _, _ = pipeline.solve(o, workloads.grid_delta(W.n, 2, b), tol=1e-12)
    assert abs(ua[b] - ub[a]) <= 1e-9 * abs(ua[b])


def test_constant_medium_one_iteration_closed_form():
    """q = 0: P = Q so M = P^{-1} Q = I, and u = G f = F^{-1}[f^ / (4 pi^2 |k|^2 - s)]."""
    n, d = 32, 2
    c = np.full((n, n), 1.3)
    o = pipeline.setup("helmholtz", n, d, 8, c, omega=2 * math.pi * 5.1)
    f = workloads.gaussian_sources(n, d, 1, 1 / 16, 3)[0]
    z = pipeline.precondition(o, f)
    assert np.linalg.norm(z - f) <= 1e-10 * np.linalg.norm(f)
    u, it, _ = pipeline.solve(o, f, tol=1e-10)
    assert it == 1
    fhat = np.fft.fftn(f)
    k2 = spectral.k_squared(n, d)
    u_exact = np.fft.ifftn(fhat / (4 * math.pi ** 2 * k2 - (2 * math.pi * 5.1 / 1.3) ** 2))
    assert np.linalg.norm(u - u_exact) <= 1e-10 * np.linalg.norm(u_exact)


def test_solution_independent_of_b_ordering_and_shift():
    n, d = 32, 2
    W = workloads.small(n, d, 4, waves=4.0, bumps=5)
    f = W.rhs[0]
    ref = pipeline.dense_solution(W.kind, n, d, W.coeff, f, W.omega)
    for b, ordering in [(4, "octree"), (8, "octree"), (4, "binary"), (16, "binary")]:
        o = pipeline.setup(W.kind, n, d, b, W.coeff, W.omega, ordering=ordering)
        u, _, _ = pipeline.solve(o, f, tol=1e-12)
        assert np.linalg.norm(u - ref) <= 1e-9 * np.linalg.norm(ref)
    o = pipeline.setup(W.kind, n, d, 8, W.coeff, W.omega)
    o.s += 37.0
    o.q = o.q + 37.0
    from oracle import stencil, nested
    o.stencils = stencil.Stencils(n, d, 8, o.s)
    o.P = o.stencils.P_matrix(o.q)
    o.factor = nested.NDFactor(o.P, nested.nd_levels(n, d, 8))
    u, _, _ = pipeline.solve(o, f, tol=1e-12)
    assert np.linalg.norm(u - ref) <= 1e-9 * np.linalg.norm(ref)


def test_3d_and_schrodinger_reach_dense_solution():
    W = workloads.small(12, 3, 3, waves=1.5, bumps=3)
    o = pipeline.setup_workload(W, ordering="binary")
    ref = pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, W.rhs[0], W.omega)
    u, it, _ = pipeline.solve(o, W.rhs[0], tol=1e-12)
    assert np.linalg.norm(u - ref) <= 1e-9 * np.linalg.norm(ref)
    for S in (workloads.schrodinger_workload(32, 2, 4, 8), workloads.schrodinger_workload(12, 3, 2, 3)):
        o = pipeline.setup_workload(S)
        ref = pipeline.dense_solution(S.kind, S.n, S.d, S.coeff, S.rhs[0], ell=S.ell, energy=S.energy)
        u, it, _ = pipeline.solve(o, S.rhs[0], tol=1e-12)
        assert np.linalg.norm(u - ref) <= 1e-9 * np.linalg.norm(ref), S.name


def paper_rows():
    rows = []
    with open(os.path.join(GOLDEN, "paper_iterations.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t = shlex.split(line)
                rows.append((t[0], float(t[2]), int(t[3]), int(t[4]), int(t[5])))
    return rows


@pytest.mark.parametrize("table,waves,n,b,n_p", paper_rows())
def test_iteration_counts_near_paper_tables(table, waves, n, b, n_p):
    """The paper's media are not fully specified (amplitudes and widths of the
    Gaussians are not given), so only the order of magnitude is pinned: the
    oracle's count on a medium of the same kind lies within a factor 2."""
    x = workloads.grid_points(n, 2)
    if table == "W21":
        centres = np.array([[0.5, 0.5]])
    else:
        centres = np.random.default_rng(7).uniform(0, 1, (3, 2))
    c = np.ones((n, n))
    for ci in centres:
        c += 0.2 * np.exp(-workloads.periodic_sq_dist(x, ci) / (2 * 0.1 ** 2))
    o = pipeline.setup("helmholtz", n, 2, b, c, omega=2 * math.pi * waves)
    _, it, _ = pipeline.solve(o, workloads.grid_delta(n, 2, (n // 2, n // 2)), tol=1e-6)
    assert n_p / 2 <= it <= 2 * n_p


def test_point_pattern_preconditioner_reaches_dense_solution():
    """The point-neighbourhood pattern (mu(j) = gamma({j}), Section 2.3)
    changes P, not u*: its preconditioned FGMRES reaches the dense solution,
    and P z = Q r holds for the preconditioned vector."""
    W = workloads.small(24, 2, 6, waves=3.0, bumps=3)
    f = W.rhs[0]
    u_star = pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, f, W.omega)
    o = pipeline.setup_workload(W, pattern="points")
    u, it, hist = pipeline.solve(o, f, tol=1e-12, max_iter=200)
    assert np.linalg.norm(u - u_star) / np.linalg.norm(u_star) <= 1e-9
    r = np.random.default_rng(3).standard_normal(f.shape) + 0j
    z = pipeline.precondition(o, r).reshape(-1)
    from oracle import stencil
    Qr = stencil.apply_Q(o.stencils, r).reshape(-1)
    assert np.linalg.norm(o.P @ z - Qr) <= 1e-10 * np.linalg.norm(Qr)
