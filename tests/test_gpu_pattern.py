"""The point-neighbourhood stencil pattern on the GPU path (Section 2.3).

Section 2.3 weighs using every point as its own set, with the neighbourhood
mu(j) = gamma({j}), against the set pattern of the leaf boxes' cells, edges,
faces and vertices, and keeps the latter because the single-point stencil
truncates too much of Q G.  Both patterns give a valid P (Q + C q on the
same front structure) and the same u*; what differs is how well P^{-1} Q
preconditions.  These tests compare the GPU's point pattern with the oracle's
(stencil, Q r, P z = Q r, the solution) and report the iteration counts of
both patterns.
"""
import numpy as np
import pytest

import workloads
from oracle import pipeline, stencil

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def solver(W, **kw):
    from paper_1409_0297_amd import Solver
    return Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, ell=W.ell, energy=W.energy, **kw)


@pytest.fixture(scope="module")
def point2d():
    W = workloads.parity_2d(nrhs=2)
    o = pipeline.setup_workload(W, pattern="points")
    S = solver(W, tol=1e-12, max_iter=300, pattern="points")
    yield W, o, S
    S.close()


def test_point_stencil_matches_oracle(point2d):
    W, o, S = point2d
    mask = (True, True)
    off, T, C = S.stencil(3)                       # the only set type with points
    assert T.shape == (1, 8) and C.shape == (1, 9)
    glob = stencil.ravel(np.mod(off.astype(np.int64), W.n), W.n)
    pos = {int(g): i for i, g in enumerate(o.stencils.beta0[mask])}
    To = o.stencils.T[mask][:, [pos[int(g)] for g in glob[1:]]]
    assert rel(T, To) <= 1e-8
    for t in range(3):                             # cells and edges have no points
        nS, nB = S.stencil(t)[1].shape
        assert nS == 0


def test_point_q_apply_and_preconditioner(point2d):
    W, o, S = point2d
    r = np.random.default_rng(21).standard_normal((2, W.n, W.n)) + 0j
    y = cpu(S.apply_q(r)).reshape(r.shape)
    for i in range(2):
        assert rel(y[i], stencil.apply_Q(o.stencils, r[i])) <= 1e-8
    z = cpu(S.apply_precond(r)).reshape(r.shape)
    for i in range(2):
        Qr = stencil.apply_Q(o.stencils, r[i]).reshape(-1)
        assert np.linalg.norm(o.P @ z[i].reshape(-1) - Qr) / np.linalg.norm(Qr) <= 1e-8


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_point_pattern_solves_and_iterations(prec):
    W = workloads.parity_2d(nrhs=1)
    u_star = pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, W.rhs[0], W.omega)
    its = {}
    for pattern in ("sets", "points"):
        S = solver(W, prec=prec, tol=1e-12, max_iter=300, pattern=pattern)
        u, iters, relres, code = S.solve(W.rhs)
        S.close()
        assert code == 0, (pattern, code)
        assert rel(cpu(u).reshape(u_star.shape), u_star) <= 1e-9
        its[pattern] = iters[0]
    print(f"64^2 omega = 2 pi 8, {prec}: iterations sets {its['sets']}, points {its['points']}")
    assert its["points"] > its["sets"]


def test_point_pattern_3d():
    W = workloads.small(12, 3, 3, waves=1.5, bumps=3)
    u_star = pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, W.rhs[0], W.omega)
    o = pipeline.setup_workload(W, pattern="points")
    uo, it_o, _ = pipeline.solve(o, W.rhs[0], tol=1e-12, max_iter=300)
    S = solver(W, tol=1e-12, max_iter=300, pattern="points")
    u, iters, relres, code = S.solve(W.rhs)
    S.close()
    assert code == 0
    assert rel(cpu(u).reshape(u_star.shape), u_star) <= 1e-9
    # CGS2 on the GPU, MGS in the oracle: the same in exact arithmetic
    assert abs(iters[0] - it_o) <= 1, (iters[0], it_o)
