"""FGMRES iterations replayed from a captured HIP graph.

The graph is captured once per factor and right-hand-side count and replayed
once per iteration with the step index in device memory.  Every replayed
solve must give the eager solve's iterations and solution (same kernels in
the same order), also after other eager work on the stream and with
repeated solves on the same factor (each replay rereads the device index).
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_graph_replays_match_eager_solves(prec):
    from paper_1409_0297_amd import Solver
    W = workloads.parity_2d(nrhs=2)
    E = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-11, max_iter=100)
    G = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-11, max_iter=100, graphs=True)
    ue, ie, re, ce = E.solve(W.rhs)
    ue = cpu(ue)
    rng = np.random.default_rng(3)
    for rep in range(3):
        z = rng.standard_normal((2, W.n * W.n)) + 0j
        E.apply_operator(z)                       # eager work between replays
        ug, ig, rg, cg = G.solve(W.rhs)
        assert cg == ce == 0
        assert ig == ie, (rep, ig, ie)
        d = np.linalg.norm(cpu(ug) - ue) / np.linalg.norm(ue)
        assert d <= 1e-13, (rep, d)
        assert np.allclose(rg, re, rtol=1e-6, atol=0)
    # one right-hand side: a second graph for nrhs = 1
    u1, i1, _, c1 = G.solve(W.rhs[0])
    u1e, i1e, _, _ = E.solve(W.rhs[0])
    assert c1 == 0 and i1 == i1e
    assert np.linalg.norm(cpu(u1) - cpu(u1e)) <= 1e-13 * np.linalg.norm(cpu(u1e))
    E.close()
    G.close()


def test_graph_replays_for_an_uneven_batch():
    from paper_1409_0297_amd import BatchSolver
    Ws = [workloads.small(48, 2, 6, waves=5.0, bumps=4), workloads.small(32, 2, 8, waves=4.0, bumps=3, instance=1),
          workloads.small(32, 2, 8, waves=3.0, bumps=3, instance=2)]
    probs = [dict(kind=W.kind, n=W.n, d=W.d, b=W.b, coeff=W.coeff, omega=W.omega) for W in Ws]
    E = BatchSolver(probs, tol=1e-11)
    G = BatchSolver(probs, tol=1e-11, graphs=True)
    fs = [W.rhs.reshape(1, -1) for W in Ws]
    ue, ie, _, ce = E.solve(fs)
    for _ in range(2):
        ug, ig, _, cg = G.solve(fs)
        assert cg == ce == 0 and ig == ie
        for a, b in zip(ug, ue):
            assert np.linalg.norm(cpu(a) - cpu(b)) <= 1e-13 * np.linalg.norm(cpu(b))
    E.close()
    G.close()



def test_cooperative_substitution_matches_level_launches():
    """SPP_F_PERSISTENT runs consecutive small-front levels of the
    substitution as one cooperative launch with grid barriers between levels;
    the fronts see the same arithmetic, so the results must agree.  With
    complex128 fronts, levels of at least 512 fronts keep the LU in place:
    on 512^2 with b = 8 that is the 4096 leaves and the 1024 fronts above."""
    from paper_1409_0297_amd import Solver
    prec = "c128"
    W = workloads.helmholtz_workload("mid", 5, 512, 2, 32.0, 16, 0.05, 8, nrhs=5)
    A = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-11, max_iter=100, persistent=True)
    B = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-11, max_iter=100)
    rng = np.random.default_rng(21)
    r = rng.standard_normal((5, W.n * W.n)) + 1j * rng.standard_normal((5, W.n * W.n))
    za, zb = cpu(A.apply_precond(r)), cpu(B.apply_precond(r))
    assert np.linalg.norm(za - zb) <= 1e-13 * np.linalg.norm(zb)
    ua, ia, _, ca = A.solve(W.rhs)
    ub, ib, _, cb = B.solve(W.rhs)
    assert ca == cb == 0 and ia == ib
    assert np.linalg.norm(cpu(ua) - cpu(ub)) <= 1e-13 * np.linalg.norm(cpu(ub))
    A.close()
    B.close()
