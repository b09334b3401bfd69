"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every GPU result is compared with the oracle on the same seeded inputs:
element by element for the operator, Green apply, coefficients, stencils and
Q; through the defining equation P z = Q r for the preconditioner; and
against the dense ground truth for full solves.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import pipeline, spectral, stencil

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def parity():
    from paper_1409_0297_amd import Solver
    W = workloads.parity_2d(nrhs=2)
    o = pipeline.setup_workload(W)
    S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-12, max_iter=100)
    yield W, o, S
    S.close()


def random_field(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_coefficients(parity):
    W, o, S = parity
    s, q = S.coefficients()
    assert abs(s - o.s) <= 1e-12 * abs(o.s)
    np.testing.assert_allclose(cpu(q).reshape(o.q.shape), o.q, rtol=0, atol=1e-10 * abs(o.s))


def test_operator_and_green_apply(parity):
    W, o, S = parity
    z = random_field((2, W.n, W.n), 11)
    w = cpu(S.apply_operator(z)).reshape(z.shape)
    ref = np.stack([spectral.apply_integral(z[i], 2, o.s, o.q) for i in range(2)])
    # Both sides round O(eps log N) per transform and the oracle's dense DFT
    # O(eps sqrt(n)); 1e-12 leaves a factor ~10 over the observed 1.2e-13.
    e = rel(w, ref)
    assert e <= 1e-12, e
    g = cpu(S.apply_green(z)).reshape(z.shape)
    refg = np.stack([spectral.apply_green(z[i], 2, o.s) for i in range(2)])
    e = rel(g, refg)
    assert e <= 1e-12, e


def stencil_maps(off, o_S, o_B, n, d):
    """Positions of the GPU's (S, beta) order inside the oracle's S and beta lists."""
    glob = stencil.ravel(np.mod(off.astype(np.int64), n), n)
    posS = {int(g): i for i, g in enumerate(o_S)}
    posB = {int(g): i for i, g in enumerate(o_B)}
    nS = len(o_S)
    return np.array([posS[int(g)] for g in glob[:nS]]), np.array([posB[int(g)] for g in glob[nS:]])


def test_stencils_match_pseudoinverse(parity):
    W, o, S = parity
    st = o.stencils
    for t in range(4):
        mask = tuple(bool((t >> i) & 1) for i in range(2))
        off, T, C = S.stencil(t)
        pS, pB = stencil_maps(off, st.S0[mask], st.beta0[mask], W.n, 2)
        To = st.T[mask][np.ix_(pS, pB)]
        e = rel(T, To)
        assert e <= 1e-8, (mask, e)
        Co = st.C[mask][np.ix_(pS, np.concatenate([pS, len(pS) + pB]))]
        e = rel(C, Co)
        assert e <= 1e-8, (mask, e)


def test_q_apply(parity):
    W, o, S = parity
    r = random_field((2, W.n, W.n), 12)
    y = cpu(S.apply_q(r)).reshape(r.shape)
    ref = np.stack([stencil.apply_Q(o.stencils, r[i]) for i in range(2)])
    # Q inherits the stencil agreement (T_S to 1e-8, Gram route vs SVD).
    e = rel(y, ref)
    assert e <= 1e-8, e


def test_preconditioner_solves_P(parity):
    W, o, S = parity
    r = random_field((2, W.n, W.n), 13)
    z = cpu(S.apply_precond(r)).reshape(r.shape)
    for i in range(2):
        Qr = stencil.apply_Q(o.stencils, r[i]).reshape(-1)
        res = np.linalg.norm(o.P @ z[i].reshape(-1) - Qr) / np.linalg.norm(Qr)
        assert res <= 1e-8, res
        e = rel(z[i], pipeline.precondition(o, r[i]))
        assert e <= 1e-7, e


def test_solve_matches_dense_solution(parity):
    W, o, S = parity
    u, iters, relres, code = S.solve(W.rhs)
    u = cpu(u).reshape(W.rhs.shape)
    assert code == 0
    for i in range(2):
        u_star = pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, W.rhs[i], W.omega)
        e = rel(u[i], u_star)
        assert e <= 1e-9, e
        _, it_o, _ = pipeline.solve(o, W.rhs[i], tol=1e-12)
        assert abs(iters[i] - it_o) <= 1
        assert relres[i] <= 1e-11


def test_unpreconditioned_and_mixed_precision_reach_same_solution():
    from paper_1409_0297_amd import Solver
    W = workloads.parity_2d()
    u_star = pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, W.rhs[0], W.omega)
    S0 = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-12, max_iter=300, unpreconditioned=True)
    u0, it0, _, code0 = S0.solve(W.rhs)
    S1 = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-12, max_iter=100, prec="c64")
    u1, it1, rr1, code1 = S1.solve(W.rhs)
    S2 = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-12, max_iter=100)
    _, it2, _, _ = S2.solve(W.rhs)
    assert code0 == 0 and code1 == 0
    e0 = rel(cpu(u0).reshape(u_star.shape), u_star)
    e1 = rel(cpu(u1).reshape(u_star.shape), u_star)
    assert e0 <= 1e-9 and e1 <= 1e-9, (e0, e1)
    assert it0[0] > 2 * it2[0]
    assert it1[0] <= it2[0] + 3
    for s in (S0, S1, S2):
        s.close()


@pytest.mark.parametrize("case", ["3d_bisect", "3d_octree", "schrodinger", "schrodinger3d", "radix3"])
def test_other_shapes_match_dense(case):
    from paper_1409_0297_amd import Solver
    if case.startswith("3d"):
        W = workloads.small(12, 3, 3, waves=1.5, bumps=3)
        order = "bisect" if case == "3d_bisect" else "octree"
    elif case == "schrodinger":
        W = workloads.schrodinger_workload(32, 2, 4, 8)
        order = "octree"
    elif case == "schrodinger3d":
        W = workloads.schrodinger_workload(12, 3, 2, 3)
        order = "octree"
    else:
        W = workloads.small(48, 2, 6, waves=5.0, bumps=4)
        order = "octree"
    f = W.rhs[0]
    u_star = pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, f, W.omega, W.ell, W.energy)
    S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, ell=W.ell, energy=W.energy,
               order=order, tol=1e-12, max_iter=100)
    u, iters, relres, code = S.solve(f)
    S.close()
    assert code == 0
    e = rel(cpu(u).reshape(f.shape), u_star)
    assert e <= 1e-9, (case, e, iters)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_wide_level_step_pairs_match_oracle(prec):
    """Levels of more than 64 fronts take two elimination steps per trailing
    update (the second block's column and row are updated on their own
    first).  128^2 with 8-point boxes has 256 leaf fronts of 49 pivots: one
    pair per front, its second block ragged (32 + 17 pivots)."""
    from paper_1409_0297_amd import Solver
    W = workloads.small(128, 2, 8, waves=8.0, bumps=4)
    f = W.rhs[0]
    o = pipeline.setup_workload(W)
    u_o, _, _ = pipeline.solve(o, f, tol=1e-13)
    S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-12, max_iter=100, prec=prec)
    u, iters, relres, code = S.solve(f)
    S.close()
    assert code == 0
    e = rel(cpu(u).reshape(f.shape), np.asarray(u_o).reshape(f.shape))
    assert e <= 1e-9, (prec, e, iters)


def test_constant_medium_converges_in_one_iteration():
    from paper_1409_0297_amd import Solver
    n = 32
    c = np.full((n, n), 1.3)
    omega = 2 * math.pi * 5.1
    f = workloads.gaussian_sources(n, 2, 1, 1 / 16, 3)[0]
    S = Solver("helmholtz", n, 2, 8, c, omega=omega, tol=1e-10, max_iter=20)
    u, iters, relres, code = S.solve(f)
    S.close()
    assert iters[0] == 1 and code == 0
    k2 = spectral.k_squared(n, 2)
    u_exact = np.fft.ifftn(np.fft.fftn(f) / (4 * math.pi ** 2 * k2 - (omega / 1.3) ** 2))
    e = rel(cpu(u).reshape(f.shape), u_exact)
    assert e <= 1e-10, e


def test_shift_on_eigenvalue_is_perturbed_and_solution_unchanged():
    """A medium whose mean of omega^2/c^2 is exactly the eigenvalue 4 pi^2 64 of L:
    s must be perturbed (Section 2.2), while L - s + q, and so u, is unchanged."""
    from paper_1409_0297_amd import Solver
    n = 32
    x = workloads.grid_points(n, 2)
    omega = 2 * math.pi * 8
    w = omega ** 2 + 300.0 * (np.cos(2 * math.pi * x[..., 0]) + np.sin(2 * math.pi * 3 * x[..., 1]))
    c = omega / np.sqrt(w)
    S = Solver("helmholtz", n, 2, 8, c, omega=omega, tol=1e-12, max_iter=100)
    st = S.stats()
    assert st["shift_moves"] == 1
    s_o, q_o, moves = pipeline.coefficients("helmholtz", n, 2, c, omega=omega)
    assert moves == 1 and abs(st["s"] - s_o) <= 1e-9 * s_o
    f = workloads.gaussian_sources(n, 2, 1, 1 / 16, 4)[0]
    u, iters, _, code = S.solve(f)
    S.close()
    u_star = pipeline.dense_solution("helmholtz", n, 2, c, f, omega=omega)
    e = rel(cpu(u).reshape(f.shape), u_star)
    assert code == 0 and e <= 1e-9, (code, e, iters)


def test_not_converged_still_returns_iterate_and_residual():
    from paper_1409_0297_amd import SPP_NOT_CONVERGED, Solver
    W = workloads.parity_2d()
    S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-14, max_iter=2)
    u, iters, relres, code = S.solve(W.rhs)
    S.close()
    assert code == SPP_NOT_CONVERGED and iters == [2]
    assert 1e-14 < relres[0] < 1.0
    assert np.isfinite(cpu(u)).all()


def test_non_finite_coefficients_are_rejected():
    from paper_1409_0297_amd import SPP_EINVAL, Solver, SppError
    c = np.ones((32, 32))
    c[3, 4] = np.nan
    with pytest.raises(SppError) as e:
        Solver("helmholtz", 32, 2, 8, c, omega=20.0)
    assert e.value.code == SPP_EINVAL
    c[3, 4] = -1.0
    with pytest.raises(SppError):
        Solver("helmholtz", 32, 2, 8, c, omega=20.0)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_side_products_and_four_product_substitution_agree(prec):
    """Levels of few fronts solved with L21 L11^-1, U11^-1 U12 (one product per
    direction) or with L21, U12 kept (four products): the same preconditioner,
    so the same solution and iteration count within one."""
    from paper_1409_0297_amd import Solver
    W = workloads.helmholtz_workload("mid", 5, 128, 2, 16.0, 16, 0.05, 8)
    f = W.rhs[0]
    res = []
    for side in (True, False):
        S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-11, max_iter=100,
                   prec=prec, side_products=side)
        u, iters, relres, code = S.solve(f)
        res.append((cpu(u).reshape(f.shape), iters[0], relres[0], code))
        S.close()
    (u0, i0, r0, c0), (u1, i1, r1, c1) = res
    assert c0 == 0 and c1 == 0 and abs(i0 - i1) <= 1, (i0, i1)
    e = rel(u0, u1)
    assert e <= 1e-9, e


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_partial_and_block_local_pivoting_agree(prec):
    """Both pivoting rules factor the same P: same solution, iterations within one."""
    from paper_1409_0297_amd import Solver
    W = workloads.helmholtz_workload("mid", 5, 128, 2, 16.0, 16, 0.05, 8)
    f = W.rhs[0]
    res = []
    for pp in (False, True):
        S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-11, max_iter=100,
                   prec=prec, partial_pivoting=pp)
        u, iters, relres, code = S.solve(f)
        res.append((cpu(u).reshape(f.shape), iters[0], relres[0], code))
        S.close()
    (u0, i0, r0, c0), (u1, i1, r1, c1) = res
    assert c0 == 0 and c1 == 0 and abs(i0 - i1) <= 1, (i0, i1)
    e = rel(u0, u1)
    assert e <= 1e-9, e
