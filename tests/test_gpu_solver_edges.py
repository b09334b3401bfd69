"""Edges of the solver boundary, through the C ABI on the GPU.

- FGMRES(restart): cycles restart from the true residual (Section 3 solves
  to a relative tolerance; the restarted method reaches the same u*).
- spp_solve_batch: per-problem right-hand-side counts, including none.
- The allocator hook: the front arena comes from PyTorch's allocator and the
  results are the ones the library's own allocation gives.
- Pivot statistics of the block-local pivoting LU (growth, smallest pivot
  against the front's largest entry).
"""
import numpy as np
import pytest

import workloads
from oracle import pipeline

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_restarted_fgmres_reaches_the_dense_solution(prec):
    from paper_1409_0297_amd import Solver
    W = workloads.parity_2d(nrhs=2)
    u_star = [pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, W.rhs[i], W.omega) for i in range(2)]
    S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-12, max_iter=120,
               restart=4)
    u, iters, relres, code = S.solve(W.rhs)
    st = S.stats()
    S.close()
    u = cpu(u).reshape(W.rhs.shape)
    assert code == 0, (code, iters, relres)
    # each cycle holds at most 4 Krylov vectors, so more than one cycle ran
    assert st["last_cycles"] >= 2 and max(iters) > 4, (st["last_cycles"], iters)
    for i in range(2):
        assert relres[i] <= 1e-12
        e = rel(u[i], u_star[i])
        assert e <= 1e-9, (i, e)
    # one cycle without restarts: fewer or equal iterations, the same solution
    S1 = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-12, max_iter=120)
    u1, it1, _, code1 = S1.solve(W.rhs)
    assert S1.stats()["last_cycles"] == 1
    S1.close()
    assert code1 == 0 and max(it1) <= max(iters)
    assert rel(cpu(u1).reshape(W.rhs.shape), u) <= 1e-9


def test_restart_budget_exhausted_reports_not_converged():
    from paper_1409_0297_amd import SPP_NOT_CONVERGED, Solver
    W = workloads.parity_2d(nrhs=1)
    S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-14, max_iter=6, restart=3,
               unpreconditioned=True)
    u, iters, relres, code = S.solve(W.rhs)
    st = S.stats()
    S.close()
    assert code == SPP_NOT_CONVERGED
    assert iters[0] == 6 and st["last_cycles"] == 2
    # relres is the true residual of the returned u
    assert 1e-14 < relres[0] < 1.0


def test_solve_batch_with_per_problem_counts():
    from paper_1409_0297_amd import BatchSolver, Solver
    Ws = [workloads.small(32, 2, 8, waves=4.0, bumps=3, nrhs=3, instance=1),
          workloads.schrodinger_workload(32, 2, 4, 8, nrhs=1),
          workloads.small(48, 2, 6, waves=5.0, bumps=4, nrhs=2)]
    probs = [dict(kind=W.kind, n=W.n, d=W.d, b=W.b, coeff=W.coeff, omega=W.omega, ell=W.ell, energy=W.energy)
             for W in Ws]
    B = BatchSolver(probs, tol=1e-12, max_iter=100)
    fs = [Ws[0].rhs[:3].reshape(3, -1), None, Ws[2].rhs[:2].reshape(2, -1)]
    us, iters, relres, code = B.solve_each(fs)
    B.close()
    assert code == 0
    assert us[1] is None and iters[1] == [] and len(iters[0]) == 3 and len(iters[2]) == 2
    for i in (0, 2):
        W = Ws[i]
        u = cpu(us[i])
        for r in range(len(iters[i])):
            u_star = pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, W.rhs[r], W.omega, W.ell, W.energy)
            assert rel(u[r].reshape(W.rhs[r].shape), u_star) <= 1e-9, (i, r)
            assert relres[i][r] <= 1e-12


def test_zero_right_hand_side_gives_zero():
    from paper_1409_0297_amd import Solver
    W = workloads.parity_2d(nrhs=2)
    f = W.rhs.copy()
    f[1] = 0
    S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-12, max_iter=100)
    u, iters, relres, code = S.solve(f)
    S.close()
    u = cpu(u)
    assert code == 0 and iters[1] == 0 and relres[1] == 0.0
    assert not np.any(u[1])
    u_star = pipeline.dense_solution(W.kind, W.n, W.d, W.coeff, W.rhs[0], W.omega)
    assert rel(u[0].reshape(u_star.shape), u_star) <= 1e-9


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_allocator_hook_serves_the_arena(prec):
    from paper_1409_0297_amd import Solver, TorchAllocator
    W = workloads.parity_2d(nrhs=1)
    A = TorchAllocator()
    S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-12, max_iter=100, allocator=A)
    u, iters, relres, code = S.solve(W.rhs)
    st = S.stats()
    S.close()
    assert A.served >= 1 and A.freed == A.served
    # the front arena: sum over fronts of F^2 entries
    assert A.bytes >= st["factor_entries"] * (16 if prec == "c128" else 8)
    S0 = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-12, max_iter=100)
    u0, it0, _, code0 = S0.solve(W.rhs)
    S0.close()
    assert code == 0 and code0 == 0 and iters == it0
    # the same kernels on the same data: identical solutions
    assert np.array_equal(cpu(u), cpu(u0))


@pytest.mark.parametrize("prec,eps", [("c128", 2.2e-16), ("c64", 1.19e-7)])
def test_pivot_statistics(prec, eps):
    from paper_1409_0297_amd import Solver
    for W in (workloads.parity_2d(), workloads.small(24, 3, 6, waves=2.0, bumps=3)):
        S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-10, max_iter=60)
        st = S.stats()
        S.close()
        assert st["breakdown_front"] == -1
        # every pivot well above the breakdown threshold 1e3 eps64 ||front||;
        # the count of pivots below 1e3 eps of the front precision is reported
        assert 1e3 * 2.2e-16 < st["min_pivot"] <= 1.0, st["min_pivot"]
        assert (st["small_pivots"] > 0) == (st["min_pivot"] < 1e3 * eps)
        assert 0.0 < st["pivot_growth"] < 1e6, st["pivot_growth"]
        assert st["device_bytes"] > st["factor_entries"] * (16 if prec == "c128" else 8)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_factor_used_at_once_from_another_stream(prec):
    """The explicit inverses of the levels solved by products run on the
    library's second stream and may still run when setup returns.  A
    preconditioner apply and a solve issued at once, on a stream other than
    the setup's, wait for them: their results equal, bit for bit, those of
    the same calls made after the device has drained."""
    from paper_1409_0297_amd import Solver
    W = workloads.small(256, 2, 16, 16.0, bumps=8)
    rng = np.random.default_rng(41)
    r = torch.as_tensor(rng.standard_normal((1, 256 * 256)) + 1j * rng.standard_normal((1, 256 * 256)),
                        dtype=torch.complex128, device="cuda")
    f = torch.as_tensor(W.rhs.reshape(1, -1), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    s_setup, s_use = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s_setup):
        S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-10, max_iter=100)
    with torch.cuda.stream(s_use):
        z_now = S.apply_precond(r)
    torch.cuda.synchronize()
    z_later = S.apply_precond(r)
    torch.cuda.synchronize()
    assert torch.equal(z_now, z_later)
    S.close()
    with torch.cuda.stream(s_setup):
        S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, prec=prec, tol=1e-10, max_iter=100)
    with torch.cuda.stream(s_use):
        u_now, it_now, _, code_now = S.solve(f)
    torch.cuda.synchronize()
    u_later, it_later, _, code_later = S.solve(f)
    torch.cuda.synchronize()
    S.close()
    assert code_now == 0 and code_later == 0 and it_now == it_later
    assert torch.equal(u_now, u_later)
