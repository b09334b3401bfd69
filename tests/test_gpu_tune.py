"""Autotuned launch parameters: same solution, a written tuning table."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autotune_keeps_the_solution_and_writes_its_table(tmp_path, monkeypatch):
    from paper_1409_0297_amd import Solver
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("SPP_TUNE_CACHE", str(path))
    W = workloads.helmholtz_workload("mid", 5, 128, 2, 16.0, 16, 0.05, 8, nrhs=2)
    A = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-11, max_iter=100, autotune=True)
    B = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-11, max_iter=100)
    ua, ia, ra, ca = A.solve(W.rhs)
    ub, ib, rb, cb = B.solve(W.rhs)
    A.close()
    B.close()
    torch.cuda.synchronize()
    assert ca == cb == 0
    assert all(abs(x - y) <= 1 for x, y in zip(ia, ib))
    d = float(torch.linalg.norm(ua - ub) / torch.linalg.norm(ub))
    assert d <= 1e-9, d
    text = path.read_text()
    assert "fft_lines@" in text and "gemv_chunks@" in text
    for line in text.splitlines():
        key, value = line.split()
        assert int(value) >= 1
