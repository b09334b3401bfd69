"""The paper's Helmholtz examples rerun on the GPU path (Section 3.1,
Figures W21, W22, W31, W32): about 3 points per wavelength, the paper's
(N, b), a delta source at the domain centre, GMRES to 1e-6.

The paper does not give the amplitude or width of its Gaussians, so the
media here are of the same kind (c = 1 + 0.2 exp(-|x - x_i|^2 / (2 0.1^2)),
one Gaussian at the centre, or three at seeded points; in 3D on the middle
slice) and the check is qualitative: the iteration count is at most twice
the paper's n_p.  (Fewer is no defect of the method: at 384^2 the single
central Gaussian of this medium takes 7 iterations where the paper's took
28, whose medium evidently scattered more at that frequency.)  The 96^3 rows
are not run (a 53k-point root front).
"""
import math
import os

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_iterations_helmholtz.txt")


def rows():
    out = []
    with open(GOLD) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t, d, w, n, b, n_p = line.split()
                out.append((t, int(d), float(w), int(n), int(b), int(n_p)))
    return out


def medium(table, n, d):
    x = workloads.grid_points(n, d)
    if table in ("W21", "W31"):
        centres = np.full((1, d), 0.5)
    else:
        centres = np.random.default_rng(7).uniform(0, 1, (3, d))
        if d == 3:
            centres[:, 2] = 0.5
    c = np.ones((n,) * d)
    for ci in centres:
        c += 0.2 * np.exp(-workloads.periodic_sq_dist(x, ci) / (2 * 0.1 ** 2))
    return c


@pytest.mark.parametrize("table,d,waves,n,b,n_p", rows())
def test_paper_helmholtz_iteration_counts(table, d, waves, n, b, n_p):
    from paper_1409_0297_amd import Solver
    c = medium(table, n, d)
    S = Solver("helmholtz", n, d, b, c, omega=2 * math.pi * waves, prec="c128", tol=1e-6, max_iter=200)
    f = workloads.grid_delta(n, d, (n // 2,) * d)
    u, iters, relres, code = S.solve(f[None])
    S.close()
    print(f"{table} {n}^{d} b={b}: GPU {iters[0]} iterations, paper n_p = {n_p}")
    assert code == 0 and relres[0] <= 1e-6
    assert 1 <= iters[0] <= 2 * n_p, (iters[0], n_p)
