"""Writes large_2d_delta_u_samples.txt: the oracle's solution of the 512^2
Helmholtz workload (omega = 2 pi 64, 64 bumps, b = 16) driven by a unit grid
delta at the centre (the source of the paper's examples, Section 3), at a
seeded sample of grid points: 512 uniform over the grid and 512 in the far
field (periodic distance at least 1/4 from the source, 16 or more
wavelengths away), for parity checks of full-size GPU solves of a field
that radiates through the whole domain.

Only the oracle and the seeded workload generators are used: oracle setup,
FGMRES to a relative residual of 1e-13, then the differential residual of
the result as a check.  Takes a few minutes on eight cores.

    python tests/golden/make_large_2d_delta_samples.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import pipeline  # noqa: E402

SAMPLE_SEED = 512065
UNIFORM = 512
FAR = 512
FAR_DISTANCE = 0.25


def main():
    W = workloads.large_2d_delta()
    o = pipeline.setup_workload(W)
    u, iters, hist = pipeline.solve(o, W.rhs[0], tol=1e-13, max_iter=400)
    dres = pipeline.differential_residual(o, u, W.rhs[0])
    n = W.n
    rng = np.random.default_rng(SAMPLE_SEED)
    uniform = rng.choice(n * n, size=UNIFORM, replace=False)
    x = workloads.grid_points(n, 2).reshape(-1, 2)
    dist2 = workloads.periodic_sq_dist(x, np.array([0.5, 0.5]))
    far_pool = np.setdiff1d(np.flatnonzero(dist2 >= FAR_DISTANCE ** 2), uniform)
    far = rng.choice(far_pool, size=FAR, replace=False)
    uf = u.reshape(-1)
    out = os.path.join(HERE, "large_2d_delta_u_samples.txt")
    with open(out, "w") as fh:
        fh.write(f"# oracle solution of {W.name}: n={n} b={W.b} omega={W.omega!r} tol=1e-13, "
                 f"unit grid delta at ({n // 2}, {n // 2})\n")
        fh.write(f"# iterations {iters}  final residual {hist[-1]:.3e}  differential residual {dres:.3e}\n")
        fh.write(f"# norm2 {float(np.linalg.norm(uf))!r}  norm_inf {float(np.abs(uf).max())!r}\n")
        fh.write(f"# sample_seed {SAMPLE_SEED} uniform {UNIFORM} far {FAR} (distance >= {FAR_DISTANCE})\n")
        fh.write("# flat_index region re im   (region 0: uniform, 1: far field)\n")
        for region, pts in ((0, uniform), (1, far)):
            for i in pts:
                fh.write(f"{int(i)} {region} {float(uf[i].real)!r} {float(uf[i].imag)!r}\n")
    print(out, iters, dres)


if __name__ == "__main__":
    main()
