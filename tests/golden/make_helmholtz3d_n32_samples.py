"""Writes helmholtz3d_n32_u_samples.txt: the oracle's solutions of the 3D
Helmholtz workload at 32^3 (omega = 2 pi 4, 8 points per wavelength, 32
Gaussian bumps of width 0.06, b = 4, nested dissection by bisection) for two
right-hand sides, a Gaussian source and a unit grid delta at the centre, at
512 seeded grid points each (the same points for both), for parity checks of
the GPU path's streamed storage and blocked substitution of the root front.

Only the oracle and the seeded workload generators are used: oracle setup
with its own bisection elimination, FGMRES to a relative residual of 1e-13,
and the differential residual of each result as a check.

    python tests/golden/make_helmholtz3d_n32_samples.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import pipeline  # noqa: E402

SAMPLE_SEED = 32043
SAMPLES = 512


def main():
    W = workloads.helmholtz_3d(32, 4, nrhs=1)
    n = W.n
    rhs = [W.rhs[0], workloads.grid_delta(n, 3, (n // 2, n // 2, n // 2))]
    o = pipeline.setup_workload(W, ordering="bisect")
    rng = np.random.default_rng(SAMPLE_SEED)
    pts = rng.choice(n ** 3, size=SAMPLES, replace=False)
    out = os.path.join(HERE, "helmholtz3d_n32_u_samples.txt")
    with open(out, "w") as fh:
        fh.write(f"# oracle solutions of {W.name}: n={n} b={W.b} omega={W.omega!r} ordering=bisect tol=1e-13\n")
        fh.write("# rhs 0: the workload's Gaussian source; rhs 1: unit grid delta at the centre\n")
        for k, f in enumerate(rhs):
            u, iters, hist = pipeline.solve(o, f, tol=1e-13, max_iter=300)
            dres = pipeline.differential_residual(o, u, f)
            uf = u.reshape(-1)
            fh.write(f"# rhs {k}: iterations {iters}  final residual {hist[-1]:.3e}  differential residual "
                     f"{dres:.3e}  norm2 {float(np.linalg.norm(uf))!r}  norm_inf {float(np.abs(uf).max())!r}\n")
            print(k, iters, dres)
            for i in pts:
                fh.write(f"{k} {int(i)} {float(uf[i].real)!r} {float(uf[i].imag)!r}\n")
    print(out)


if __name__ == "__main__":
    main()
