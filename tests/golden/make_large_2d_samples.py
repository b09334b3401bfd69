"""Writes large_2d_u_samples.txt: the oracle's solution of the 512^2 Helmholtz
workload (omega = 2 pi 64, 64 bumps, b = 16, one Gaussian source) at a seeded
sample of grid points, for parity checks of full-size GPU solves.

Only the oracle and the seeded workload generators are used: oracle setup,
FGMRES to a relative residual of 1e-13, then the differential residual of the
result as a check.  Takes about two minutes on eight cores.

    python tests/golden/make_large_2d_samples.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import pipeline  # noqa: E402

SAMPLE_SEED = 512064
SAMPLES = 1024


def main():
    W = workloads.large_2d()
    o = pipeline.setup_workload(W)
    u, iters, hist = pipeline.solve(o, W.rhs[0], tol=1e-13, max_iter=300)
    dres = pipeline.differential_residual(o, u, W.rhs[0])
    rng = np.random.default_rng(SAMPLE_SEED)
    flat = rng.choice(W.n * W.n, size=SAMPLES, replace=False)
    uf = u.reshape(-1)
    out = os.path.join(HERE, "large_2d_u_samples.txt")
    with open(out, "w") as fh:
        fh.write(f"# oracle solution of {W.name}: n={W.n} b={W.b} omega={W.omega!r} tol=1e-13\n")
        fh.write(f"# iterations {iters}  final residual {hist[-1]:.3e}  differential residual {dres:.3e}\n")
        fh.write(f"# norm2 {float(np.linalg.norm(uf))!r}  norm_inf {float(np.abs(uf).max())!r}\n")
        fh.write(f"# sample_seed {SAMPLE_SEED} samples {SAMPLES}\n")
        fh.write("# flat_index re im\n")
        for i in flat:
            fh.write(f"{int(i)} {float(uf[i].real)!r} {float(uf[i].imag)!r}\n")
    print(out, iters, dres)


if __name__ == "__main__":
    main()
