"""Writes schrodinger_batch_u_samples.txt: the oracle's solutions of three
members of the batched 2D Schroedinger family (instances 0, 1 and 2: one each
of n = 128, 192 and 256, ell = n / 8, b = n / 16), for their first and last
Gaussian sources, at a seeded sample of grid points.  Used by the full-size
batch parity test.

Only the oracle and the seeded workload generators are used: oracle setup,
FGMRES to a relative residual of 1e-13, then the differential residual of
each result as a check.  Takes about half a minute on eight cores.

    python tests/golden/make_schrodinger_batch_samples.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import pipeline  # noqa: E402

SAMPLE_SEED = 4016
SAMPLES = 128
INSTANCES = (0, 1, 2)
SOURCES = (0, 15)


def main():
    batch = workloads.schrodinger_batch()
    out = os.path.join(HERE, "schrodinger_batch_u_samples.txt")
    rng = np.random.default_rng(SAMPLE_SEED)
    with open(out, "w") as fh:
        fh.write("# oracle solutions of the batched 2D Schroedinger family (workloads.schrodinger_batch), tol=1e-13\n")
        fh.write(f"# sample_seed {SAMPLE_SEED} samples {SAMPLES} per (instance, source)\n")
        for i in INSTANCES:
            W = batch[i]
            o = pipeline.setup_workload(W)
            for r in SOURCES:
                u, iters, hist = pipeline.solve(o, W.rhs[r], tol=1e-13, max_iter=300)
                dres = pipeline.differential_residual(o, u, W.rhs[r])
                uf = u.reshape(-1)
                fh.write(f"# instance {i} {W.name} b={W.b} energy={W.energy!r} source {r}: iterations {iters} "
                         f"final residual {hist[-1]:.3e} differential residual {dres:.3e} "
                         f"norm2 {float(np.linalg.norm(uf))!r}\n")
                flat = rng.choice(W.n * W.n, size=SAMPLES, replace=False)
                for j in flat:
                    fh.write(f"{i} {r} {int(j)} {float(uf[j].real)!r} {float(uf[j].imag)!r}\n")
                print(i, r, W.name, iters, dres, flush=True)
    print(out)


if __name__ == "__main__":
    main()
