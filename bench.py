"""Throughput benchmark: solves/sec of the sparsifying-preconditioned GMRES solve.

One step = one full pass of the hot path on one right-hand side: setup
(shift and potential, Green kernel, stencils, assembly, nested-dissection
multifrontal factorisation) followed by the preconditioned FGMRES solve and
its true-residual check, on the 2D Helmholtz workload of a 512 x 512 grid,
omega = 2 pi 64 (8 points per wavelength), 64 Gaussian bumps, b = 16.
Inputs are generated once and are resident in GPU memory before timing.

Prints one JSON line (see the design doc for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", choices=["c128", "c64"], default="c128")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--cpu-baseline", choices=["sample", "off"], default="sample")
    ap.add_argument("--profile-only", action="store_true",
                    help="run the timed steps only (for rocprofv3), no baseline")
    return ap.parse_args()


def cpu_baseline(W, tol):
    """The oracle (plain FP64 numpy/scipy) on a bounded sample of the same workload.

    Sample: the full oracle setup (shift, stencils by explicit pseudoinverse,
    assembly of the sparse P, nested-dissection elimination) and two FGMRES
    iterations of the solve; the solve time is scaled to the iteration count
    the GPU needed.  Returns (solves_per_sec, threads, description).
    """
    import numpy as np  # noqa: F401
    from oracle import gmres, pipeline, spectral
    t0 = time.perf_counter()
    o = pipeline.setup_workload(W)
    t1 = time.perf_counter()
    g = pipeline.rhs_transform(o, W.rhs[0])
    A = lambda z: spectral.apply_integral(z, o.d, o.s, o.q)
    M = lambda r: pipeline.precondition(o, r)
    t2 = time.perf_counter()
    _, its, _ = gmres.fgmres(A, g, M, tol=1e-300, max_iter=2)
    t3 = time.perf_counter()
    return o, t1 - t0, (t3 - t2) / its, t2 - t1


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads
    import paper_1409_0297_amd as spp

    W = workloads.large_2d()
    dev = torch.device("cuda:0")
    coeff = torch.as_tensor(W.coeff, dtype=torch.float64, device=dev).contiguous()
    f = torch.as_tensor(W.rhs, dtype=torch.complex128, device=dev).contiguous()
    u = torch.empty_like(f)
    stream = torch.cuda.current_stream().cuda_stream
    pb = spp.binding.spp_problem(dim=W.d, n=W.n, b=W.b, kind=spp.SPP_HELMHOLTZ, omega=W.omega,
                                 ell=1.0, energy=0.0, coeff=coeff.data_ptr())
    op = spp.binding.spp_options(prec=spp.SPP_C128 if args.prec == "c128" else spp.SPP_C64_FRONTS,
                                 order=spp.SPP_ORDER_OCTREE, tol=args.tol, max_iter=200, flags=0)

    def step():
        h = spp.spp_setup(pb, op, stream)
        code, iters, relres = spp.spp_solve(h, f.data_ptr(), 1, u.data_ptr(), stream)
        st = spp.spp_stats(h)
        spp.spp_destroy(h)
        return iters[0], relres[0], st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec = []
    for _ in range(args.steps):
        rec.append(step())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    iters = [r[0] for r in rec]
    st = rec[-1][2]
    out = {
        "metric": "solves/sec to rel. err 1e-8 (mixed vs FP64), GMRES iters, HBM/MFMA % peak",
        "value": 1.0 / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "c128" else "c64-fronts/f64",
        "data": "synthetic",
        "config": {"workload": W.name, "grid": [W.n, W.n], "omega_over_2pi": 64, "b": W.b,
                   "bumps": 64, "nrhs": 1, "tol": args.tol, "ordering": "octree",
                   "fronts": args.prec},
        "gmres_iters": iters[-1],
        "relres": rec[-1][1],
        "t_setup_ms": st["t_setup_ms"],
        "t_factor_ms": st["t_factor_ms"],
        "t_solve_ms": st["t_solve_ms"],
        "factor_gb": st["factor_bytes"] / 1e9,
        "factor_gflop": st["factor_flops"] / 1e9,
        "roofline": None,
        "cpu_baseline": None,
    }
    if not args.profile_only and args.cpu_baseline == "sample":
        o, t_setup, t_iter, t_rhs = cpu_baseline(W, args.tol)
        t_cpu = t_setup + t_rhs + t_iter * iters[-1]
        out["cpu_baseline"] = {"value": 1.0 / t_cpu, "unit": "solves/s", "cores": os.cpu_count(),
                               "kind": "oracle",
                               "sample": f"full oracle setup ({t_setup:.1f} s) + 2 FGMRES iterations "
                                         f"({t_iter:.2f} s each) scaled to {iters[-1]} iterations"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
