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


def cpu_baseline(W, gpu_iters):
    """The oracle (plain FP64 numpy/scipy) on a bounded sample of the same workload.

    Sample: the complete oracle setup on the full 512^2 problem (shift,
    stencils by explicit SVD pseudoinverse, sparse P, nested-dissection
    elimination), the right-hand-side transform, and two FGMRES iterations of
    the preconditioned solve; the per-iteration time is scaled to the
    iteration count the GPU needed.  Returns a dict for the JSON line.
    """
    from oracle import gmres, pipeline, spectral
    t0 = time.perf_counter()
    o = pipeline.setup_workload(W)
    t1 = time.perf_counter()
    g = pipeline.rhs_transform(o, W.rhs[0])
    t2 = time.perf_counter()
    A = lambda z: spectral.apply_integral(z, o.d, o.s, o.q)
    M = lambda r: pipeline.precondition(o, r)
    _, its, _ = gmres.fgmres(A, g, M, tol=1e-300, max_iter=2)
    t3 = time.perf_counter()
    t_iter = (t3 - t2) / its
    t_total = (t1 - t0) + (t2 - t1) + t_iter * gpu_iters
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count()
    return {"value": 1.0 / t_total, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle setup on the full problem ({t1 - t0:.1f} s) + G f ({t2 - t1:.2f} s) + "
                      f"2 FGMRES iterations ({t_iter:.2f} s each) scaled to the GPU's {gpu_iters}"}


KCLASS_BOUND = {"fft": "hbm", "gemv": "hbm", "tri": "hbm", "qapply": "hbm", "gemm": "mfma"}


def roofline(timing, prec):
    """Dominant roofline-bound kernel class of the timed region."""
    best = None
    for name, t in timing.items():
        if name not in KCLASS_BOUND or t["launches"] == 0 or t["ms"] <= 0:
            continue
        if best is None or t["ms"] > timing[best]["ms"]:
            best = name
    if best is None:
        return None
    t = timing[best]
    sec = t["ms"] / 1e3
    if KCLASS_BOUND[best] == "hbm":
        achieved = t["bytes"] / sec / 1e9
        peak, unit = HBM_PEAK_GBS, "GB/s"
    else:
        achieved = t["flops"] / sec / 1e12
        peak, unit = (FP64_PEAK_TFS if prec == "c128" else FP32_PEAK_TFS), "TFLOP/s"
    return {"bound": KCLASS_BOUND[best], "kernel_class": best, "achieved": achieved, "peak": peak,
            "unit": unit, "frac": achieved / peak, "traffic": None,
            "avg_launch_us": 1e3 * t["ms"] / t["launches"], "launches": t["launches"],
            "algorithmic_per_launch": (t["bytes"] if KCLASS_BOUND[best] == "hbm" else t["flops"]) / t["launches"]}


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
    def options(flags):
        return spp.binding.spp_options(prec=spp.SPP_C128 if args.prec == "c128" else spp.SPP_C64_FRONTS,
                                       order=spp.SPP_ORDER_OCTREE, tol=args.tol, max_iter=200, flags=flags)

    def step(op):
        h = spp.spp_setup(pb, op, stream)
        code, iters, relres = spp.spp_solve(h, f.data_ptr(), 1, u.data_ptr(), stream)
        return h, iters[0], relres[0]

    plain = options(0)
    for _ in range(args.warmup):
        spp.spp_destroy(step(plain)[0])
    torch.cuda.synchronize()
    # Timed region: K full steps (setup + solve), inputs already in HBM.
    t0 = time.perf_counter()
    rec = [step(plain) for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = spp.spp_stats(rec[-1][0])
    iters = [r[1] for r in rec]
    for h, _, _ in rec:
        spp.spp_destroy(h)
    # Same K steps again with per-kernel-class HIP events on the launch stream.
    timing = None
    if not args.profile_only:
        timing = {k: {"ms": 0.0, "launches": 0, "bytes": 0.0, "flops": 0.0} for k in spp.KERNEL_CLASSES}
        timed = options(spp.SPP_F_TIMING)
        for _ in range(args.steps):
            h, _, _ = step(timed)
            for name, kc in spp.KERNEL_CLASSES.items():
                t = spp.spp_kernel_timing(h, kc)
                for key in timing[name]:
                    timing[name][key] += t[key]
            spp.spp_destroy(h)
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
        "relres": rec[-1][2],
        "t_setup_ms": st["t_setup_ms"],
        "t_factor_ms": st["t_factor_ms"],
        "t_solve_ms": st["t_solve_ms"],
        "factor_gb": st["factor_bytes"] / 1e9,
        "factor_gflop": st["factor_flops"] / 1e9,
        "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in timing.items()} if timing else None,
        "roofline": roofline(timing, args.prec) if timing else None,
        "cpu_baseline": None,
    }
    if not args.profile_only and args.cpu_baseline == "sample":
        print("bench: timing the CPU oracle baseline (about a minute)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(W, iters[-1])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
