"""Throughput benchmark: solves/sec of the sparsifying-preconditioned GMRES solve.

One step = one full pass of the hot path on one right-hand side: setup
(shift and potential, Green kernel, stencils, assembly, nested-dissection
multifrontal factorisation) followed by the preconditioned FGMRES solve and
its true-residual check, on the 2D Helmholtz workload of a 512 x 512 grid,
omega = 2 pi 64 (8 points per wavelength), 64 Gaussian bumps, b = 16, driven
by a unit grid delta at the centre (the paper's source: the field radiates
through the whole domain), FGMRES to 1e-10 (the tolerance at which the
solution matches the FP64 oracle to 1e-8 norm-wise and element-wise, checked
by tests/test_gpu_full_size.py).  Inputs are generated once and resident in
GPU memory before timing.

The headline is the mixed-precision path (complex64 fronts, FP64 operator,
residuals and GMRES); the same K steps are also timed with complex128 fronts
and reported beside it, and two keyed records follow: the same medium with
the Gaussian source (a field that stays local), and the batched 2D
Schroedinger family (48 problems of 128^2-256^2, 16 sources each).  Prints
one JSON line.
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
    ap.add_argument("--prec", choices=["c64", "c128"], default="c64",
                    help="front precision of the headline value")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--order", choices=["octree", "bisect"], default="octree",
                    help="nested-dissection ordering above the leaves of the 512^2 headline (the same P^-1)")
    ap.add_argument("--graphs", action="store_true", help="replay FGMRES iterations from a HIP graph")
    ap.add_argument("--persistent", action="store_true",
                    help="cooperative launch for runs of small-front substitution levels")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="skip tuning launch parameters in the warm-up step (SPP_F_AUTOTUNE)")
    ap.add_argument("--cpu-baseline", choices=["full", "sample", "off"], default="full",
                    help="full: the oracle timed on the benchmark workload itself (setup + solve); "
                         "sample: the scaled 256^2 estimate only")
    ap.add_argument("--records", choices=["all", "none", "maxwell"], default="all",
                    help="keyed records beside the headline (Gaussian source, batched Schroedinger, Maxwell "
                         "512^2, 3D 128^3); maxwell: that record only")
    ap.add_argument("--profile-only", action="store_true",
                    help="run the timed steps only (for rocprofv3): no timing pass, no other precision, no baseline")
    ap.add_argument("--workload", choices=["large2d", "schrodinger-batch", "helmholtz3d"], default="large2d",
                    help="large2d: the 512^2 Helmholtz solve (default, with roofline and CPU baseline); "
                         "schrodinger-batch: the 48-instance batched Schroedinger family, 16 sources each; "
                         "helmholtz3d: one step of the 128^3 3D configuration (for profiling)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the warm-up steps, copy a MIB-MiB device buffer once (a plain copy kernel of known "
                         "size, to scale hardware byte counters)")
    return ap.parse_args()


def cpu_baseline(gpu_iters, stats512, stats256):
    """The oracle (plain FP64 numpy/scipy) timed on a bounded sample.

    Sample: the complete oracle (shift, explicit-SVD stencils, sparse P,
    nested-dissection elimination, G f, two FGMRES iterations) on the 256^2
    member of the same family (omega = 2 pi 32, so the same 8 points per
    wavelength and the same b = 16).  Each component is scaled to 512^2 by
    what drives its cost: N for coefficients, stencils (their least-squares
    matrices have N - |gamma| columns), assembly and G f; the factorisation
    flops of the two nested-dissection plans for the elimination; the factor
    entries for an FGMRES iteration, times the GPU's iteration count.
    """
    import workloads
    from oracle import gmres, nested, pipeline, spectral, stencil
    W = workloads.helmholtz_workload("helmholtz2d_n256_w32", 2, 256, 2, 32.0, 64, 0.05, 16)
    t = {}
    t0 = time.perf_counter()
    s, q, _ = pipeline.coefficients(W.kind, W.n, W.d, W.coeff, W.omega)
    t["coefficients"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    st = stencil.Stencils(W.n, W.d, W.b, s)
    t["stencils"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    P = st.P_matrix(q)
    t["assembly"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    fac = nested.NDFactor(P, nested.nd_levels(W.n, W.d, W.b, "octree"))
    t["factorisation"] = time.perf_counter() - t0
    o = pipeline.OracleSetup(n=W.n, d=W.d, b=W.b, s=s, q=q, shift_moves=0, stencils=st, P=P, factor=fac)
    t0 = time.perf_counter()
    g = pipeline.rhs_transform(o, W.rhs[0])
    t["rhs"] = time.perf_counter() - t0
    A = lambda z: spectral.apply_integral(z, o.d, o.s, o.q)
    M = lambda r: pipeline.precondition(o, r)
    t0 = time.perf_counter()
    _, its, _ = gmres.fgmres(A, g, M, tol=1e-300, max_iter=2)
    t["iteration"] = (time.perf_counter() - t0) / its
    rN = 4.0
    rF = stats512["factor_flops"] / stats256["factor_flops"]
    rE = stats512["factor_entries"] / stats256["factor_entries"]
    est = ((t["coefficients"] + t["stencils"] + t["assembly"] + t["rhs"]) * rN + t["factorisation"] * rF
           + t["iteration"] * rE * gpu_iters)
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count()
    sample = ("oracle on the 256^2 member of the workload family (omega = 2 pi 32, b = 16): "
              + ", ".join(f"{k} {v:.2f} s" for k, v in t.items())
              + f"; scaled to 512^2 by N (x{rN:.0f}), factorisation flops (x{rF:.2f}) and factor entries"
              f" (x{rE:.2f}) times {gpu_iters} iterations")
    return {"value": 1.0 / est, "unit": "solves/s", "cores": threads, "kind": "oracle", "sample": sample,
            "est_seconds_per_solve": est}


def cpu_baseline_full(W, tol):
    """The oracle (plain FP64 numpy/scipy) timed on the benchmark workload
    itself: setup (shift, explicit-SVD stencils, sparse P, nested-dissection
    elimination with LAPACK fronts) plus the preconditioned FGMRES solve to
    the benchmark's tolerance, one right-hand side."""
    from oracle import pipeline
    t0 = time.perf_counter()
    o = pipeline.setup_workload(W)
    t1 = time.perf_counter()
    u, its, hist = pipeline.solve(o, W.rhs[0], tol=tol, max_iter=300)
    t2 = time.perf_counter()
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count()
    return {"value": 1.0 / (t2 - t0), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"the complete oracle on {W.name} (n = {W.n}, b = {W.b}): setup {t1 - t0:.1f} s, "
                       f"FGMRES to {tol:g} in {its} iterations {t2 - t1:.1f} s; one run"),
            "seconds_per_solve": t2 - t0, "oracle_iters": its}


KCLASS_BOUND = {"fft": "hbm", "gemv": "hbm", "tri": "hbm", "qapply": "hbm", "gemm": "mfma", "inv": "mfma",
                "solve_blk": "hbm"}


def measured_traffic(kernel_class, prec):
    """HBM bytes per launch of the dominant kernel class from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel
    of known size), or None when there is none for this class or the kernel
    source has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"large2d_{prec}_{kernel_class}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    fields = dict(re.findall(r"^(\w+): (\S+)$", text, flags=re.M))
    src = os.path.join(ROOT, "paper_1409_0297_amd", "csrc", "mf.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("kernel_class") != kernel_class or fields.get("source_sha256") != sha:
        return None
    return float(fields["traffic_per_launch_bytes"])


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
            "unit": unit, "frac": achieved / peak, "traffic": measured_traffic(best, prec),
            "avg_launch_us": 1e3 * t["ms"] / t["launches"], "launches": t["launches"],
            "algorithmic_per_launch": (t["bytes"] if KCLASS_BOUND[best] == "hbm" else t["flops"]) / t["launches"]}


def batch_record(args, steps, warmup, precs):
    """Solves per second of the batched 2D Schroedinger family: 48 instances
    (16 each of 128^2, 192^2, 256^2) with 16 Gaussian sources each, set up
    and solved as one batch; a step is one spp_setup_batch + one spp_solve of
    all 768 right-hand sides, inputs resident in HBM."""
    import torch

    import workloads
    import paper_1409_0297_amd as spp

    nrhs = 16
    Ws = workloads.schrodinger_batch(nrhs=nrhs)
    dev = torch.device("cuda:0")
    coeffs = [torch.as_tensor(W.coeff, dtype=torch.float64, device=dev).contiguous().reshape(-1) for W in Ws]
    pbs = [spp.binding.spp_problem(dim=W.d, n=W.n, b=W.b, kind=spp.SPP_SCHRODINGER, omega=0.0, ell=W.ell,
                                   energy=W.energy, coeff=c.data_ptr()) for W, c in zip(Ws, coeffs)]
    f = torch.cat([torch.as_tensor(W.rhs.reshape(nrhs, -1), dtype=torch.complex128, device=dev).reshape(-1)
                   for W in Ws]).contiguous()
    u = torch.empty_like(f)
    stream = torch.cuda.current_stream().cuda_stream
    flags = ((spp.SPP_F_GRAPHS if args.graphs else 0) | (spp.SPP_F_PERSISTENT if args.persistent else 0)
             | (spp.SPP_F_AUTOTUNE if args.autotune else 0))

    def timed_run(prec):
        op = spp.binding.spp_options(prec=spp.SPP_C128 if prec == "c128" else spp.SPP_C64_FRONTS,
                                     order=spp.SPP_ORDER_OCTREE, tol=args.tol, max_iter=40, flags=flags)

        def step():
            h = spp.spp_setup_batch(pbs, op, stream)
            code, iters, relres = spp.spp_solve(h, f.data_ptr(), nrhs, u.data_ptr(), stream, nproblems=len(Ws))
            return h, code, iters, relres
        for _ in range(warmup):
            spp.spp_destroy(step()[0])
        # Each step's factor (about 45 GB with the Krylov basis) is released
        # before the next, outside the timed intervals.
        dt = 0.0
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h, code, iters, relres = step()
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            st = spp.spp_stats(h)
            spp.spp_destroy(h)
        return dt / steps, st, code, [int(min(iters)), int(max(iters))], float(max(relres))

    solves = len(Ws) * nrhs
    rec = {"workload": "schrodinger2d_batch48_n128-256_l16-32", "instances": len(Ws), "nrhs": nrhs,
           "grids": [128, 192, 256], "b": [8, 12, 16], "tol": args.tol, "steps": steps, "warmup": warmup}
    for i, prec in enumerate(precs):
        dt, st, code, it, rr = timed_run(prec)
        r = {"fronts": prec, "value": solves / dt, "unit": "solves/s", "ms_per_step": dt * 1e3, "code": code,
             "gmres_iters": it, "relres_max": rr, "t_setup_ms": st["t_setup_ms"], "t_solve_ms": st["t_solve_ms"],
             "factor_gb": st["factor_bytes"] / 1e9}
        if i == 0:
            rec.update(r)
        else:
            rec["other_precision"] = r
    return rec


def record_3d(args):
    """One timed step of the 3D Helmholtz configuration: 128^3, omega = 2 pi 16
    (8 points per wavelength), 32 Gaussian bumps of width 0.06, b = 8 (8^3
    leaf boxes), bisection ordering, complex64 fronts in streamed storage,
    FP64 FGMRES; setup + solve of 4 Gaussian sources to the bench tolerance.
    The step runs once, without a warm-up (it holds about 230 GB while it
    runs); its time includes building the host plan of this geometry."""
    import torch

    import workloads
    import paper_1409_0297_amd as spp

    W = workloads.helmholtz_3d(128, 8, nrhs=4)
    dev = torch.device("cuda:0")
    coeff = torch.as_tensor(W.coeff, dtype=torch.float64, device=dev).contiguous()
    f = torch.as_tensor(W.rhs.reshape(4, -1), dtype=torch.complex128, device=dev).contiguous()
    u = torch.empty_like(f)
    stream = torch.cuda.current_stream().cuda_stream
    pb = spp.binding.spp_problem(dim=3, n=W.n, b=W.b, kind=spp.SPP_HELMHOLTZ, omega=W.omega, ell=1.0, energy=0.0,
                                 coeff=coeff.data_ptr())
    op = spp.binding.spp_options(prec=spp.SPP_C64_FRONTS, order=spp.SPP_ORDER_BISECT, tol=args.tol, max_iter=80,
                                 flags=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = spp.spp_setup(pb, op, stream)
    code, iters, relres = spp.spp_solve(h, f.data_ptr(), 4, u.data_ptr(), stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = spp.spp_stats(h)
    spp.spp_destroy(h)
    del u, f, coeff
    torch.cuda.empty_cache()
    return {"workload": W.name, "grid": [W.n] * 3, "omega_over_2pi": 16, "b": W.b, "bumps": 32, "nrhs": 4,
            "ordering": "bisect", "fronts": "c64", "storage": "streamed" if st["storage"] else "resident",
            "tol": args.tol, "steps": 1, "warmup": 0, "value": 4.0 / dt, "unit": "solves/s", "s_per_step": dt,
            "code": code, "gmres_iters": iters, "relres_max": max(relres), "t_setup_ms": st["t_setup_ms"],
            "t_factor_ms": st["t_factor_ms"], "t_solve_ms": st["t_solve_ms"], "factor_gb": st["factor_bytes"] / 1e9,
            "factor_tflop": st["factor_flops"] / 1e12,
            "factor_tflops_achieved": st["factor_flops"] / (st["t_factor_ms"] / 1e3) / 1e12,
            "max_front": st["max_front"]}


def record_maxwell(args, steps=3, warmup=1):
    """The Maxwell (curl-curl) extension on the headline's grid: the 2D
    in-plane field on 512^2, omega = 2 pi 32 (16 points per wavelength: at
    the headline's 8 the iterations of this extension outgrow 400),
    permittivity 1 / c^2 of the headline's 64-bump medium family, b = 16,
    one vector source (two independent Gaussians of width 1/32), complex128
    fronts (complex64 fronts lose the solve at this size), FP64 FGMRES to
    the bench tolerance; one step = setup + solve."""
    import torch

    import workloads
    import paper_1409_0297_amd as spp

    W = workloads.maxwell_workload(512, 2, 16, 32.0, bumps=64, width=0.05, nrhs=1, config=2)
    dev = torch.device("cuda:0")
    coeff = torch.as_tensor(W.coeff, dtype=torch.float64, device=dev).contiguous()
    f = torch.as_tensor(W.rhs.reshape(1, -1), dtype=torch.complex128, device=dev).contiguous()
    u = torch.empty_like(f)
    stream = torch.cuda.current_stream().cuda_stream
    pb = spp.binding.spp_problem(dim=2, n=W.n, b=W.b, kind=spp.SPP_MAXWELL, omega=W.omega, ell=1.0, energy=0.0,
                                 coeff=coeff.data_ptr())
    op = spp.binding.spp_options(prec=spp.SPP_C128, order=spp.SPP_ORDER_OCTREE, tol=args.tol, max_iter=400,
                                 flags=spp.SPP_F_AUTOTUNE if args.autotune else 0)
    times, last = [], None
    for k in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = spp.spp_setup(pb, op, stream)
        code, iters, relres = spp.spp_solve(h, f.data_ptr(), 1, u.data_ptr(), stream)
        torch.cuda.synchronize()
        if k >= warmup:
            times.append(time.perf_counter() - t0)
        if last is not None:
            spp.spp_destroy(last)
        last = h
    st = spp.spp_stats(last)
    spp.spp_destroy(last)
    dt = sum(times) / len(times)
    del u, f, coeff
    torch.cuda.empty_cache()
    return {"workload": "maxwell2d_n512_w32", "grid": [512, 512], "components": 2, "omega_over_2pi": 32,
            "b": 16, "bumps": 64, "nrhs": 1, "fronts": "c128", "tol": args.tol, "steps": steps, "warmup": warmup,
            "value": 1.0 / dt, "unit": "solves/s", "ms_per_step": dt * 1e3, "code": code, "gmres_iters": iters,
            "relres": relres, "t_setup_ms": st["t_setup_ms"], "t_factor_ms": st["t_factor_ms"],
            "t_solve_ms": st["t_solve_ms"], "factor_gb": st["factor_bytes"] / 1e9,
            "factor_gflop": st["factor_flops"] / 1e9, "max_front": st["max_front"]}


def batch_main(args):
    rec = batch_record(args, args.steps, args.warmup, [args.prec, "c128" if args.prec == "c64" else "c64"])
    out = {
        "metric": "solves/sec to rel. err 1e-8 (mixed vs FP64), GMRES iters, HBM/MFMA % peak",
        "value": rec["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64-fronts/f64" if args.prec == "c64" else "f64", "data": "synthetic",
        "config": {"workload": rec["workload"], "instances": rec["instances"], "nrhs": rec["nrhs"],
                   "grids": rec["grids"], "b": rec["b"], "tol": args.tol, "fronts": args.prec, "outer": "f64",
                   "graphs": args.graphs, "persistent": args.persistent, "autotune": args.autotune},
        "code": rec["code"], "gmres_iters": rec["gmres_iters"], "relres_max": rec["relres_max"],
        "t_setup_ms": rec["t_setup_ms"], "t_solve_ms": rec["t_solve_ms"], "factor_gb": rec["factor_gb"],
        "other_precision": rec.get("other_precision"),
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this library runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "schrodinger-batch":
        return batch_main(args)
    if args.workload == "helmholtz3d":
        rec = record_3d(args)
        print(json.dumps({"metric": "solves/sec to rel. err 1e-8 (mixed vs FP64), GMRES iters, HBM/MFMA % peak",
                          "value": rec["value"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
                          "ms_per_step": rec["s_per_step"] * 1e3, "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "c64-fronts/f64", "data": "synthetic",
                          "config": {"workload": rec["workload"]}, "record": rec, "roofline": None,
                          "cpu_baseline": None}), flush=True)
        return
    import torch

    import workloads
    import paper_1409_0297_amd as spp

    W = workloads.large_2d_delta()
    dev = torch.device("cuda:0")
    coeff = torch.as_tensor(W.coeff, dtype=torch.float64, device=dev).contiguous()
    f = torch.as_tensor(W.rhs, dtype=torch.complex128, device=dev).contiguous()
    f_gauss = torch.as_tensor(workloads.large_2d().rhs, dtype=torch.complex128, device=dev).contiguous()
    u = torch.empty_like(f)
    stream = torch.cuda.current_stream().cuda_stream
    pb = spp.binding.spp_problem(dim=W.d, n=W.n, b=W.b, kind=spp.SPP_HELMHOLTZ, omega=W.omega,
                                 ell=1.0, energy=0.0, coeff=coeff.data_ptr())
    base_flags = ((spp.SPP_F_GRAPHS if args.graphs else 0) | (spp.SPP_F_PERSISTENT if args.persistent else 0)
                  | (spp.SPP_F_AUTOTUNE if args.autotune else 0))

    def options(prec, flags):
        return spp.binding.spp_options(prec=spp.SPP_C128 if prec == "c128" else spp.SPP_C64_FRONTS,
                                       order=spp.SPP_ORDER_OCTREE if args.order == "octree" else spp.SPP_ORDER_BISECT,
                                       tol=args.tol, max_iter=200, flags=flags)

    def step(op, rhs):
        h = spp.spp_setup(pb, op, stream)
        code, iters, relres = spp.spp_solve(h, rhs.data_ptr(), 1, u.data_ptr(), stream)
        return h, iters[0], relres[0]

    def calibration_copy():
        # A device-to-device copy of known size just before the timed steps
        # (after the warm-up and its tuning), so that counter runs can scale
        # their readings and take the step's dispatches as those after it.
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"bench: copied {nbytes} bytes device to device", file=sys.stderr, flush=True)
        del src, dst

    def timed_run(prec, rhs, steps, warmup, calibrate=False):
        plain = options(prec, base_flags)
        for _ in range(warmup):
            spp.spp_destroy(step(plain, rhs)[0])
        torch.cuda.synchronize()
        if calibrate:
            calibration_copy()
        # Timed region: K full steps (setup, solve, release of the factor, whose
        # device buffers the next setup takes back from the library's cache),
        # inputs already in HBM.
        t0 = time.perf_counter()
        for k in range(steps):
            h, iters, relres = step(plain, rhs)
            if k == steps - 1:
                st = spp.spp_stats(h)
            spp.spp_destroy(h)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        return dt, st, iters, relres

    dt, st, iters, relres = timed_run(args.prec, f, args.steps, args.warmup, calibrate=args.calibrate_copy > 0)
    # The same K steps again with per-kernel-class HIP events on the launch stream.
    timing = None
    other = None
    records = {}
    if not args.profile_only:
        timing = {k: {"ms": 0.0, "launches": 0, "bytes": 0.0, "flops": 0.0} for k in spp.KERNEL_CLASSES}
        timed = options(args.prec, spp.SPP_F_TIMING | (base_flags & (spp.SPP_F_PERSISTENT | spp.SPP_F_AUTOTUNE)))
        for _ in range(args.steps):
            h, _, _ = step(timed, f)
            for name, kc in spp.KERNEL_CLASSES.items():
                t = spp.spp_kernel_timing(h, kc)
                for key in timing[name]:
                    timing[name][key] += t[key]
            spp.spp_destroy(h)
        oprec = "c128" if args.prec == "c64" else "c64"
        odt, ost, oit, orr = timed_run(oprec, f, args.steps, args.warmup)
        other = {"fronts": oprec, "value": 1.0 / odt, "ms_per_step": odt * 1e3, "gmres_iters": oit,
                 "relres": orr, "t_setup_ms": ost["t_setup_ms"], "t_solve_ms": ost["t_solve_ms"]}
        if args.records == "all":
            gdt, gst, git, grr = timed_run(args.prec, f_gauss, args.steps, 1)
            records["gaussian_source"] = {
                "workload": "helmholtz2d_n512_w64", "rhs": "Gaussian of width 1/32 (non-radiating)",
                "fronts": args.prec, "value": 1.0 / gdt, "unit": "solves/s", "ms_per_step": gdt * 1e3,
                "gmres_iters": git, "relres": grr, "t_setup_ms": gst["t_setup_ms"], "t_solve_ms": gst["t_solve_ms"],
                "steps": args.steps, "warmup": 1}
            print("bench: timing the batched Schroedinger family", file=sys.stderr, flush=True)
            records["schrodinger_batch"] = batch_record(args, 3, 1, [args.prec])
            print("bench: timing the 512^2 Maxwell (curl-curl) solve", file=sys.stderr, flush=True)
            records["maxwell2d_512"] = record_maxwell(args)
            print("bench: timing one step of the 3D 128^3 configuration (about a minute)", file=sys.stderr,
                  flush=True)
            records["helmholtz3d_128"] = record_3d(args)
        elif args.records == "maxwell":
            records["maxwell2d_512"] = record_maxwell(args)
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
        "dtype": "c64-fronts/f64" if args.prec == "c64" else "f64",
        "data": "synthetic",
        "config": {"workload": W.name, "grid": [W.n, W.n], "omega_over_2pi": 64, "b": W.b,
                   "bumps": 64, "rhs": "unit grid delta at the centre", "nrhs": 1, "tol": args.tol,
                   "ordering": args.order, "fronts": args.prec, "outer": "f64", "graphs": args.graphs,
                   "persistent": args.persistent, "autotune": args.autotune},
        "gmres_iters": iters,
        "relres": relres,
        "t_setup_ms": st["t_setup_ms"],
        "t_factor_ms": st["t_factor_ms"],
        "t_solve_ms": st["t_solve_ms"],
        "factor_gb": st["factor_bytes"] / 1e9,
        "factor_gflop": st["factor_flops"] / 1e9,
        "pivot_growth": st["pivot_growth"],
        "min_pivot": st["min_pivot"],
        "other_precision": other,
        "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in timing.items()} if timing else None,
        "roofline": roofline(timing, args.prec) if timing else None,
        "records": records or None,
        "cpu_baseline": None,
    }
    if not args.profile_only and args.cpu_baseline != "off":
        W2 = workloads.helmholtz_workload("helmholtz2d_n256_w32", 2, 256, 2, 32.0, 64, 0.05, 16)
        c2 = torch.as_tensor(W2.coeff, dtype=torch.float64, device=dev).contiguous()
        pb2 = spp.binding.spp_problem(dim=2, n=256, b=16, kind=spp.SPP_HELMHOLTZ, omega=W2.omega,
                                      ell=1.0, energy=0.0, coeff=c2.data_ptr())
        h2 = spp.spp_setup(pb2, options("c128", 0), stream)
        st256 = spp.spp_stats(h2)
        spp.spp_destroy(h2)
        if args.cpu_baseline == "full":
            print("bench: timing the CPU oracle on the benchmark workload (one to two minutes)", file=sys.stderr,
                  flush=True)
            cb = cpu_baseline_full(W, args.tol)
            print("bench: timing the scaled 256^2 oracle sample (cross-check)", file=sys.stderr, flush=True)
            cb["cross_check"] = cpu_baseline(iters, st, st256)
        else:
            print("bench: timing the CPU oracle baseline (about half a minute)", file=sys.stderr, flush=True)
            cb = cpu_baseline(iters, st, st256)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
