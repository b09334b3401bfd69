"""Training and evaluation of the learned flexible-GMRES stage.

Pairs (v_j, M v_j) come from the first Arnoldi steps of sparsifying-
preconditioned FGMRES solves over a family of seeded random media (M the
sparsifying preconditioner, v_j unit-norm Krylov vectors); the network is
trained on them with Adam by the library's own forward / backward kernels,
then attached to solves of unseen media, where FGMRES keeps each network step
only if it reduces the residual enough (the sparsifying preconditioner is the
fallback).  Every step runs through the C ABI; this module only drives it.
"""
from __future__ import annotations

import math
import time

import numpy as np

import workloads

from .binding import CNN, Solver


def family_workload(n: int, waves: float, bumps: int, width: float, seed: int):
    """One medium of the random-media family and one Gaussian source."""
    omega = 2.0 * math.pi * waves
    med = workloads.gaussian_bump_medium(n, 2, omega, bumps, width, seed)
    f = workloads.gaussian_sources(n, 2, 1, 1.0 / 32, seed + 500)[0]
    return omega, med.c, f


def training_pairs(n: int, b: int, waves: float, bumps: int, width: float, seeds, per_medium: int = 20,
                   tol: float = 1e-10, exact_count: bool = False):
    """(V, Z): complex tensors [pairs][n^2], scaled so that each v has unit RMS.
    exact_count: run per_medium iterations whatever the residual (tolerance 0
    and max_iter = per_medium), so that every medium gives per_medium pairs."""
    import torch
    vs, zs = [], []
    for seed in seeds:
        omega, c, f = family_workload(n, waves, bumps, width, seed)
        if exact_count:
            S = Solver("helmholtz", n, 2, b, c, omega=omega, tol=1e-300, max_iter=per_medium)
        else:
            S = Solver("helmholtz", n, 2, b, c, omega=omega, tol=tol, max_iter=max(per_medium + 1, 60))
        _, iters, _, _ = S.solve(f)
        for j in range(min(per_medium, iters[0])):
            v, z = S.krylov(j)
            vs.append(v[0])
            zs.append(z[0])
        S.close()
    s = math.sqrt(n * n)
    return torch.stack(vs) * s, torch.stack(zs) * s


def he_init(channels, seed: int):
    """He-normal weights, one (Cout, Cin, 3, 3) array per layer (std sqrt(2 / (9 Cin)))."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((co, ci, 3, 3)) * math.sqrt(2.0 / (9 * ci))
            for ci, co in zip(channels[:-1], channels[1:])]


def train(cnn: CNN, V, Z, epochs: int, batch: int, lr: float = 1e-3, seed: int = 0):
    """Adam on mean ||net(v) - z||^2 / ||z||^2; returns the mean loss per epoch."""
    import torch
    rng = np.random.default_rng(seed)
    hist = []
    P = V.shape[0]
    for _ in range(epochs):
        order = rng.permutation(P)
        tot, cnt = 0.0, 0
        for k in range(0, P - batch + 1, batch):
            idx = torch.as_tensor(order[k:k + batch], device=V.device)
            loss = cnn.loss_grad(V[idx], Z[idx])
            cnn.adam_step(lr)
            tot += loss
            cnt += 1
        hist.append(tot / max(cnt, 1))
    return hist


def evaluate(cnn, n: int, b: int, waves: float, bumps: int, width: float, seeds, tol: float = 1e-10,
             rho: float = 0.9):
    """Per held-out medium: iterations and time without / with the network, accepted and
    rejected network steps, and the relative difference of the two solutions."""
    import torch
    rows = []
    for seed in seeds:
        omega, c, f = family_workload(n, waves, bumps, width, seed)
        S = Solver("helmholtz", n, 2, b, c, omega=omega, tol=tol, max_iter=200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u0, it0, rr0, _ = S.solve(f)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        S.attach_cnn(cnn, rho)
        u1, it1, rr1, code = S.solve(f)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        acc, rej = S.learned_stats()
        S.attach_cnn(None)
        S.close()
        diff = float(torch.linalg.norm(u1 - u0) / torch.linalg.norm(u0))
        rows.append({"seed": seed, "iters_plain": it0[0], "iters_learned": it1[0], "accepted": acc,
                     "rejected": rej, "precond_applies_learned": it1[0] - acc + 0,
                     "ms_plain": 1e3 * (t1 - t0), "ms_learned": 1e3 * (t2 - t1),
                     "relres": rr1[0], "code": code, "diff": diff})
    return rows


def protocol(n: int = 256, b: int = 16, waves: float = 32.0, bumps: int = 64, width: float = 0.05,
             train_seeds=range(0, 200), test_seeds=range(10000, 10100), per_medium: int = 20, epochs: int = 50,
             batch: int = 32, lr: float = 1e-3, tol: float = 1e-8, rho: float = 0.9, dtype: str = "bf16",
             log=print):
    """The learned stage's configuration end to end: per_medium (v_j, M v_j)
    pairs from each training medium, Adam for `epochs` epochs on the GPU
    kernels, then every held-out medium solved to tol with and without the
    network (sparsifying preconditioner as fallback and judge).  Returns a
    summary dict (iterations, solves per second, accept rate, loss history)."""
    import torch
    t0 = time.perf_counter()
    V, Z = training_pairs(n, b, waves, bumps, width, train_seeds, per_medium=per_medium, exact_count=True)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    log(f"learned: {V.shape[0]} pairs from {len(train_seeds)} media in {t_pairs:.1f} s")
    cnn = CNN(n, dtype=dtype, max_batch=batch)
    cnn.set_weights(he_init(cnn.channels, 0))
    t0 = time.perf_counter()
    hist = []
    for e in range(epochs):
        hist += train(cnn, V, Z, epochs=1, batch=batch, lr=lr, seed=e)
        if e % 10 == 0 or e == epochs - 1:
            log(f"learned: epoch {e} loss {hist[-1]:.4f}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del V, Z
    torch.cuda.empty_cache()
    rows = evaluate(cnn, n, b, waves, bumps, width, test_seeds, tol=tol, rho=rho)
    cnn.close()
    ms0 = sum(r["ms_plain"] for r in rows)
    ms1 = sum(r["ms_learned"] for r in rows)
    it0 = [r["iters_plain"] for r in rows]
    it1 = [r["iters_learned"] for r in rows]
    acc = sum(r["accepted"] for r in rows)
    rej = sum(r["rejected"] for r in rows)
    return {
        "grid": n, "b": b, "omega_over_2pi": waves, "bumps": bumps, "train_media": len(train_seeds),
        "pairs": len(train_seeds) * per_medium, "epochs": epochs, "batch": batch, "lr": lr, "dtype": dtype,
        "held_out_media": len(rows), "tol": tol, "rho": rho,
        "t_pairs_s": t_pairs, "t_train_s": t_train,
        "train_samples_per_s": len(train_seeds) * per_medium * epochs / t_train,
        "loss_first": hist[0], "loss_last": hist[-1],
        "iters_plain_mean": float(np.mean(it0)), "iters_learned_mean": float(np.mean(it1)),
        "iters_plain_range": [int(min(it0)), int(max(it0))], "iters_learned_range": [int(min(it1)), int(max(it1))],
        "solves_per_s_plain": len(rows) / (ms0 / 1e3), "solves_per_s_learned": len(rows) / (ms1 / 1e3),
        "accepted": acc, "rejected": rej, "accept_rate": acc / max(acc + rej, 1),
        "all_converged": all(r["code"] == 0 for r in rows), "max_diff": max(r["diff"] for r in rows),
        "max_relres_learned": max(r["relres"] for r in rows),
    }


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned FGMRES stage: train and evaluate at its configuration")
    ap.add_argument("--media", type=int, default=200)
    ap.add_argument("--held-out", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=50)
    ap.add_argument("--out", default=None, help="write the summary JSON here")
    a = ap.parse_args()
    res = protocol(train_seeds=range(0, a.media), test_seeds=range(10000, 10000 + a.held_out), epochs=a.epochs,
                   log=lambda m: print(m, flush=True))
    text = json.dumps(res)
    print(text, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")
