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
                   tol: float = 1e-10):
    """(V, Z): complex tensors [pairs][n^2], scaled so that each v has unit RMS."""
    import torch
    vs, zs = [], []
    for seed in seeds:
        omega, c, f = family_workload(n, waves, bumps, width, seed)
        S = Solver("helmholtz", n, 2, b, c, omega=omega, tol=tol, max_iter=max(per_medium + 1, 60))
        _, iters, _, _ = S.solve(f)
        for j in range(min(per_medium, iters[0])):
            v, z = S.krylov(j)
            vs.append(v[0])
            zs.append(z[0])
        S.close()
    s = math.sqrt(n * n)
    return torch.stack(vs) * s, torch.stack(zs) * s


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
