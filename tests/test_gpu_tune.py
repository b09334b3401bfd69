"""Autotuned launch parameters and factorisation schedules: same solution,
a written tuning table, and every schedule / solve form the tuner can pick
giving the same solution as the untuned factor."""
import itertools

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# mf_steps values: bit 0 paired steps, bit 1 64 x 64 L21 / U12 tiles, bit 2
# fused single steps (one launch per step); every combination the tuner tries.
SCHEDULES = [2, 0, 1, 3, 6, 4]


def rel(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def case(name):
    if name == "2d_128":
        return workloads.helmholtz_workload("mid", 5, 128, 2, 16.0, 16, 0.05, 8, nrhs=2), "octree"
    if name == "3d_octree":
        return workloads.small(12, 3, 3, waves=1.5, bumps=3, nrhs=2), "octree"
    return workloads.small(24, 3, 3, waves=3.0, bumps=3, nrhs=2), "bisect"


@pytest.mark.parametrize("name", ["2d_128", "3d_octree", "3d_bisect_24"])
def test_autotune_and_every_schedule_keep_the_solution(tmp_path, monkeypatch, name):
    from paper_1409_0297_amd import Solver, binding
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("SPP_TUNE_CACHE", str(path))
    W, order = case(name)
    kw = dict(omega=W.omega, tol=1e-11, max_iter=100, order=order)
    B = Solver(W.kind, W.n, W.d, W.b, W.coeff, **kw)          # untuned: heuristic schedules
    ub, ib, rb, cb = B.solve(W.rhs)
    B.close()
    A = Solver(W.kind, W.n, W.d, W.b, W.coeff, autotune=True, **kw)
    ua, ia, ra, ca = A.solve(W.rhs)
    A.close()
    torch.cuda.synchronize()
    assert ca == cb == 0
    assert all(abs(x - y) <= 1 for x, y in zip(ia, ib))
    assert rel(ua, ub) <= 1e-9
    text = path.read_text()
    for kind in ("fft_lines@", "gemv_chunks@", "mf_form@", "mf_steps@"):
        assert kind in text, kind
    mf_keys, gemv_keys = [], []
    for line in text.splitlines():
        key, value = line.split()
        if key.startswith("mf_form@"):
            assert int(value) in (0, 1, 2)
            mf_keys.append(key)
        elif key.startswith("mf_steps@"):
            assert int(value) in SCHEDULES
            mf_keys.append(key)
        elif key.startswith("gemv_chunks@"):
            assert int(value) >= 0   # (0: 16-row tiles, columns not split)
            gemv_keys.append((key, int(value)))
        else:
            assert int(value) >= 1
        assert binding.spp_tune_get(key) == int(value)
    # Every product shape of the substitution on 16-row tiles, then on 64-row
    # tiles without a column split, then split in two, then on 16-row tiles
    # split in two (1024 + 2): the same solution.
    try:
        for c in (0, 1, 2, 1026):
            for key, _ in gemv_keys:
                binding.spp_tune_set(key, c)
            C = Solver(W.kind, W.n, W.d, W.b, W.coeff, **kw)
            uc, ic, rc, cc = C.solve(W.rhs)
            C.close()
            torch.cuda.synchronize()
            assert cc == 0, c
            assert all(abs(x - y) <= 1 for x, y in zip(ic, ib)), (c, ic, ib)
            e = rel(uc, ub)
            print(f"{name}: substitution chunks {c}: iterations {ic}, vs untuned {e:.1e}")
            assert e <= 1e-9, (c, e)
    finally:
        for key, v in gemv_keys:
            binding.spp_tune_set(key, v)
    # Every candidate the tuner times is a valid factorisation: force each
    # schedule and solve form on every level and compare with the untuned
    # solution (same tolerance, so equal to roundoff times the conditioning).
    try:
        for steps, form in itertools.product(SCHEDULES, range(3)):
            for key in mf_keys:
                binding.spp_tune_set(key, steps if key.startswith("mf_steps@") else form)
            C = Solver(W.kind, W.n, W.d, W.b, W.coeff, **kw)
            uc, ic, rc, cc = C.solve(W.rhs)
            C.close()
            torch.cuda.synchronize()
            assert cc == 0, (steps, form)
            assert all(abs(x - y) <= 1 for x, y in zip(ic, ib)), (steps, form, ic, ib)
            e = rel(uc, ub)
            print(f"{name}: steps {steps} form {form}: iterations {ic}, vs untuned {e:.1e}")
            assert e <= 1e-9, (steps, form, e)
    finally:
        for key in mf_keys:
            binding.spp_tune_set(key, -1)
