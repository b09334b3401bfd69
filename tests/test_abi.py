"""CPU checks of the C ABI boundary: the library loads, exports every entry
point declared in include/spp.h, and rejects bad arguments before touching
the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1409_0297_amd as spp
from paper_1409_0297_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "spp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = spp.library()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert "spp_setup" in names and "spp_solve" in names


def test_error_strings():
    for code in range(-7, 1):
        assert spp.spp_error_string(code)
    assert spp.spp_error_string(99) == "unknown error"


def test_struct_layouts_match_header():
    assert ctypes.sizeof(binding.spp_problem) == 48
    assert binding.spp_problem.coeff.offset == 40
    assert ctypes.sizeof(binding.spp_options) == 56
    assert binding.spp_options.restart.offset == 24
    assert binding.spp_options.alloc.offset == 32
    assert binding.spp_options.alloc_ctx.offset == 48
    assert binding.spp_stats_t.breakdown_front.offset == 76
    assert binding.spp_stats_t.pivot_growth.offset == 88
    assert binding.spp_stats_t.small_pivots.offset == 112
    assert ctypes.sizeof(binding.spp_stats_t) == 120


@pytest.mark.parametrize("dim,n,b", [(4, 32, 8), (2, 30, 8), (2, 48, 16), (2, 32, 32), (2, 7, 1), (2, 96, 8)])
def test_setup_rejects_bad_grids_on_host(dim, n, b):
    """dim in {2,3}; n even; b | n; n / b a power of two >= 2 -- checked before any GPU call.
    (n = 96, b = 8 gives 12 leaf boxes per axis: not a power of two.)"""
    coeff = np.ones(4)
    pb = binding.spp_problem(dim=dim, n=n, b=b, kind=0, omega=1.0, ell=1.0, energy=0.0,
                             coeff=coeff.ctypes.data)
    op = binding.spp_options(prec=0, order=0, tol=1e-8, max_iter=10, flags=0)
    with pytest.raises(spp.SppError) as e:
        spp.spp_setup(pb, op, 0)
    assert e.value.code == spp.SPP_EINVAL


def test_setup_rejects_null_and_bad_options():
    pb = binding.spp_problem(dim=2, n=32, b=8, kind=0, omega=1.0, ell=1.0, energy=0.0, coeff=None)
    op = binding.spp_options(prec=0, order=0, tol=1e-8, max_iter=10, flags=0)
    with pytest.raises(spp.SppError) as e:
        spp.spp_setup(pb, op, 0)
    assert e.value.code == spp.SPP_EINVAL
    coeff = np.ones(32 * 32)
    pb.coeff = coeff.ctypes.data
    for bad in (dict(tol=0.0), dict(max_iter=0), dict(prec=5), dict(order=9), dict(restart=-1),
                dict(restart=501), dict(pattern=2), dict(pattern=-1)):
        o = binding.spp_options(prec=0, order=0, tol=1e-8, max_iter=10, flags=0)
        for k, v in bad.items():
            setattr(o, k, v)
        with pytest.raises(spp.SppError) as e:
            spp.spp_setup(pb, o, 0)
        assert e.value.code == spp.SPP_EINVAL
    pb.kind = 0
    pb.omega = -1.0
    with pytest.raises(spp.SppError):
        spp.spp_setup(pb, op, 0)


def test_null_handle_calls_fail_cleanly():
    lib = spp.library()
    assert lib.spp_solve(None, None, 1, None, None, None, None) == spp.SPP_EINVAL
    assert lib.spp_apply_operator(None, None, None, 1, None) == spp.SPP_EINVAL
    assert lib.spp_stats(None, None) == spp.SPP_EINVAL
    lib.spp_destroy(None)


def test_setup_rejects_half_an_allocator_hook():
    """alloc and free come together or not at all (checked before any GPU call)."""
    coeff = np.ones(32 * 32)
    pb = binding.spp_problem(dim=2, n=32, b=8, kind=0, omega=1.0, ell=1.0, energy=0.0, coeff=coeff.ctypes.data)
    op = binding.spp_options(prec=0, order=0, tol=1e-8, max_iter=10, flags=0)
    op.alloc = binding.ALLOC_FN(lambda n, ctx: None)
    with pytest.raises(spp.SppError) as e:
        spp.spp_setup(pb, op, 0)
    assert e.value.code == spp.SPP_EINVAL


def test_attach_cnn_and_batch_solve_reject_bad_arguments():
    lib = spp.library()
    # rho must be in (0, 1): with rho = 1 every network step would be kept
    fake_net = ctypes.c_void_p(8)   # never dereferenced: rho is checked first
    for rho in (1.0, 0.0, 1.5, float("nan")):
        assert lib.spp_attach_cnn(None, fake_net, ctypes.c_double(rho)) == spp.SPP_EINVAL
        assert "rho" in spp.spp_last_error()
    assert lib.spp_attach_cnn(None, fake_net, ctypes.c_double(0.5)) == spp.SPP_EINVAL
    assert "null factor" in spp.spp_last_error()
    assert lib.spp_solve_batch(None, None, None, None, None, None, None) == spp.SPP_EINVAL


def test_tuning_table_entries_round_trip(monkeypatch):
    """spp_tune_set / spp_tune_get touch only the host table (no GPU call)."""
    monkeypatch.delenv("SPP_TUNE_CACHE", raising=False)
    lib = spp.library()
    key = "mf_steps@test:8:1024:289:225"
    assert binding.spp_tune_get(key) is None
    binding.spp_tune_set(key, 3)
    assert binding.spp_tune_get(key) == 3
    binding.spp_tune_set(key, 1)
    assert binding.spp_tune_get(key) == 1
    binding.spp_tune_set(key, -1)
    assert binding.spp_tune_get(key) is None
    assert lib.spp_tune_set(None, 1) == spp.SPP_EINVAL
    assert lib.spp_tune_set(b"", 1) == spp.SPP_EINVAL
    v = ctypes.c_int32(0)
    assert lib.spp_tune_get(None, ctypes.byref(v)) == spp.SPP_EINVAL
    assert lib.spp_tune_get(key.encode(), None) == spp.SPP_EINVAL


def test_maxwell_setup_rejects_bad_problems_on_host():
    """Maxwell problems: omega > 0, leaf unknowns d (b + 1)^d <= 1024, and one
    problem per factor: refused before any GPU work."""
    lib = spp.library()
    eps = ctypes.c_double(1.0)   # (never read: the checks come first)
    op = binding.spp_options(prec=spp.SPP_C128, order=0, tol=1e-8, max_iter=10)
    out = ctypes.c_void_p()
    bad_omega = binding.spp_problem(dim=2, n=16, b=4, kind=spp.SPP_MAXWELL, omega=0.0,
                                    coeff=ctypes.addressof(eps))
    assert lib.spp_setup(ctypes.byref(bad_omega), ctypes.byref(op), None, ctypes.byref(out)) == spp.SPP_EINVAL
    big_leaf = binding.spp_problem(dim=3, n=48, b=6, kind=spp.SPP_MAXWELL, omega=1.0,
                                   coeff=ctypes.addressof(eps))   # 3 * 7^3 = 1029 unknowns
    assert lib.spp_setup(ctypes.byref(big_leaf), ctypes.byref(op), None, ctypes.byref(out)) == spp.SPP_ENOTIMPL
    ok = binding.spp_problem(dim=2, n=16, b=4, kind=spp.SPP_MAXWELL, omega=1.0, coeff=ctypes.addressof(eps))
    arr = (binding.spp_problem * 2)(ok, ok)
    assert lib.spp_setup_batch(arr, 2, ctypes.byref(op), None, ctypes.byref(out)) == spp.SPP_ENOTIMPL
