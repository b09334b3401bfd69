"""3D Helmholtz with streamed front storage and blocked substitution of the
large top fronts (what the 128^3 configuration needs: its resident arena,
the sum of F^2 over all fronts, would exceed the device).

- Streamed storage (factors copied to a compact store, the arena holding two
  adjacent levels) gives the same solution bit for bit as resident storage
  where both use the same substitution forms.
- 32^3 (b = 4, bisection; the root front of 2048 pivots goes in blocked
  steps) against the oracle's own nested-dissection solve at 512 seeded
  points, for a Gaussian and a grid-delta source.
- 48^3 (b = 6, bisection): blocked levels with boundary rows (L21 / U12
  products beside the block steps) against resident storage, whose top
  levels use explicit inverses, and the oracle's differential residual.
- 128^3 (b = 8, bisection, complex64 fronts): the 3D configuration itself,
  4 Gaussian sources to 1e-10, checked by the invariants that hold at any
  size: the true residual, a real solution for real data, the differential
  residual under the oracle's spectral operator, and reciprocity of two
  grid-delta solutions (A = L - s + q is real symmetric).
"""
import os

import numpy as np
import pytest

import workloads
from oracle import pipeline, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD32 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "helmholtz3d_n32_u_samples.txt")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def solver(W, **kw):
    from paper_1409_0297_amd import Solver
    return Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, ell=W.ell, energy=W.energy, **kw)


@pytest.mark.parametrize("case", ["2d_64", "3d_12_bisect", "3d_16_bisect"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_streamed_storage_matches_resident(case, prec):
    W, order = {"2d_64": (workloads.parity_2d(nrhs=2), "octree"),
                "3d_12_bisect": (workloads.small(12, 3, 3, waves=1.5, bumps=3, nrhs=2), "bisect"),
                "3d_16_bisect": (workloads.helmholtz_3d(16, 4, nrhs=2), "bisect")}[case]
    out = []
    for streamed in (False, True):
        S = solver(W, prec=prec, order=order, tol=1e-11, max_iter=80, streamed=streamed)
        u, iters, relres, code = S.solve(W.rhs)
        st = S.stats()
        S.close()
        assert code == 0 and st["storage"] == int(streamed)
        out.append((cpu(u), iters))
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


def load32():
    samples = {0: ([], []), 1: ([], [])}
    norm_inf = {}
    with open(GOLD32) as fh:
        for line in fh:
            if line.startswith("#"):
                if "norm_inf" in line:
                    k = int(line.split("rhs")[1].split(":")[0])
                    norm_inf[k] = float(line.split("norm_inf")[1].split()[0])
                continue
            k, i, re, im = line.split()
            samples[int(k)][0].append(int(i))
            samples[int(k)][1].append(complex(float(re), float(im)))
    return {k: (np.array(v[0]), np.array(v[1])) for k, v in samples.items()}, norm_inf


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_3d_32_streamed_blocked_matches_oracle(prec):
    W = workloads.helmholtz_3d(32, 4, nrhs=1)
    n = W.n
    f = np.stack([W.rhs[0], workloads.grid_delta(n, 3, (n // 2, n // 2, n // 2))])
    S = solver(W, prec=prec, order="bisect", tol=1e-11, max_iter=100, streamed=True)
    u, iters, relres, code = S.solve(f)
    st = S.stats()
    S.close()
    assert code == 0 and st["storage"] == 1 and max(relres) <= 1e-11
    u = cpu(u).reshape(2, -1)
    gold, norm_inf = load32()
    for k in (0, 1):
        idx, ref = gold[k]
        e = rel(u[k][idx], ref)
        worst = np.max(np.abs(u[k][idx] - ref)) / norm_inf[k]
        print(f"3d 32^3 {prec} rhs {k}: iters {iters[k]}, err {e:.2e}, worst {worst:.2e}")
        assert e <= 1e-8 and worst <= 1e-8, (prec, k, e, worst)
    # resident storage solves the root with explicit inverses: same u
    S = solver(W, prec=prec, order="bisect", tol=1e-11, max_iter=100)
    u0, it0, _, code0 = S.solve(f)
    S.close()
    assert code0 == 0 and rel(cpu(u0).reshape(2, -1), u) <= 1e-9


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_3d_48_blocked_levels_with_boundary(prec):
    W = workloads.helmholtz_3d(48, 6, nrhs=2)
    S = solver(W, prec=prec, order="bisect", tol=1e-11, max_iter=100, streamed=True)
    u, iters, relres, code = S.solve(W.rhs)
    st = S.stats()
    S.close()
    assert code == 0 and st["storage"] == 1
    S = solver(W, prec=prec, order="bisect", tol=1e-11, max_iter=100)
    u0, it0, _, code0 = S.solve(W.rhs)
    S.close()
    assert code0 == 0
    u, u0 = cpu(u).reshape(W.rhs.shape), cpu(u0).reshape(W.rhs.shape)
    assert rel(u, u0) <= 1e-9
    s, q, _ = pipeline.coefficients(W.kind, W.n, W.d, W.coeff, W.omega)
    for k in range(2):
        r = W.rhs[k] - spectral.apply_differential(u[k], 3, s, q)
        assert np.linalg.norm(r) / np.linalg.norm(W.rhs[k]) <= 1e-7


def test_3d_128_configuration():
    """3D Helmholtz 128^3, omega = 2 pi 16, 32 bumps, b = 8 (8^3 leaves),
    bisection, complex64 fronts with FP64 FGMRES, 4 Gaussian sources."""
    W = workloads.helmholtz_3d(128, 8, nrhs=4)
    n = W.n
    S = solver(W, prec="c64", order="bisect", tol=1e-10, max_iter=80)
    st = S.stats()
    assert st["storage"] == 1 and st["max_front"] == 48896
    u, iters, relres, code = S.solve(W.rhs)
    st = S.stats()
    print(f"3d 128^3: setup {st['t_setup_ms']:.0f} ms (factor {st['t_factor_ms']:.0f} ms), "
          f"solve {st['t_solve_ms']:.0f} ms, iters {iters}, relres {max(relres):.2e}, "
          f"factor {st['factor_bytes'] / 1e9:.1f} GB, {st['factor_flops'] / 1e12:.0f} TFLOP, "
          f"min pivot {st['min_pivot']:.1e}, growth {st['pivot_growth']:.1f}")
    assert code == 0 and max(relres) <= 1e-10 and max(iters) <= 60
    u = cpu(u).reshape(W.rhs.shape)
    # real data: the solution is real
    assert np.linalg.norm(u.imag) <= 1e-8 * np.linalg.norm(u.real)
    s, q, _ = pipeline.coefficients(W.kind, W.n, W.d, W.coeff, W.omega)
    assert abs(st["s"] - s) <= 1e-12 * s
    for k in range(4):
        r = W.rhs[k] - spectral.apply_differential(u[k], 3, s, q)
        dres = np.linalg.norm(r) / np.linalg.norm(W.rhs[k])
        assert dres <= 1e-7, (k, dres)
    # reciprocity of two grid-delta solutions
    a, b = (n // 2, n // 2, n // 2), (n // 4, 3 * n // 4, n // 8)
    fd = np.stack([workloads.grid_delta(n, 3, a), workloads.grid_delta(n, 3, b)])
    ud, itd, rrd, coded = S.solve(fd)
    S.close()
    assert coded == 0
    ud = cpu(ud).reshape(fd.shape)
    uab, uba = ud[0][b], ud[1][a]
    print(f"reciprocity: u_a(b) = {uab:.6e}, u_b(a) = {uba:.6e}, iters {itd}")
    # (each solution carries its FGMRES error, about 1e-10 relative in norm)
    assert abs(uab) > 1e-3 * np.abs(ud[0]).max()
    assert abs(uab - uba) <= 1e-6 * max(abs(uab), abs(uba))
