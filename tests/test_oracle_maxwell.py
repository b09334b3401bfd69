"""Pins of the Maxwell (curl-curl) oracle (Section 4) against facts that do
not come from its own formulas: curl taken twice by spectral derivatives
(numpy's FFT, not the oracle's DFT), the null space of curl curl, transverse
plane waves, the inverse relation of G, the normal equations of the
least-squares stencils, the rotation symmetry of the stencils (which moves
points and turns field components), P against a dense Q G, and end-to-end
solves against a dense solve."""
import math

import numpy as np
import pytest

import workloads
from oracle import maxwell, stencil


def deriv(u, axis):
    """Spectral derivative d/dx_axis on [0, 1)^d by numpy's FFT, Nyquist
    mode dropped (the odd derivative of the real trigonometric interpolant)."""
    n = u.shape[axis]
    k = np.fft.fftfreq(n, 1.0 / n)
    k[n // 2] = 0.0
    shape = [1] * u.ndim
    shape[axis] = n
    return np.fft.ifft(2j * math.pi * k.reshape(shape) * np.fft.fft(u, axis=axis), axis=axis)


def curl_curl_2d(E):
    """In-plane field: curl E = d0 E1 - d1 E0 (out of plane), curl (c e_z) = (d1 c, -d0 c)."""
    c = deriv(E[1], 0) - deriv(E[0], 1)
    return np.stack([deriv(c, 1), -deriv(c, 0)])


def curl_3d(E):
    return np.stack([deriv(E[2], 1) - deriv(E[1], 2),
                     deriv(E[0], 2) - deriv(E[2], 0),
                     deriv(E[1], 0) - deriv(E[0], 1)])


def rand_field(rng, d, n):
    return rng.standard_normal((d,) + (n,) * d) + 1j * rng.standard_normal((d,) + (n,) * d)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("d,n", [(2, 12), (3, 6)])
def test_curlcurl_is_curl_taken_twice(d, n):
    E = rand_field(np.random.default_rng(1), d, n)
    want = curl_curl_2d(E) if d == 2 else curl_3d(curl_3d(E))
    assert rel(maxwell.apply_curlcurl(E), want) <= 1e-12


@pytest.mark.parametrize("d,n", [(2, 12), (3, 8)])   # (|k_a| < n / 2: no aliased wave numbers)
def test_gradients_are_the_null_space_and_transverse_waves_scale(d, n):
    rng = np.random.default_rng(2)
    phi = rng.standard_normal((n,) * d)
    grad = np.stack([deriv(phi, a) for a in range(d)])
    assert np.linalg.norm(maxwell.apply_curlcurl(grad)) <= 1e-10 * np.linalg.norm(grad) * n * n
    x = workloads.grid_points(n, d)
    k = np.array([1, -2, 3][:d], dtype=np.float64)
    v = np.array([2.0, 1.0, 0.0][:d]) if d == 2 else np.array([3.0, 0.0, -1.0])
    assert abs(v @ k) < 1e-15                      # transverse: v perpendicular to k
    E = v.reshape((d,) + (1,) * d) * np.exp(2j * math.pi * (x @ k))[None]
    assert rel(maxwell.apply_curlcurl(E), 4 * math.pi ** 2 * (k @ k) * E) <= 1e-12
    L = k.reshape((d,) + (1,) * d) * np.exp(2j * math.pi * (x @ k))[None]   # longitudinal
    assert np.linalg.norm(maxwell.apply_curlcurl(L)) <= 1e-10 * np.linalg.norm(L)


@pytest.mark.parametrize("d,n", [(2, 12), (3, 6)])
def test_green_inverts_the_shifted_operator(d, n):
    rng = np.random.default_rng(3)
    s = 4 * math.pi ** 2 * 2.37
    v = rand_field(rng, d, n)
    Kv = maxwell.apply_curlcurl(v) - s * v
    assert rel(maxwell.apply_green(Kv, s), v) <= 1e-12
    assert rel(maxwell.apply_curlcurl(maxwell.apply_green(v, s)) - s * maxwell.apply_green(v, s), v) <= 1e-12
    phi = rng.standard_normal((n,) * d)
    grad = np.stack([deriv(phi, a) for a in range(d)])
    assert rel(maxwell.apply_green(grad, s), -grad / s) <= 1e-12    # K grad = 0


def test_green_kernels_are_real_even_symmetric_columns_of_G():
    """G(k) is a real symmetric d x d matrix, even in k: the kernels are real,
    even, and g[a, b] = g[b, a]; they turn with the grid; and they are the
    columns of G."""
    d, n, s = 2, 8, 4 * math.pi ** 2 * 1.7
    g = maxwell.green_kernels(n, d, s)
    assert np.abs(g.imag).max() <= 1e-14 * np.abs(g).max()
    for a in range(d):
        for b in range(d):
            assert np.allclose(g[a, b], g[b, a], atol=1e-15)
            mirrored = np.roll(np.flip(g[a, b], axis=(0, 1)), 1, axis=(0, 1))   # g[-m]
            assert np.allclose(g[a, b], mirrored, atol=1e-15)
    R = np.array([[0, -1], [1, 0]])
    for m in [(1, 0), (2, 3), (5, 1), (4, 3), (3, 7)]:
        Rm = (R @ np.array(m)) % n
        assert np.allclose(g[:, :, Rm[0], Rm[1]], R @ g[:, :, m[0], m[1]] @ R.T, atol=1e-15)
    for b in range(d):
        e = np.zeros((d, n, n), dtype=np.complex128)
        e[b, 0, 0] = 1.0
        col = maxwell.apply_green(e, s)          # G e_(b, 0): column (b, 0), entries g[a, b][i]
        for a in range(d):
            assert np.allclose(col[a], g[a, b], atol=1e-14)


def test_dense_operator_matches_the_spectral_apply():
    d, n = 2, 8
    rng = np.random.default_rng(4)
    s = 4 * math.pi ** 2 * 1.3
    q = rng.standard_normal((n, n))
    E = rand_field(rng, d, n)
    A = maxwell.dense_differential(n, d, s, q)
    assert rel((A @ E.reshape(-1)).reshape(E.shape), maxwell.apply_differential(E, s, q)) <= 1e-12


@pytest.fixture(scope="module")
def st2d():
    return maxwell.VectorStencils(16, 2, 4, 4 * math.pi ** 2 * 2.9)


def test_stencils_solve_their_normal_equations(st2d):
    st = st2d
    for mask in st.masks:
        S, beta = st.S0[mask], st.beta0[mask]
        uS, uB = maxwell.unknowns(S, 2, st.N), maxwell.unknowns(beta, 2, st.N)
        out = np.setdiff1d(np.arange(2 * st.N), np.concatenate([uS, uB]))
        A = maxwell.green_block(st.g, uB, out, st.n, 2)
        B = maxwell.green_block(st.g, uS, out, st.n, 2)
        lhs = st.T[mask] @ (A @ A.conj().T)
        assert rel(lhs, B @ A.conj().T) <= 1e-8, mask
        assert st.T[mask].shape == (2 * S.size, 2 * beta.size)


def test_stencils_turn_with_the_grid(st2d):
    """A quarter turn about the set's centre maps cells and vertices onto
    themselves; T_S must be invariant when the points move with it and the
    field components turn with it: R = [[0, -1], [1, 0]] on (x0, x1)."""
    st = st2d
    n, b = st.n, st.b
    R = np.array([[0, -1], [1, 0]])
    for mask, centre in (((False, False), (b // 2, b // 2)), ((True, True), (0, 0))):
        S, beta = st.S0[mask], st.beta0[mask]

        def turned(idx):
            p = stencil.unravel(idx, n, 2) - np.array(centre)
            p = (p @ R.T + np.array(centre)) % n
            return stencil.ravel(p, n)

        def perm(lst):
            pos = {int(v): i for i, v in enumerate(lst)}
            return np.array([pos[int(v)] for v in turned(lst)])

        pS, pB = perm(S), perm(beta)
        # unknown (i, a) -> (pi(i), R a): matrix M with (M x)_(pi(i)) = R x_i
        def op(p, m):
            M = np.zeros((2 * m, 2 * m))
            for i in range(m):
                M[2 * p[i]:2 * p[i] + 2, 2 * i:2 * i + 2] = R
            return M
        MS, MB = op(pS, S.size), op(pB, beta.size)
        T = st.T[mask]
        assert rel(MS @ T @ MB.T, T) <= 1e-8, mask


def test_stencils_translate(st2d):
    """T_S computed directly at another anchor equals the anchor-0 one."""
    st = st2d
    mask = (True, False)
    shift = np.array([2, 1]) * st.b
    S, beta = (stencil.ravel((stencil.unravel(x, st.n, 2) + shift) % st.n, st.n)
               for x in (st.S0[mask], st.beta0[mask]))   # the anchor-0 lists, moved
    uS, uB = maxwell.unknowns(S, 2, st.N), maxwell.unknowns(beta, 2, st.N)
    out = np.setdiff1d(np.arange(2 * st.N), np.concatenate([uS, uB]))
    A = maxwell.green_block(st.g, uB, out, st.n, 2)
    T = maxwell.green_block(st.g, uS, out, st.n, 2) @ np.linalg.pinv(A, rcond=max(A.shape) * np.finfo(float).eps)
    assert rel(T, st.T[mask]) <= 1e-8


def test_P_is_Q_plus_QG_times_q_on_its_pattern():
    n, d, b = 8, 2, 4
    rng = np.random.default_rng(5)
    s = 4 * math.pi ** 2 * 1.9
    q = rng.standard_normal((n, n))
    st = maxwell.VectorStencils(n, d, b, s)
    Q = st.Q_matrix().toarray()
    P = st.P_matrix(q).toarray()
    N = n * n
    Gd = np.zeros((d * N, d * N), dtype=np.complex128)
    for j in range(d * N):
        e = np.zeros(d * N, dtype=np.complex128)
        e[j] = 1.0
        Gd[:, j] = maxwell.apply_green(e.reshape(d, n, n), s).reshape(-1)
    QG = Q @ Gd
    qu = np.tile(q.reshape(-1), d)
    for mask in st.masks:
        rows, cols = st.instances(mask)
        for r, c in zip(rows, cols):
            want = Q[np.ix_(r, c)] + QG[np.ix_(r, c)] * qu[c][None, :]
            assert np.allclose(P[np.ix_(r, c)], want, atol=1e-10)
    assert np.array_equal(np.abs(Q) > 0, (np.abs(Q) > 0) & (np.abs(P) > 0) | (np.abs(Q) > 0))
    pattern = np.zeros(P.shape, dtype=bool)
    for mask in st.masks:
        rows, cols = st.instances(mask)
        for r, c in zip(rows, cols):
            pattern[np.ix_(r, c)] = True
    assert not np.any((np.abs(P) > 0) & ~pattern)     # nothing outside the sets' blocks


@pytest.mark.parametrize("d,n,b,waves,max_it", [(2, 16, 4, 2.0, 40), (3, 8, 4, 1.0, 100)])
def test_preconditioned_solve_matches_dense(d, n, b, waves, max_it):
    W = workloads.maxwell_workload(n, d, b, waves, bumps=3)
    o = maxwell.MaxwellSetup(n, d, b, W.coeff, W.omega)
    f = W.rhs[0]
    E, it, hist = maxwell.solve(o, f, tol=1e-12, max_iter=200)
    Estar = maxwell.dense_solution(n, d, W.coeff, W.omega, f)
    assert rel(E, Estar) <= 1e-9
    assert it < max_it, it
    r = f - maxwell.apply_differential(E, o.s, o.q)
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(f)


def test_constant_permittivity_converges_in_one_iteration():
    n, d, b = 16, 2, 4
    eps = np.full((n, n), 1.3)
    f = workloads.maxwell_workload(n, d, b, 2.0).rhs[0]
    o = maxwell.MaxwellSetup(n, d, b, eps, 2 * math.pi * 2.0)
    assert np.abs(o.q).max() <= 1e-12 * o.s          # (the mean's rounding)
    E, it, _ = maxwell.solve(o, f, tol=1e-10)
    assert it == 1
    assert rel(E, maxwell.dense_solution(n, d, eps, 2 * math.pi * 2.0, f)) <= 1e-9


def test_preconditioner_pays_in_2d_with_wide_leaf_boxes():
    """64^2 at 8 points per wavelength: leaf boxes of 16 points cut the
    iterations well below unpreconditioned GMRES; boxes of 4 points do not
    (the longitudinal part of G decays only algebraically, so one ring of
    neighbours around a small set cannot localise Q G)."""
    W = workloads.maxwell_workload(64, 2, 16, 8.0, bumps=3)
    f = W.rhs[0]
    wide = maxwell.MaxwellSetup(64, 2, 16, W.coeff, W.omega)
    _, it_wide, _ = maxwell.solve(wide, f, tol=1e-10, max_iter=300)
    _, it_none, _ = maxwell.solve(wide, f, tol=1e-10, max_iter=300, preconditioned=False)
    narrow = maxwell.MaxwellSetup(64, 2, 4, W.coeff, W.omega)
    _, it_narrow, _ = maxwell.solve(narrow, f, tol=1e-10, max_iter=300)
    print(f"64^2 Maxwell: b = 16 {it_wide}, b = 4 {it_narrow}, unpreconditioned {it_none}")
    assert it_wide * 2 <= it_none
    assert it_narrow > it_wide
