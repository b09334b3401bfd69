"""Pins for the oracle's sparsifying stencil (Section 2.3) and P = Q + C q (Section 2.2).

G is rebuilt here column by column from the DFT route (G applied to grid
deltas), so the stencil code's own kernel indexing is checked against an
independent construction.
"""
import itertools
import math

import numpy as np
import pytest

import workloads
from oracle import spectral, stencil


def dense_G(n, d, s):
    N = n ** d
    eye = np.eye(N, dtype=np.complex128).reshape((N,) + (n,) * d)
    cols = spectral.apply_green(eye, d, s).reshape(N, N)   # row t = G e_t
    return cols.T


@pytest.mark.parametrize("d,n,b", [(2, 16, 4), (2, 24, 6), (3, 8, 4), (3, 12, 3)])
def test_set_partition_and_sizes(d, n, b):
    """Cells hold (b-1)^d points, faces (b-1)^2, edges b-1, vertices 1; closures (b+1)^d;
    together the translates of all set types partition the grid (Section 2.3)."""
    m = n // b
    seen = np.zeros(n ** d, dtype=int)
    for mask in stencil.set_masks(d):
        free = d - sum(mask)
        S, beta = stencil.set_geometry(n, d, b, mask)
        assert S.size == (b - 1) ** free
        assert S.size + beta.size == (b + 1) ** free * 3 ** (d - free)
        for anchor in itertools.product(range(m), repeat=d):
            seen[stencil.ravel(stencil.set_points(n, b, mask, anchor), n)] += 1
    assert (seen == 1).all()
    assert stencil.set_kind((False,) * d) == "cell" and stencil.set_kind((True,) * d) == "vertex"


def test_gamma_of_point_and_wraparound():
    """gamma({j}) is the 3^d l-inf ball, taken mod n (Section 2.3)."""
    n = 6
    g = stencil.gamma(np.array([[0, 5]]), n)
    pts = {tuple(p) for p in stencil.unravel(g, n, 2)}
    assert pts == {((0 + a) % n, (5 + c) % n) for a in (-1, 0, 1) for c in (-1, 0, 1)}


@pytest.mark.parametrize("d,n,b", [(2, 16, 4), (3, 8, 2)])
def test_T_solves_least_squares(d, n, b):
    """T_S = G(S, gamma^c) G(beta, gamma^c)^+: the normal equations (B - T A) A^H = 0 hold."""
    s = 4 * math.pi ** 2 * (1.7 if d == 2 else 1.3)
    G = dense_G(n, d, s)
    g = spectral.green_kernel(n, d, s)
    for mask in stencil.set_masks(d):
        T, S, beta = stencil.stencil_T(g, n, d, b, mask)
        gam = np.concatenate([S, beta])
        out = np.setdiff1d(np.arange(n ** d), gam)
        A = G[np.ix_(beta, out)]
        B = G[np.ix_(S, out)]
        resid = (B - T @ A) @ A.conj().T
        assert np.linalg.norm(resid) <= 1e-10 * np.linalg.norm(B) * np.linalg.norm(A)
        # The Gram (normal-equation) formula gives the same T when A has full row rank.
        T_gram = B @ A.conj().T @ np.linalg.inv(A @ A.conj().T)
        assert np.linalg.norm(T_gram - T) <= 1e-8 * np.linalg.norm(T)


def test_T_translation_and_symmetry_invariance():
    """T_S is the same for every translate (Section 2.3), orientations are axis
    permutations of each other, and the cell stencil is invariant under the
    reflections of its box."""
    n, d, b = 32, 2, 8
    s = 4 * math.pi ** 2 * 16.3
    g = spectral.green_kernel(n, d, s)
    T0 = {m: stencil.stencil_T(g, n, d, b, m) for m in stencil.set_masks(d)}

    def perm(src, dst, fn):
        """Index map src-order -> dst-order under the point map fn."""
        dpos = {int(p): i for i, p in enumerate(dst)}
        mapped = stencil.ravel(fn(stencil.unravel(src, n, d)), n)
        return np.array([dpos[int(p)] for p in mapped])

    for mask in stencil.set_masks(d):
        T1, S1, b1 = stencil.stencil_T(g, n, d, b, mask, anchor=(2, 3))
        T, S, bb = T0[mask]
        move = lambda P: (P + np.array([2 * b, 3 * b])) % n
        pS, pb = perm(S, S1, move), perm(bb, b1, move)
        np.testing.assert_allclose(T1[np.ix_(pS, pb)], T, atol=1e-12 * np.abs(T).max())

    TA, SA, bA = T0[(True, False)]
    TB, SB, bB = T0[(False, True)]
    swap = lambda P: P[:, ::-1]
    pS, pb = perm(SA, SB, swap), perm(bA, bB, swap)
    np.testing.assert_allclose(TA, TB[np.ix_(pS, pb)], atol=1e-12 * np.abs(TA).max())

    Tc, Sc, bc = T0[(False, False)]
    for flip in ([0], [1], [0, 1]):
        def refl(P, flip=flip):
            P = P.copy()
            P[:, flip] = (b - P[:, flip]) % n
            return P
        pS, pb = perm(Sc, Sc, refl), perm(bc, bc, refl)
        np.testing.assert_allclose(Tc, Tc[np.ix_(pS, pb)], atol=1e-11 * np.abs(Tc).max())


def test_P_matches_dense_definition():
    """P = Q + C q with C(S, gamma(S)) = (Q G)(S, gamma(S)) on Q's pattern (Section 2.2)."""
    n, d, b = 16, 2, 4
    W = workloads.small(n, d, b, waves=2.0)
    s, q = spectral.split_helmholtz(W.omega, W.coeff)
    st = stencil.Stencils(n, d, b, s)
    Qd = st.Q_matrix().toarray()
    # Pattern from the definition: row j of Q is supported on gamma of j's set.
    pattern = np.zeros((n ** d, n ** d), dtype=bool)
    for mask in stencil.set_masks(d):
        for anchor in itertools.product(range(n // b), repeat=d):
            pts = stencil.set_points(n, b, mask, anchor)
            pattern[np.ix_(stencil.ravel(pts, n), stencil.gamma(pts, n))] = True
    assert not Qd[~pattern].any()
    G = dense_G(n, d, s)
    C = np.where(pattern, Qd @ G, 0.0)
    P_expected = Qd + C * q.reshape(-1)[None, :]
    np.testing.assert_allclose(st.P_matrix(q).toarray(), P_expected, atol=1e-12 * np.abs(P_expected).max())
    # Q has unit diagonal blocks and every row's support is gamma of its set.
    assert np.allclose(np.diag(Qd), 1.0)
    rng = np.random.default_rng(0)
    r = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    np.testing.assert_allclose(stencil.apply_Q(st, r).reshape(-1), Qd @ r.reshape(-1), atol=1e-12)


def test_Q_sparsifies_G():
    """Q G is essentially supported on gamma(S) (Section 2.2): the dropped part is small."""
    W = workloads.parity_2d()
    n, d, b = W.n, W.d, W.b
    s, q = spectral.split_helmholtz(W.omega, W.coeff)
    g = spectral.green_kernel(n, d, s)
    for mask in stencil.set_masks(d):
        T, S, beta = stencil.stencil_T(g, n, d, b, mask)
        gam = np.concatenate([S, beta])
        QG = np.concatenate([np.eye(S.size), -T], axis=1) @ stencil.green_block(g, gam, np.arange(n ** d), n, d)
        out = np.setdiff1d(np.arange(n ** d), gam)
        ratio = np.linalg.norm(QG[:, out]) / np.linalg.norm(QG)
        assert ratio < 0.1, (mask, ratio)
        # Without Q (rows of G itself) the off-neighbourhood part dominates.
        Grows = stencil.green_block(g, S, np.arange(n ** d), n, d)
        assert np.linalg.norm(Grows[:, out]) / np.linalg.norm(Grows) > 5 * ratio


def test_constant_medium_gives_P_equal_Q():
    """With constant c, q = 0 and P = Q (Section 2.2)."""
    n, d, b = 16, 2, 4
    s, q = spectral.split_helmholtz(2 * math.pi * 2.3, np.full((n, n), 1.0))
    assert np.abs(q).max() <= 1e-15 * s
    st = stencil.Stencils(n, d, b, s)
    assert abs(st.P_matrix(q) - st.Q_matrix()).max() <= 1e-12
    assert abs(st.P_matrix(np.zeros_like(q)) - st.Q_matrix()).max() == 0


@pytest.mark.parametrize("d,n", [(2, 16), (3, 8)])
def test_point_pattern_stencil(d, n):
    """The point pattern (every point its own set, mu(j) = gamma({j}), Section
    2.3): one stencil of 3^d - 1 neighbours, least-squares optimal against an
    independently built G, invariant under the reflections and axis swaps of
    the grid, and the rows of Q = [1  -T] partition the grid one point each."""
    s = 4 * math.pi ** 2 * (1.7 if d == 2 else 1.3)
    st = stencil.Stencils(n, d, 1, s)
    assert st.masks == [(True,) * d]
    mask = st.masks[0]
    T, S, beta = st.T[mask], st.S0[mask], st.beta0[mask]
    assert T.shape == (1, 3 ** d - 1) and S.tolist() == [0]
    G = dense_G(n, d, s)
    gam = np.concatenate([S, beta])
    out = np.setdiff1d(np.arange(n ** d), gam)
    A, B = G[np.ix_(beta, out)], G[np.ix_(S, out)]
    assert np.linalg.norm((B - T @ A) @ A.conj().T) <= 1e-10 * np.linalg.norm(B) * np.linalg.norm(A)
    # symmetric neighbourhood and symmetric kernel: T(offset) = T(-offset) and
    # T is invariant under axis permutations
    offs = stencil.unravel(beta, n, d)
    offs = np.where(offs > n // 2, offs - n, offs)
    val = {tuple(o): T[0, i] for i, o in enumerate(offs)}
    for o, v in val.items():
        assert abs(val[tuple(-x for x in o)] - v) <= 1e-10 * abs(v)
        assert abs(val[tuple(reversed(o))] - v) <= 1e-10 * abs(v)
    rows, cols = st.instances(mask)
    assert np.array_equal(np.sort(rows.reshape(-1)), np.arange(n ** d))
    Q = st.Q_matrix()
    assert Q.nnz == n ** d * 3 ** d
