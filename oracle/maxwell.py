"""The sparsifying preconditioner for the Maxwell (curl-curl) equation (Section 4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4 names the time-harmonic Maxwell equation for the electric field,
(curl curl - omega^2 eps(x)) E = f in units with c = 1, as the next target of
the method and gives no algorithm for it.  This module is the reading the
GPU path implements, written out with plain dense linear algebra:

* E has d components on the periodic grid of Section 2.1 (2D: the in-plane
  components E_0, E_1 of a field that does not depend on the third
  coordinate; 3D: all three).  Component a points along grid axis a.  A
  vector field is stored component-major, shape (d,) + (n,)*d, so unknown
  (a, j) has the flat index a N + j.
* curl is built from spectral first derivatives, whose wave numbers drop
  the Nyquist mode (the odd derivative of a real trigonometric interpolant):
  kt_a = k_a, except kt_a = 0 at the index n/2 along axis a.  Then curl curl
  has the d x d symbol K(k) = 4 pi^2 (|kt|^2 I - kt kt^T) per wave vector,
  acting on the d Fourier components together; it is real, even in k, turns
  with the grid, and vanishes on gradients built from the same derivatives.
  (With the Nyquist wave number -n/2 kept in the cross terms k_a k_b, which
  has no partner +n/2 on the grid, the kernel of G below would be complex
  and not rotation-equivariant.)
* The split of eq. (Dsq) carries over with w = omega^2 eps: s = mean(w),
  q = s - w, and the operator is K - s + q.  K is zero on longitudinal
  fields (kt parallel to the field) and 4 pi^2 |kt|^2 on transverse ones, so
  K - s is invertible for s > 0 unless some 4 pi^2 |kt|^2 equals s: the shift
  perturbation of Section 2.2 applies with these eigenvalues.
* G = (K - s)^{-1} has the symbol
  G(k) = (I - k^ k^T) / (4 pi^2 |kt|^2 - s) - k^ k^T / s with k^ = kt / |kt|,
  and G = -I / s where kt = 0; the integral equation is (I + G q) E = G f.
* The sets S, their neighbourhoods gamma(S) = S + beta(S) and the nested
  dissection boxes of Sections 2.3 and Figure 1 are unchanged.  A set's
  unknowns are all components of its points, ordered point-major (point i,
  component a at position i d + a) in the set's own lists; T_S =
  G(S, gamma^c) G(beta, gamma^c)^+ over those unknowns (explicit SVD
  pseudoinverse, MATLAB's cutoff), Q(S, gamma(S)) = [I  -T_S],
  C(S, gamma(S)) = Q(S, gamma(S)) G(gamma, gamma) and P = Q + C q, with q
  at each unknown's point.
* A box eliminates all components of its points.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp

from . import gmres, nested, spectral, stencil


# ---------------------------------------------------------------- symbols
def split_maxwell(omega: float, eps: np.ndarray):
    """Eq. (Dsq) with w = omega^2 eps: s = mean(w), q = s - w."""
    w = (omega * omega) * np.asarray(eps, dtype=np.float64)
    s = float(np.mean(w))
    return s, s - w


def shift_distance(n: int, d: int, s: float) -> float:
    """min over K of |4 pi^2 |kt|^2 - s| / |s| (transverse eigenvalues of K)."""
    kt = k_vectors(n, d)
    lam = 4.0 * math.pi ** 2 * np.sum(kt * kt, axis=0)
    return float(np.min(np.abs(lam - s)) / abs(s))


def coefficients(n: int, d: int, eps, omega: float, rel_gap: float = 1e-6,
                 step: float = 4.0 * math.pi ** 2 * 1e-3, tries: int = 10):
    """(s, q, shift perturbations); eps must be positive (s > 0).  The shift
    moves as in the scalar case (Section 2.2): while the relative gap to the
    nearest transverse eigenvalue is below rel_gap, s and q both gain step."""
    eps = np.asarray(eps, dtype=np.float64)
    if not np.all(eps > 0):
        raise ValueError("eps must be positive")
    s, q = split_maxwell(omega, eps)
    for t in range(tries + 1):
        if shift_distance(n, d, s) >= rel_gap:
            return s, q, t
        if t == tries:
            break
        s, q = s + step, q + step
    raise ValueError("could not move the shift away from the spectrum of curl curl")


def k_vectors(n: int, d: int) -> np.ndarray:
    """First-derivative wave vectors kt on K, shape (d,) + (n,)*d, FFT order
    along every axis, 0 at the Nyquist index n/2."""
    k = spectral.k_axis(n).astype(np.float64)
    k[n // 2] = 0.0
    out = np.zeros((d,) + (n,) * d)
    for a in range(d):
        shape = [1] * d
        shape[a] = n
        out[a] = np.broadcast_to(k.reshape(shape), (n,) * d)
    return out


def curlcurl_symbol(n: int, d: int) -> np.ndarray:
    """K(k) = 4 pi^2 (|kt|^2 I - kt kt^T), shape (d, d) + (n,)*d."""
    k = k_vectors(n, d)
    k2 = np.sum(k * k, axis=0)
    K = np.zeros((d, d) + (n,) * d)
    for a in range(d):
        for b in range(d):
            K[a, b] = 4.0 * math.pi ** 2 * ((k2 if a == b else 0.0) - k[a] * k[b])
    return K


def green_symbol(n: int, d: int, s: float) -> np.ndarray:
    """G(k) = (I - k^ k^T) / (4 pi^2 |kt|^2 - s) - k^ k^T / s, -I / s where kt = 0."""
    k = k_vectors(n, d)
    k2 = np.sum(k * k, axis=0)
    safe = np.where(k2 > 0, k2, 1.0)
    trans = 1.0 / (4.0 * math.pi ** 2 * k2 - s)
    G = np.zeros((d, d) + (n,) * d)
    for a in range(d):
        for b in range(d):
            proj = np.where(k2 > 0, k[a] * k[b] / safe, 0.0)   # k^_a k^_b (0 at k = 0)
            G[a, b] = ((1.0 if a == b else 0.0) - proj) * trans - proj / s
    return G


def apply_symbol(M: np.ndarray, E: np.ndarray) -> np.ndarray:
    """F^{-1} M(k) F E for a (d, d)-matrix symbol M and a field E of shape (d,) + (n,)*d."""
    d = E.shape[0]
    Eh = spectral.fourier(np.asarray(E, dtype=np.complex128), d)
    out = np.zeros_like(Eh)
    for a in range(d):
        for b in range(d):
            out[a] += M[a, b] * Eh[b]
    return spectral.inverse_fourier(out, d)


def apply_curlcurl(E: np.ndarray) -> np.ndarray:
    d, n = E.shape[0], E.shape[-1]
    return apply_symbol(curlcurl_symbol(n, d), E)


def apply_green(v: np.ndarray, s: float) -> np.ndarray:
    d, n = v.shape[0], v.shape[-1]
    return apply_symbol(green_symbol(n, d, s), v)


def apply_differential(E: np.ndarray, s: float, q: np.ndarray) -> np.ndarray:
    """(K - s + q) E, q acting pointwise on every component."""
    return apply_curlcurl(E) - s * E + q[None] * E


def apply_integral(E: np.ndarray, s: float, q: np.ndarray) -> np.ndarray:
    """(I + G q) E."""
    return E + apply_green(q[None] * E, s)


def green_kernels(n: int, d: int, s: float) -> np.ndarray:
    """g[a, b] with G((a, i), (b, j)) = g[a, b][(i - j) mod n], shape (d, d) + (n,)*d."""
    G = green_symbol(n, d, s)
    g = np.zeros(G.shape, dtype=np.complex128)
    for a in range(d):
        for b in range(d):
            g[a, b] = spectral.inverse_fourier(G[a, b].astype(np.complex128), d) / n ** (d / 2.0)
    return g


def dense_differential(n: int, d: int, s: float, q: np.ndarray) -> np.ndarray:
    """Dense (d N) x (d N) matrix of K - s + q, component-major unknowns; d N <= ~4000."""
    W = spectral.dft_matrix(n)
    V = spectral.idft_matrix(n)
    Fd, Fi = W, V
    for _ in range(d - 1):
        Fd = np.kron(Fd, W)
        Fi = np.kron(Fi, V)
    K = curlcurl_symbol(n, d)
    N = n ** d
    A = np.zeros((d * N, d * N), dtype=np.complex128)
    for a in range(d):
        for b in range(d):
            A[a * N:(a + 1) * N, b * N:(b + 1) * N] = (Fi * K[a, b].reshape(-1)[None, :]) @ Fd
    A -= s * np.eye(d * N)
    A += np.diag(np.tile(np.asarray(q, dtype=np.float64).reshape(-1), d))
    return A


# ---------------------------------------------------------------- stencils
def unknowns(points: np.ndarray, d: int, N: int) -> np.ndarray:
    """Global indices of the point-major unknown list of a point list: (i, a) -> a N + points[i]."""
    return (np.asarray(points, dtype=np.int64)[:, None] + N * np.arange(d)[None, :]).reshape(-1)


def green_block(g: np.ndarray, rows: np.ndarray, cols: np.ndarray, n: int, d: int) -> np.ndarray:
    """G(rows, cols) for global unknown indices a N + j (eq. G per component pair)."""
    N = n ** d
    ra, rj = np.divmod(np.asarray(rows, dtype=np.int64), N)
    ca, cj = np.divmod(np.asarray(cols, dtype=np.int64), N)
    rp = stencil.unravel(rj, n, d)
    cp = stencil.unravel(cj, n, d)
    diff = (rp[:, None, :] - cp[None, :, :]) % n
    return g[(ra[:, None], ca[None, :]) + tuple(diff[..., i] for i in range(d))]


class VectorStencils:
    """T_S and C_S of every set type over the d components of its points
    (one computation per type at anchor 0: translates share them)."""

    def __init__(self, n: int, d: int, b: int, s: float):
        if n % b or (n // b) < 2:
            raise ValueError("b must divide n with at least two leaf boxes per axis")
        self.n, self.d, self.b, self.s = n, d, b, s
        self.N = n ** d
        self.g = green_kernels(n, d, s)
        self.masks = stencil.set_masks(d)
        self.T, self.C, self.S0, self.beta0 = {}, {}, {}, {}
        for mask in self.masks:
            S, beta = stencil.set_geometry(n, d, b, mask)
            self.S0[mask], self.beta0[mask] = S, beta
            uS, uB = unknowns(S, d, self.N), unknowns(beta, d, self.N)
            gam = np.concatenate([uS, uB])
            outside = np.setdiff1d(np.arange(d * self.N), gam)
            A = green_block(self.g, uB, outside, n, d)
            pinvA = np.linalg.pinv(A, rcond=max(A.shape) * np.finfo(np.float64).eps)
            T = green_block(self.g, uS, outside, n, d) @ pinvA
            Qblk = np.concatenate([np.eye(uS.size), -T], axis=1)
            self.T[mask] = T
            self.C[mask] = Qblk @ green_block(self.g, gam, gam, n, d)

    def instances(self, mask):
        """(rows, cols): global unknown indices of every translate, rows (m^d, d |S|),
        cols (m^d, d |gamma|) in the (S, beta) order, point-major inside each part."""
        n, d, b = self.n, self.d, self.b
        base = np.concatenate([self.S0[mask], self.beta0[mask]])
        base_pts = stencil.unravel(base, n, d)
        nS = self.S0[mask].size
        rows, cols = [], []
        for anchor in itertools.product(range(n // b), repeat=d):
            pts = stencil.ravel((base_pts + np.array(anchor, dtype=np.int64) * b) % n, n)
            u = unknowns(pts, d, self.N)
            rows.append(u[: d * nS])
            cols.append(u)
        return np.array(rows), np.array(cols)

    def _assemble(self, value_fn):
        M = self.d * self.N
        R, Cc, V = [], [], []
        for mask in self.masks:
            rows, cols = self.instances(mask)
            vals = value_fn(mask, cols)
            R.append(np.broadcast_to(rows[:, :, None], vals.shape).reshape(-1))
            Cc.append(np.broadcast_to(cols[:, None, :], vals.shape).reshape(-1))
            V.append(vals.reshape(-1))
        return sp.coo_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(Cc))), shape=(M, M)).tocsr()

    def Q_matrix(self):
        def fn(mask, cols):
            blk = np.concatenate([np.eye(self.T[mask].shape[0]), -self.T[mask]], axis=1)
            return np.broadcast_to(blk, (cols.shape[0],) + blk.shape)
        return self._assemble(fn)

    def P_matrix(self, q: np.ndarray):
        """P = Q + C q, q taken at each column unknown's point."""
        qu = np.tile(np.asarray(q, dtype=np.float64).reshape(-1), self.d)

        def fn(mask, cols):
            blk = np.concatenate([np.eye(self.T[mask].shape[0]), -self.T[mask]], axis=1)
            return blk[None] + self.C[mask][None] * qu[cols][:, None, :]
        return self._assemble(fn)


def apply_Q(st: VectorStencils, r: np.ndarray) -> np.ndarray:
    """(Q r)_S = r_S - T_S r_beta(S) per set, r of shape (d,) + (n,)*d."""
    flat = np.asarray(r, dtype=np.complex128).reshape(-1)
    out = np.empty_like(flat)
    for mask in st.masks:
        rows, cols = st.instances(mask)
        k = rows.shape[1]
        out[rows] = flat[rows] - flat[cols[:, k:]] @ st.T[mask].T
    return out.reshape(r.shape)


def nd_levels(n: int, d: int, b: int, ordering: str = "octree"):
    """The scalar nested-dissection boxes with every point's d unknowns."""
    N = n ** d
    return [[unknowns(g, d, N) for g in groups] for groups in nested.nd_levels(n, d, b, ordering)]


# ---------------------------------------------------------------- pipeline
class MaxwellSetup:
    def __init__(self, n: int, d: int, b: int, eps, omega: float, ordering: str = "octree"):
        self.n, self.d, self.b, self.omega = n, d, b, omega
        self.s, self.q, self.shift_moves = coefficients(n, d, eps, omega)
        self.stencils = VectorStencils(n, d, b, self.s)
        self.P = self.stencils.P_matrix(self.q)
        self.factor = nested.NDFactor(self.P, nd_levels(n, d, b, ordering))


def precondition(o: MaxwellSetup, r: np.ndarray) -> np.ndarray:
    """z = P^{-1} Q r."""
    return o.factor.solve(apply_Q(o.stencils, r).reshape(-1)).reshape(r.shape)


def solve(o: MaxwellSetup, f: np.ndarray, tol: float = 1e-10, max_iter: int = 300, preconditioned: bool = True):
    """(I + G q) E = G f by FGMRES; returns (E, iterations, history)."""
    g = apply_green(f, o.s)
    A = lambda z: apply_integral(z, o.s, o.q)
    M = (lambda r: precondition(o, r)) if preconditioned else None
    return gmres.fgmres(A, g, M, tol=tol, max_iter=max_iter)


def dense_solution(n: int, d: int, eps, omega: float, f: np.ndarray) -> np.ndarray:
    """E* of (K - s + q) E = f by a dense solve; d n^d <= ~4000."""
    s, q, _ = coefficients(n, d, eps, omega)
    A = dense_differential(n, d, s, q)
    return np.linalg.solve(A, np.asarray(f, dtype=np.complex128).reshape(-1)).reshape(f.shape)
