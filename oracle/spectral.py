"""Pseudospectral discretisation (Section 2.1) and the Green operator (Section 2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything is FP64 / complex128 and deliberately slow: the Fourier transform
is applied as a dense n x n DFT matrix along each axis, not as an FFT.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------- shift, q
def split_helmholtz(omega: float, c: np.ndarray):
    """Eq. (Dsq) for the Helmholtz case: s = mean of omega^2/c^2, q = s - omega^2/c^2.

    The paper writes s as an integral over the unit torus; on the periodic
    grid the spectrally exact quadrature is the plain mean over J.
    """
    w = (omega * omega) / (np.asarray(c, dtype=np.float64) ** 2)
    s = float(np.mean(w))
    return s, s - w


def split_schrodinger(ell: float, energy: float, V: np.ndarray):
    """Eq. (Dsq) for the rescaled Schroedinger case (eq. schr).

    s = mean of (-ell^2 V + ell^2 E), q = ell^2 V - ell^2 E + s.
    """
    V = np.asarray(V, dtype=np.float64)
    s = float(np.mean(-ell * ell * V + ell * ell * energy))
    return s, ell * ell * V - ell * ell * energy + s


def k_axis(n: int) -> np.ndarray:
    """Fourier indices of K along one axis, in FFT order: r -> r - n [r >= n/2]."""
    r = np.arange(n)
    return r - n * (r >= n // 2)


def k_squared(n: int, d: int) -> np.ndarray:
    """|k|^2 on K, shape (n,)*d, FFT order along every axis."""
    k = k_axis(n).astype(np.float64)
    out = np.zeros((n,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = n
        out = out + (k * k).reshape(shape)
    return out


def shift_distance(n: int, d: int, s: float) -> float:
    """min over K of |4 pi^2 |k|^2 - s| / |s|: how close L - s is to singular."""
    lam = 4.0 * math.pi ** 2 * k_squared(n, d)
    return float(np.min(np.abs(lam - s)) / abs(s))


def perturb_shift(n: int, d: int, s: float, q: np.ndarray, rel_gap: float = 1e-6,
                  step: float = 4.0 * math.pi ** 2 * 1e-3, tries: int = 10):
    """Perturb s until L - s is safely invertible (Section 2.2 assumes it is).

    Reading of the paper's "perturbing s slightly": while the relative gap
    to the nearest eigenvalue 4 pi^2 |k|^2 is below ``rel_gap``, add ``step``
    to s and to q (so L - s + q, the operator being solved, is unchanged).
    Returns (s, q, number_of_perturbations).
    """
    for t in range(tries + 1):
        if shift_distance(n, d, s) >= rel_gap:
            return s, q, t
        if t == tries:
            break
        s = s + step
        q = q + step
    raise ValueError("could not move the shift away from the spectrum of L")


# ---------------------------------------------------------------- DFT
def dft_matrix(n: int) -> np.ndarray:
    """W[k, j] = n^{-1/2} exp(-2 pi i j k / n), rows in FFT order of K (Section 2.1)."""
    k = k_axis(n).astype(np.float64)
    j = np.arange(n, dtype=np.float64)
    return np.exp(-2j * math.pi * np.outer(k, j) / n) / math.sqrt(n)


def idft_matrix(n: int) -> np.ndarray:
    """V[j, k] = n^{-1/2} exp(+2 pi i j k / n) for k in FFT order (Section 2.1)."""
    k = k_axis(n).astype(np.float64)
    j = np.arange(n, dtype=np.float64)
    return np.exp(2j * math.pi * np.outer(j, k) / n) / math.sqrt(n)


def _apply_axes(M: np.ndarray, x: np.ndarray, d: int) -> np.ndarray:
    """Apply the n x n matrix M along each of the last d axes of x."""
    x = np.asarray(x, dtype=np.complex128)
    lead = x.ndim - d
    for ax in range(lead, x.ndim):
        x = np.moveaxis(np.tensordot(M, x, axes=([1], [ax])), 0, ax)
    return x


def fourier(x: np.ndarray, d: int) -> np.ndarray:
    """(F x)_k, the unitary DFT of Section 2.1, over the last d axes."""
    return _apply_axes(dft_matrix(x.shape[-1]), x, d)


def inverse_fourier(y: np.ndarray, d: int) -> np.ndarray:
    """(F^{-1} y)_j over the last d axes."""
    return _apply_axes(idft_matrix(y.shape[-1]), y, d)


def apply_laplacian(u: np.ndarray, d: int) -> np.ndarray:
    """L u with L = F^{-1} diag(4 pi^2 |k|^2) F (Section 2.1)."""
    n = u.shape[-1]
    return inverse_fourier(4.0 * math.pi ** 2 * k_squared(n, d) * fourier(u, d), d)


def green_symbol(n: int, d: int, s: float) -> np.ndarray:
    """sigma_k = 1 / (4 pi^2 |k|^2 - s) on K (eq. G)."""
    return 1.0 / (4.0 * math.pi ** 2 * k_squared(n, d) - s)


def apply_green(v: np.ndarray, d: int, s: float) -> np.ndarray:
    """G v with G = (L - s)^{-1} = F^{-1} diag(sigma) F (eq. G)."""
    n = v.shape[-1]
    return inverse_fourier(green_symbol(n, d, s) * fourier(v, d), d)


def green_kernel(n: int, d: int, s: float) -> np.ndarray:
    """Convolution kernel of G: G[i, j] = g[(i - j) mod n] (eq. G).

    g_m = N^{-1} sum_k sigma_k e^{2 pi i m.k / n} = n^{-d/2} (F^{-1} sigma)_m.
    """
    return inverse_fourier(green_symbol(n, d, s).astype(np.complex128), d) / n ** (d / 2.0)


def apply_differential(u: np.ndarray, d: int, s: float, q: np.ndarray) -> np.ndarray:
    """(L - s + q) u, eq. (Lsq)."""
    return apply_laplacian(u, d) - s * u + q * u


def apply_integral(u: np.ndarray, d: int, s: float, q: np.ndarray) -> np.ndarray:
    """(I + G q) u, the integral reformulation of Section 2.2."""
    return u + apply_green(q * u, d, s)


def dense_differential(n: int, d: int, s: float, q: np.ndarray) -> np.ndarray:
    """The dense N x N matrix of L - s + q (eq. Lsq), C-order unknowns; N <= ~4096."""
    W = dft_matrix(n)
    V = idft_matrix(n)
    Fd = W
    Fi = V
    for _ in range(d - 1):
        Fd = np.kron(Fd, W)
        Fi = np.kron(Fi, V)
    lam = 4.0 * math.pi ** 2 * k_squared(n, d).reshape(-1)
    A = (Fi * lam[None, :]) @ Fd
    A = A - s * np.eye(n ** d) + np.diag(np.asarray(q, dtype=np.float64).reshape(-1))
    return A
