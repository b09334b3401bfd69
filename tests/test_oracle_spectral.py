"""Pins for the oracle's discretisation (Section 2.1) and Green operator (eq. G).

Each check ties the oracle to something outside itself: numpy's FFT, the
analytic Laplacian of band-limited functions, closed forms for single
Fourier modes, and the algebraic identities the paper states.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import spectral


@pytest.mark.parametrize("n", [4, 6, 16])
def test_dft_matches_numpy_fft(n):
    """F is numpy's orthonormal FFT; rows follow K's FFT order (Section 2.1)."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    np.testing.assert_allclose(spectral.fourier(x, 2), np.fft.fftn(x, norm="ortho"), atol=1e-12)
    np.testing.assert_allclose(spectral.inverse_fourier(x, 2), np.fft.ifftn(x, norm="ortho"), atol=1e-12)
    W = spectral.dft_matrix(n)
    np.testing.assert_allclose(W @ W.conj().T, np.eye(n), atol=1e-13)


def test_k_grid_includes_negative_nyquist():
    """K = {-n/2 <= k < n/2} (Section 2.1), stored in FFT order."""
    for n in (4, 8, 10):
        k = spectral.k_axis(n)
        assert sorted(k.tolist()) == list(range(-n // 2, n // 2))
        assert k[n // 2] == -n // 2


@pytest.mark.parametrize("d", [1, 2, 3])
def test_fourier_mode_is_eigenvector_of_L(d):
    """L e_k = 4 pi^2 |k|^2 e_k for a single plane wave (Section 2.1)."""
    n = 8
    x = workloads.grid_points(n, d)
    for k0 in [(1,) * d, tuple(range(-2, -2 + d)), (3,) + (0,) * (d - 1)]:
        k0 = np.array(k0, dtype=np.float64)
        e = np.exp(2j * math.pi * (x @ k0))
        np.testing.assert_allclose(spectral.apply_laplacian(e, d),
                                   4 * math.pi ** 2 * (k0 @ k0) * e, atol=1e-9)


def test_laplacian_of_trig_polynomial_is_exact():
    """Spectral differentiation is exact on band-limited functions."""
    n = 16
    x = workloads.grid_points(n, 2)
    u = np.sin(2 * math.pi * 3 * x[..., 0]) * np.cos(2 * math.pi * 5 * x[..., 1]) + 0.3
    minus_lap = 4 * math.pi ** 2 * (9 + 25) * (u - 0.3)
    np.testing.assert_allclose(spectral.apply_laplacian(u, 2).real, minus_lap, atol=1e-9)


def test_green_inverts_shifted_laplacian():
    """G = (L - s)^{-1} (eq. G): G (L - s) v = v and (L - s) G v = v."""
    n, d, s = 12, 2, 4 * math.pi ** 2 * 7.3
    rng = np.random.default_rng(2)
    v = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Lv = spectral.apply_laplacian(v, d) - s * v
    np.testing.assert_allclose(spectral.apply_green(Lv, d, s), v, atol=1e-10)
    Gv = spectral.apply_green(v, d, s)
    np.testing.assert_allclose(spectral.apply_laplacian(Gv, d) - s * Gv, v, atol=1e-10)


def test_green_of_plane_wave_closed_form():
    """G e_k = e_k / (4 pi^2 |k|^2 - s) (eq. G)."""
    n, d, s = 16, 2, 1234.5
    x = workloads.grid_points(n, d)
    k0 = np.array([3.0, -5.0])
    e = np.exp(2j * math.pi * (x @ k0))
    np.testing.assert_allclose(spectral.apply_green(e, d, s), e / (4 * math.pi ** 2 * 34 - s), atol=1e-14)


def test_green_kernel_is_columns_of_G_and_real_even():
    """G[i, j] = g[(i - j) mod n]; g is real and even for real s."""
    n, d, s = 10, 2, 2000.0
    g = spectral.green_kernel(n, d, s)
    for j in [(0, 0), (3, 7), (9, 1)]:
        col = spectral.apply_green(workloads.grid_delta(n, d, j), d, s)
        np.testing.assert_allclose(np.roll(g, shift=j, axis=(0, 1)), col, atol=1e-15)
    assert np.abs(g.imag).max() < 1e-15
    np.testing.assert_allclose(g, np.roll(np.flip(g, axis=(0, 1)), 1, axis=(0, 1)), atol=1e-15)


def test_helmholtz_split_preserves_operator_and_has_zero_mean():
    """Eq. (Dsq): -s + q = -omega^2/c^2 pointwise; with the discrete mean, mean(q) = 0."""
    W = workloads.parity_2d()
    s, q = spectral.split_helmholtz(W.omega, W.coeff)
    np.testing.assert_allclose(-s + q, -W.omega ** 2 / W.coeff ** 2, rtol=1e-14)
    assert abs(q.mean()) < 1e-10 * s
    s1, q1 = spectral.split_helmholtz(3.0, np.full((4, 4), 2.0))
    assert s1 == pytest.approx(9.0 / 4.0) and np.abs(q1).max() == 0


def test_schrodinger_split_preserves_operator():
    """Eq. (schr) + (Dsq): -s + q = ell^2 V - ell^2 E."""
    lat = workloads.gaussian_well_lattice(32, 2, 4, seed=5)
    s, q = spectral.split_schrodinger(lat.ell, lat.energy, lat.V)
    np.testing.assert_allclose(-s + q, lat.ell ** 2 * lat.V - lat.ell ** 2 * lat.energy,
                               rtol=1e-12, atol=1e-9)
    assert s == pytest.approx(lat.ell ** 2 * (lat.energy - lat.V.mean()))


def test_shift_on_eigenvalue_is_perturbed():
    """A constant medium with omega = 2 pi 8 puts s on 4 pi^2 |k|^2 = 4 pi^2 64 (Section 2.2)."""
    n, d = 32, 2
    s, q = spectral.split_helmholtz(2 * math.pi * 8, np.ones((n, n)))
    assert spectral.shift_distance(n, d, s) < 1e-12
    s2, q2, moves = spectral.perturb_shift(n, d, s, q)
    assert moves == 1 and spectral.shift_distance(n, d, s2) > 1e-6
    np.testing.assert_allclose(-s2 + q2, -s + q, atol=1e-9)


def test_dense_operator_matches_apply_and_is_symmetric():
    """The dense L - s + q equals its matrix-free form, and is real symmetric."""
    n, d = 8, 2
    rng = np.random.default_rng(3)
    q = rng.standard_normal((n, n))
    A = spectral.dense_differential(n, d, 17.0, q)
    v = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    np.testing.assert_allclose((A @ v.reshape(-1)).reshape(n, n),
                               spectral.apply_differential(v, d, 17.0, q), atol=1e-9)
    assert np.abs(A.imag).max() < 1e-10
    np.testing.assert_allclose(A, A.T, atol=1e-10)
