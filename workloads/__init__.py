"""Seeded synthetic inputs for the periodic Helmholtz / Schroedinger solves.

This module only draws random media and right-hand sides.  It holds none of
the method's arithmetic (no shift, no Fourier transform, no stencil, no
factorisation): both the CPU oracle and the GPU path take their inputs from
here and from nowhere else.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws in
the order written in its docstring, so a (generator, seed) pair fixes the
arrays bit for bit.  Arrays are laid out in C order (last axis fastest) on
the grid x_j = j h, h = 1/n, j in [0, n)^d (Section 2.1 of the paper).

The paper does not publish its media (Gaussian amplitudes, widths and
positions are not given, Section 3), so these families are stand-ins of the
same kind: smooth Gaussian perturbations of a unit background, delta-like
Gaussian sources, and lattices of Gaussian wells for the Schroedinger case.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 14090297


def seed_for(config: int, instance: int = 0) -> int:
    """Base seed of instance ``instance`` of workload family ``config``."""
    return BASE_SEED + 1000 * config + instance


def grid_points(n: int, d: int) -> np.ndarray:
    """Physical grid coordinates, shape (n,)*d + (d,), x_j = j / n."""
    axes = [np.arange(n, dtype=np.float64) / n] * d
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack(mesh, axis=-1)


def periodic_sq_dist(x: np.ndarray, centre: np.ndarray, period: float = 1.0) -> np.ndarray:
    """Squared distance to the nearest periodic image of ``centre``."""
    delta = x - centre
    delta = delta - period * np.round(delta / period)
    return np.sum(delta * delta, axis=-1)


@dataclasses.dataclass
class HelmholtzMedium:
    n: int
    d: int
    omega: float
    c: np.ndarray          # wave speed c(x_j), real, shape (n,)*d
    amplitudes: np.ndarray
    centres: np.ndarray
    width: float


def gaussian_bump_medium(n: int, d: int, omega: float, bumps: int, width: float,
                         seed: int, amp: float = 0.2) -> HelmholtzMedium:
    """Wave speed with 1/c = 1 + sum_i a_i exp(-|x - x_i|^2_per / (2 width^2)).

    Draw order: a ~ U[-amp, amp]^bumps, then x_i ~ U[0,1)^(bumps x d).
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(-amp, amp, size=bumps)
    centres = rng.uniform(0.0, 1.0, size=(bumps, d))
    x = grid_points(n, d)
    slowness = np.ones((n,) * d)
    for ai, ci in zip(a, centres):
        slowness += ai * np.exp(-periodic_sq_dist(x, ci) / (2.0 * width * width))
    return HelmholtzMedium(n=n, d=d, omega=omega, c=1.0 / slowness,
                           amplitudes=a, centres=centres, width=width)


def gaussian_sources(n: int, d: int, count: int, width: float, seed: int) -> np.ndarray:
    """``count`` Gaussian right-hand sides of peak 1, complex128, (count,)+(n,)*d.

    Draw order: centres x0 ~ U[0,1)^(count x d).
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(count, d))
    x = grid_points(n, d)
    out = np.empty((count,) + (n,) * d, dtype=np.complex128)
    for i in range(count):
        out[i] = np.exp(-periodic_sq_dist(x, centres[i]) / (2.0 * width * width))
    return out


def grid_delta(n: int, d: int, index) -> np.ndarray:
    """Unit grid delta at the multi-index ``index`` (complex128)."""
    f = np.zeros((n,) * d, dtype=np.complex128)
    f[tuple(index)] = 1.0
    return f


@dataclasses.dataclass
class SchrodingerLattice:
    n: int
    d: int
    ell: float
    energy: float
    V: np.ndarray          # V at the physical points ell * x_j, shape (n,)*d
    depths: np.ndarray
    centres: np.ndarray


def gaussian_well_lattice(n: int, d: int, ell: int, seed: int, width: float = 0.1,
                          depth=(5.0, 10.0), jitter: float = 0.05,
                          energy=(1.0, 3.0)) -> SchrodingerLattice:
    """Lattice of Gaussian wells on [0, ell)^d, one well per unit cell.

    V(y) = -sum_i D_i exp(-|y - y_i|^2_per / (2 width^2)), y_i = cell centre +
    jitter.  Draw order: D ~ U[depth]^(ell^d), jitter ~ U[-jitter, jitter]^(ell^d x d),
    then E ~ U[energy].
    """
    rng = np.random.default_rng(seed)
    cells = ell ** d
    D = rng.uniform(depth[0], depth[1], size=cells)
    jit = rng.uniform(-jitter, jitter, size=(cells, d))
    E = float(rng.uniform(energy[0], energy[1]))
    idx = np.stack(np.meshgrid(*([np.arange(ell)] * d), indexing="ij"), axis=-1).reshape(-1, d)
    centres = idx + 0.5 + jit
    # The periodic squared distance is a sum over axes, so each well is a
    # product of one Gaussian factor per axis: V = -sum_i D_i prod_k E_k[i, x_k].
    y = np.arange(n, dtype=np.float64) / n * ell
    factors = []
    for k in range(d):
        delta = y[None, :] - centres[:, k:k + 1]
        delta = delta - float(ell) * np.round(delta / float(ell))
        factors.append(np.exp(-(delta * delta) / (2.0 * width * width)))
    sub = "abcdefgh"[:d]
    V = -np.einsum("i," + ",".join("i" + c for c in sub) + "->" + sub, D, *factors)
    return SchrodingerLattice(n=n, d=d, ell=float(ell), energy=E, V=V, depths=D, centres=centres)


# --------------------------------------------------------------------------
# Named workloads.  Sizes follow the benchmark configurations of the build:
# "parity" is the small case the oracle finishes in seconds, "large2d" the
# single-GPU throughput case.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    kind: str               # "helmholtz" | "schrodinger" | "maxwell"
    n: int
    d: int
    b: int
    omega: float = 0.0
    ell: float = 1.0
    energy: float = 0.0
    coeff: np.ndarray = None     # c(x_j), V(ell x_j) or eps(x_j)
    rhs: np.ndarray = None       # (nrhs,)+(n,)*d complex128; Maxwell: (nrhs, d)+(n,)*d
    tol: float = 1e-10


def helmholtz_workload(name: str, config: int, n: int, d: int, waves: float, bumps: int,
                       width: float, b: int, nrhs: int = 1, src_width: float = 1.0 / 32,
                       tol: float = 1e-10, instance: int = 0) -> Workload:
    omega = 2.0 * math.pi * waves
    med = gaussian_bump_medium(n, d, omega, bumps, width, seed_for(config, instance))
    rhs = gaussian_sources(n, d, nrhs, src_width, seed_for(config, instance) + 500)
    return Workload(name=name, kind="helmholtz", n=n, d=d, b=b, omega=omega,
                    coeff=med.c, rhs=rhs, tol=tol)


def parity_2d(nrhs: int = 1) -> Workload:
    """2D Helmholtz, 64^2 grid, omega = 2 pi 8, 8 bumps of width 0.05, b = 8."""
    return helmholtz_workload("helmholtz2d_n64_w8", 1, 64, 2, 8.0, 8, 0.05, 8, nrhs=nrhs, tol=1e-10)


def large_2d(nrhs: int = 1) -> Workload:
    """2D Helmholtz, 512^2 grid, omega = 2 pi 64, 64 bumps of width 0.05, b = 16."""
    return helmholtz_workload("helmholtz2d_n512_w64", 2, 512, 2, 64.0, 64, 0.05, 16, nrhs=nrhs, tol=1e-8)


def large_2d_delta() -> Workload:
    """The 512^2 medium of ``large_2d`` driven by a unit grid delta at the
    centre j = (n/2, n/2), the source of the paper's examples (Section 3).
    A delta excites the propagating band |k| ~ omega / (2 pi) fully, so the
    solution is a field radiating through the whole domain (the Gaussian of
    ``large_2d`` has no content there and its solution stays local)."""
    W = large_2d()
    W.name = "helmholtz2d_n512_w64_delta"
    W.rhs = grid_delta(W.n, W.d, (W.n // 2, W.n // 2))[None]
    return W


def helmholtz_3d(n: int = 128, b: int = 8, nrhs: int = 4) -> Workload:
    """3D Helmholtz on [0,1)^3 at 8 points per wavelength (omega = 2 pi n / 8),
    32 Gaussian bumps of width 0.06 and amplitude U[-0.2, 0.2] in 1/c, nrhs
    Gaussian sources of width 1/32 at seeded points; n = 128, b = 8 is the 3D
    configuration (8^3 leaf boxes, one wavelength wide); smaller n keep the
    same points per wavelength and leaf width in wavelengths when b = n / 16."""
    return helmholtz_workload(f"helmholtz3d_n{n}_w{n // 8}", 3, n, 3, n / 8.0, 32, 0.06, b,
                              nrhs=nrhs, tol=1e-8)


def small(n: int, d: int, b: int, waves: float, bumps: int = 4, width: float = 0.08,
          nrhs: int = 1, instance: int = 0, tol: float = 1e-10) -> Workload:
    """Small Helmholtz case for unit tests (any n, d, b)."""
    return helmholtz_workload(f"helmholtz{d}d_n{n}_b{b}", 9, n, d, waves, bumps, width, b,
                              nrhs=nrhs, tol=tol, instance=instance)


def maxwell_workload(n: int, d: int, b: int, waves: float, bumps: int = 4, width: float = 0.08,
                     nrhs: int = 1, instance: int = 0, config: int = 10, tol: float = 1e-10) -> Workload:
    """Maxwell (curl-curl) case: permittivity eps = 1 / c^2 of the Gaussian-bump
    medium of ``gaussian_bump_medium`` (so omega^2 eps is the Helmholtz
    omega^2 / c^2 of the same draw), omega = 2 pi waves; right-hand sides are
    vector fields, shape (nrhs, d) + (n,)*d, every component an independent
    Gaussian of width 1/32 (the d nrhs Gaussians of one ``gaussian_sources``
    draw, right-hand side major)."""
    omega = 2.0 * math.pi * waves
    med = gaussian_bump_medium(n, d, omega, bumps, width, seed_for(config, instance))
    rhs = gaussian_sources(n, d, nrhs * d, 1.0 / 32, seed_for(config, instance) + 500)
    return Workload(name=f"maxwell{d}d_n{n}_b{b}", kind="maxwell", n=n, d=d, b=b, omega=omega,
                    coeff=1.0 / med.c ** 2, rhs=rhs.reshape((nrhs, d) + (n,) * d), tol=tol)


def schrodinger_workload(n: int, d: int, ell: int, b: int, nrhs: int = 1, instance: int = 0,
                         config: int = 4, tol: float = 1e-8) -> Workload:
    lat = gaussian_well_lattice(n, d, ell, seed_for(config, instance))
    rhs = gaussian_sources(n, d, nrhs, 1.0 / 32, seed_for(config, instance) + 500)
    return Workload(name=f"schrodinger{d}d_n{n}_l{ell}", kind="schrodinger", n=n, d=d, b=b,
                    ell=float(ell), energy=lat.energy, coeff=lat.V, rhs=rhs, tol=tol)


def schrodinger_paper(n: int, d: int, example: str, seed: int = 0) -> Workload:
    """Stand-in for the paper's Schroedinger examples (Section 3.2): ell = n
    (one grid step per unit of the potential's length scale), E = 2.5 (about
    4 points per wavelength), a unit grid delta at the centre.  The paper
    describes its potentials only in words, so these are of the same kind:
    V(y) = -sum_i D_i exp(-|y - y_i|^2_per / (2 * 1.5^2)) on [0, n)^d with one
    well per 8^d cell of the domain.  example "random": the (n/8)^d wells at
    uniformly random positions, D_i ~ U[1, 2] (draw order: positions, then
    depths); "vacancy": the wells at the cell centres 8 i + 4, D_i = 1.5, the
    one nearest the domain centre left out."""
    rng = np.random.default_rng(seed_for(6, seed))
    cells = (n // 8) ** d
    if example == "random":
        centres = rng.uniform(0.0, float(n), size=(cells, d))
        D = rng.uniform(1.0, 2.0, size=cells)
    elif example == "vacancy":
        idx = np.stack(np.meshgrid(*([np.arange(n // 8)] * d), indexing="ij"), axis=-1).reshape(-1, d)
        centres = 8.0 * idx + 4.0
        far = np.argmin(np.sum((centres - n / 2.0) ** 2, axis=1))
        centres = np.delete(centres, far, axis=0)
        D = np.full(len(centres), 1.5)
    else:
        raise ValueError(example)
    y = np.arange(n, dtype=np.float64)
    factors = []
    for k in range(d):
        delta = y[None, :] - centres[:, k:k + 1]
        delta = delta - float(n) * np.round(delta / float(n))
        factors.append(np.exp(-(delta * delta) / (2.0 * 1.5 * 1.5)))
    sub = "abcdefgh"[:d]
    V = -np.einsum("i," + ",".join("i" + c for c in sub) + "->" + sub, D, *factors)
    rhs = grid_delta(n, d, (n // 2,) * d)[None]
    return Workload(name=f"schrodinger{d}d_paper_{example}_n{n}", kind="schrodinger", n=n, d=d, b=0,
                    ell=float(n), energy=2.5, coeff=V, rhs=rhs, tol=1e-6)


def schrodinger_batch(nrhs: int = 16, per_size: int = 16) -> list:
    """Batched 2D Schroedinger family: per_size instances each of n = 128, 192
    and 256 (ell = n / 8 unit cells per side, so 8 grid points per cell; boxes
    of b = n / 16, so every instance has a 16 x 16 leaf grid and the same tree
    depth), instance i of size n_i = (128, 192, 256)[i % 3], with its own
    well lattice, energy and nrhs Gaussian sources."""
    out = []
    for i in range(3 * per_size):
        n = (128, 192, 256)[i % 3]
        out.append(schrodinger_workload(n, 2, n // 8, n // 16, nrhs=nrhs, instance=i, config=4))
    return out
