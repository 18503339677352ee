"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no part of the transform's arithmetic: it only draws random
numbers and shapes them like the grids a plane-wave electronic-structure code
hands to its 3D FFTs (the application of Section I and Section III of the
paper).  Both the GPU path and the CPU oracle receive the very same arrays.

Conventions (every generator):
* numpy ``default_rng(seed)`` (PCG64); real parts are drawn before imaginary
  parts, each as one C-order block;
* values are generated in float64 and cast to complex64 (the FP32 path's
  input type); the oracle is always given the cast values;
* layout [batch][z][y][x], x contiguous.

Recipes:
* ``uniform_grid`` -- Re, Im i.i.d. U[-1, 1].
* ``sphere_grid`` -- plane-wave coefficients: with the signed frequency
  G_d = k_d for k_d < N_d/2 and k_d - N_d otherwise, the coefficient is
  non-zero only strictly inside the sphere |G|^2 < (N/4)^2, where it is
  (a + i b) * exp(-|G|^2 / (N/8)^2) with a, b i.i.d. N(0, 1); N is the
  smallest grid dimension.
* ``smooth_potential`` -- a real, smooth periodic potential
  V(r) = sum_{j<16} a_j cos(2 pi G_j . (x/Nx, y/Ny, z/Nz) + phi_j) with
  G_j drawn from {-2..2}^3 minus the origin, a_j ~ U[0.5, 1.5],
  phi_j ~ U[0, 2 pi); returned as float32.
"""
from __future__ import annotations

import numpy as np


def _shape(n, batch):
    if isinstance(n, int):
        nx = ny = nz = n
    else:
        nx, ny, nz = n
    return (batch, nz, ny, nx) if batch is not None else (nz, ny, nx)


def uniform_grid(n, seed: int, batch=None) -> np.ndarray:
    """Complex64 grid with Re, Im i.i.d. uniform on [-1, 1]."""
    shape = _shape(n, batch)
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=shape)
    im = rng.uniform(-1.0, 1.0, size=shape)
    return (re + 1j * im).astype(np.complex64)


def signed_freq(n: int) -> np.ndarray:
    k = np.arange(n)
    return np.where(k < n / 2.0, k, k - n).astype(np.float64)


def sphere_mask_and_envelope(n):
    """(mask, envelope) on the [z, y, x] grid for the sphere-cutoff recipe."""
    nz, ny, nx = _shape(n, None)
    nmin = min(nx, ny, nz)
    gz = signed_freq(nz)[:, None, None]
    gy = signed_freq(ny)[None, :, None]
    gx = signed_freq(nx)[None, None, :]
    g2 = gx * gx + gy * gy + gz * gz
    mask = g2 < (nmin / 4.0) ** 2
    env = np.exp(-g2 / (nmin / 8.0) ** 2) * mask
    return mask, env


def sphere_grid(n, seed: int) -> np.ndarray:
    """One complex64 [z, y, x] grid of sphere-cutoff plane-wave coefficients."""
    shape = _shape(n, None)
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(size=shape)
    im = rng.standard_normal(size=shape)
    _, env = sphere_mask_and_envelope(n)
    return ((re + 1j * im) * env).astype(np.complex64)


def sphere_batch(n, seeds) -> np.ndarray:
    """[len(seeds), z, y, x] complex64 batch, grid j drawn with seeds[j]."""
    seeds = list(seeds)
    nz, ny, nx = _shape(n, None)
    out = np.empty((len(seeds), nz, ny, nx), dtype=np.complex64)
    for j, s in enumerate(seeds):
        out[j] = sphere_grid(n, s)
    return out


def smooth_potential(n, seed: int, terms: int = 16) -> np.ndarray:
    """Real float32 [z, y, x] potential: a sum of low-|G| cosines."""
    nz, ny, nx = _shape(n, None)
    rng = np.random.default_rng(seed)
    G = []
    while len(G) < terms:
        g = rng.integers(-2, 3, size=3)
        if np.any(g != 0):
            G.append(g)
    amp = rng.uniform(0.5, 1.5, size=terms)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=terms)
    z = np.arange(nz)[:, None, None] / nz
    y = np.arange(ny)[None, :, None] / ny
    x = np.arange(nx)[None, None, :] / nx
    V = np.zeros((nz, ny, nx), dtype=np.float64)
    for j in range(terms):
        gx, gy, gz = (float(v) for v in G[j])
        V += amp[j] * np.cos(2.0 * np.pi * (gx * x + gy * y + gz * z) + phase[j])
    return V.astype(np.float32)


# Seeds of the named workloads (one place, used by tests and the bench).
SEED_SMALL_UNIFORM = 1001          # single 16^3 grid, uniform entries
SEED_SINGLE = {64: 2064, 128: 2128}  # single 64^3 / 128^3 sphere grids
SEED_BATCH128 = 3000               # 32 x 128^3 batch: seeds 3000 + j
SEED_BATCH64 = 4000                # 256 x 64^3 batch: seeds 4000 + j
SEED_MIXED = 4500                  # mixed grids: seed 4500 + N
SEED_ORBITALS = 5000               # 128 x 96^3 orbitals: seeds 5000 + n
SEED_POTENTIAL = 5999              # the smooth potential V
MIXED_SIZES = (48, 72, 96, 100, 120)
