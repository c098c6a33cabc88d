"""Seeded input generators (host side, numpy).

* ``gaussian_random_field`` draws a stationary Gaussian field with covariance
  exp(-r^2 / (2 L^2)) (L in grid cells) by spectral synthesis on a periodic grid
  padded by at least 4L on each axis, then crops it and normalises it to sample
  mean 0 and sample standard deviation ``std``.
* ``lognormal_kappa`` maps such a field g to a cell-centred diffusion
  coefficient kappa = kappa0 * exp(g).
* ``first_block_rhs`` builds b = (b_1, 0, ..., 0) with b_1 ~ N(0, 1), the
  right-hand side structure of the all-at-once system (Section 1, eq. (1);
  Section 5 draws b_1 from the standard normal distribution).

All arrays are float64 and use the block-major layout x[k*N + i] with
i = iy*nx + ix.
"""

from __future__ import annotations

import numpy as np


def gaussian_random_field(nx: int, ny: int, corr_len: float, std: float, seed: int) -> np.ndarray:
    """Return an (ny, nx) float64 field (ny == 1 gives a 1D field)."""
    rng = np.random.default_rng(seed)
    pad = int(np.ceil(4 * corr_len)) + 1
    px = nx + 2 * pad
    py = ny + 2 * pad if ny > 1 else 1
    white = rng.standard_normal((py, px))
    kx = np.fft.fftfreq(px)
    ky = np.fft.fftfreq(py) if py > 1 else np.zeros(1)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    # Spectral density of the squared-exponential covariance (up to a constant,
    # which the final normalisation removes).
    amp = np.exp(-np.pi ** 2 * corr_len ** 2 * k2)
    field = np.fft.ifft2(np.fft.fft2(white) * amp).real
    if ny > 1:
        field = field[pad:pad + ny, pad:pad + nx]
    else:
        field = field[:, pad:pad + nx]
    field = field - field.mean()
    s = field.std()
    if s > 0:
        field = field / s
    return np.ascontiguousarray(field * std)


def lognormal_kappa(nx: int, ny: int, kappa0: float, corr_len: float, std: float, seed: int) -> np.ndarray:
    """Cell-centred coefficient kappa0 * exp(g), flattened row-major (length nx*ny)."""
    g = gaussian_random_field(nx, ny, corr_len, std, seed)
    return np.ascontiguousarray((kappa0 * np.exp(g)).reshape(-1))


def drifting_kappa_blocks(nx: int, ny: int, ell: int, kappa0: float, corr_len: float, std: float, drift: float,
                          seed: int) -> np.ndarray:
    """l coefficient fields kappa_k = kappa0 exp(g + drift (k / l) h), k = 0..l-1, with g, h
    independent Gaussian random fields: a log-normal field whose pattern drifts through
    the time window (drift 0 gives l equal blocks).  Shape (l, nx*ny)."""
    g = gaussian_random_field(nx, ny, corr_len, std, seed).reshape(-1)
    h = gaussian_random_field(nx, ny, corr_len, std, seed + 1).reshape(-1)
    return np.stack([kappa0 * np.exp(g + drift * (k / ell) * h) for k in range(ell)])


def first_block_rhs(n: int, ell: int, seed: int) -> np.ndarray:
    """b = (b_1, 0, ..., 0), b_1 = default_rng(seed).standard_normal(n)."""
    b = np.zeros(ell * n)
    b[:n] = np.random.default_rng(seed).standard_normal(n)
    return b


def random_block_vector(n: int, ell: int, seed: int) -> np.ndarray:
    """A dense N(0,1) block vector of length ell*n (used for operator-level checks)."""
    return np.random.default_rng(seed).standard_normal(ell * n)


def batched_problem_specs(count: int, seed: int = 2026):
    """Uneven batch: grid side from {128, 256, 512, 1024}, ell from {6, 8, 10, 12},
    field std uniform in [0.5, 1.5]; returns a list of dicts (no arrays)."""
    rng = np.random.default_rng(seed)
    sides = rng.choice([128, 256, 512, 1024], size=count)
    ells = rng.choice([6, 8, 10, 12], size=count)
    stds = rng.uniform(0.5, 1.5, size=count)
    seeds = rng.integers(0, 2 ** 31 - 1, size=count)
    return [
        {"nx": int(s), "ny": int(s), "ell": int(e), "std": float(d), "seed": int(z)}
        for s, e, d, z in zip(sides, ells, stds, seeds)
    ]
