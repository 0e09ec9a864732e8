"""Seeded synthetic inputs shared by the product, the oracle runs and the tests.

This module holds no arithmetic of the method: it only draws fields and
parameters.  Every draw uses numpy's PCG64 generator from an explicit seed, in
float64.

* gaussian_random_field: white noise smoothed by a periodic Gaussian filter
  exp(-|k|^2 l^2 / 2) in Fourier space, normalised to zero mean and unit
  standard deviation (the perturbed-field workloads).
* riemann_step: a density step (left / right), zero velocity, on nx x ny cells.
* tube_draws: parameters of a batch of shock tubes (length log-uniform,
  density ratio and relaxation time uniform).
"""
from __future__ import annotations

import math

import numpy as np


def gaussian_random_field(shape, corr_len: float, seed: int = 0) -> np.ndarray:
    """Periodic Gaussian random field of the given shape (x fastest: shape is
    (nz, ny, nx) or (ny, nx)), zero mean, unit standard deviation."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    spec = np.fft.fftn(noise)
    k2 = np.zeros(shape)
    for axis, n in enumerate(shape):
        k = 2.0 * math.pi * np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[axis] = n
        k2 = k2 + (k.reshape(sh)) ** 2
    field = np.real(np.fft.ifftn(spec * np.exp(-0.5 * k2 * corr_len ** 2)))
    field -= field.mean()
    sd = field.std()
    return field / sd if sd > 0 else field


def perturbed_field(shape, amplitude: float, corr_len: float, drift, seed: int = 0):
    """n = 1 + amplitude G, u0 uniform = drift (a D-vector); returns float64
    arrays n [cells] and u0 [D, cells] in x-fastest order."""
    G = gaussian_random_field(shape, corr_len, seed)
    n = 1.0 + amplitude * G.reshape(-1)
    D = len(drift)
    u = np.empty((D, n.size))
    for d in range(D):
        u[d] = drift[d]
    return n, u


def riemann_step(nx: int, ny: int, n_left: float, n_right: float, left_cells: int | None = None, D: int = 2):
    """Density n_left for x < left_cells (default nx/2) and n_right beyond, on every
    row; velocity zero.  Returns n [ny*nx], u0 [D, ny*nx]."""
    if left_cells is None:
        left_cells = nx // 2
    x = np.arange(nx)
    n = np.tile(np.where(x < left_cells, n_left, n_right), ny).astype(np.float64)
    return n, np.zeros((D, n.size))


def tube_draws(count: int, seed: int, nx_range=(256, 8192), ratio_range=(0.5, 0.95),
               tau_range=(0.51, 1.0)):
    """Shock-tube parameters: nx = round(exp(U[ln a, ln b])), n_right / n_left ~ U,
    tau ~ U.  Returns a dict of arrays (nx, n_left, n_right, tau)."""
    rng = np.random.default_rng(seed)
    lo, hi = math.log(nx_range[0]), math.log(nx_range[1])
    nx = np.rint(np.exp(rng.uniform(lo, hi, count))).astype(np.int64)
    ratio = rng.uniform(ratio_range[0], ratio_range[1], count)
    tau = rng.uniform(tau_range[0], tau_range[1], count)
    return {"nx": nx, "n_left": np.ones(count), "n_right": ratio, "tau": tau}


def porous_obstacles(shape, count: int, radius: float, seed: int = 0):
    """Solid mask of `count` discs (2D) or balls (3D) of the given radius at
    uniformly drawn centres, periodic in every axis: a cell is solid when its
    distance to a centre is at most `radius`.  shape = (nx, ny) or (nx, ny, nz);
    returns a bool array [ny][nx] or [nz][ny][nx]."""
    rng = np.random.default_rng(seed)
    dims = tuple(int(v) for v in shape)
    D = len(dims)
    centres = rng.uniform(0.0, 1.0, (count, D)) * np.array(dims)
    grids = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")  # [nx][ny](...)
    solid = np.zeros(dims, dtype=bool)
    for c in centres:
        d2 = np.zeros(dims)
        for k in range(D):
            dk = np.abs(grids[k] - c[k])
            dk = np.minimum(dk, dims[k] - dk)
            d2 += dk * dk
        solid |= d2 <= radius * radius
    return solid.transpose(tuple(range(D - 1, -1, -1)))  # x fastest
