"""Fermi-Dirac weights at theta > 0 evaluated in every cell and every step: the
lattice BGK iteration with local weights.  Plain, slow, float64.

TEST INFRASTRUCTURE ONLY.  Nothing under ``oracle/`` belongs to the product
path: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import it.  It shares no code with the HIP library.

The paper makes the lattice weights functions of the weight's moments I_2N and
asks for them to be updated at every time step (section "The Gaussian
quadrature"); for electrons at a temperature theta > 0 the moments follow from
the local chemical potential mu by eq. sommerfeld.  Per step and per cell:

  1. n = sum_a f_a and u0 = sum_a f_a e_a / n;
  2. mu from n: I_0(mu, theta) = kappa n, where kappa fixes the density unit
     (the reference density rho_ref has the chemical potential mu_ref = 1 and
     theta = r0 mu_ref, so kappa = I_0(1, r0) / rho_ref);
  3. the moments I_2N(mu, theta) of eq. sommerfeld, cut after (theta/mu)^2;
  4. the lattice model of those moments (polynomial coefficients, quadrature
     weights, c_0 = sqrt(3 I_4 / I_2)) and f_eq = n w_hat_a S(c_0 e_a, c_0 u0)
     by the tensor expansion (eq. expansao0);
  5. BGK relaxation f* = f - (f - f_eq) / tau;
  6. streaming f_a(x + e_a) = f*_a(x), periodic on every axis.

Reading (the paper does not say how a lattice with a local c_0 streams): the
geometric lattice e_a is fixed and one step moves every population by e_a, so
a cell's velocities are in units of its own c_0; u0 = j / n is the velocity in
those units, and the equilibrium depends on mu only through J_L(theta/mu).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq

from . import theory as th


def I0_sommerfeld(D: int, mu: float, theta: float) -> float:
    return th.moments_sommerfeld(D, mu, theta, nmax=0)[0]


def mu_of_density(D: int, x: float, r0: float) -> float:
    """mu (in units of mu_ref) of a cell whose density is x rho_ref: the root of
    I_0(mu, theta = r0) = x I_0(1, r0), bracketed and solved to full precision."""
    if not x > 0:
        raise ValueError("density must be positive")
    target = x * I0_sommerfeld(D, 1.0, r0)
    if r0 == 0.0:
        return x ** (2.0 / D)
    f = lambda mu: I0_sommerfeld(D, mu, r0) - target
    guess = x ** (2.0 / D)
    lo, hi = 0.5 * guess, 2.0 * guess
    while f(lo) > 0:
        lo *= 0.5
    while f(hi) < 0:
        hi *= 2.0
    return brentq(f, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=200)


def local_moments(D: int, x: float, r0: float) -> dict:
    """The moments I_L of the weight in a cell of density x rho_ref."""
    mu = mu_of_density(D, x, r0)
    return th.moments_sommerfeld(D, mu, r0)


class LocalOracle:
    """Periodic box, Fermi-Dirac weights in the Sommerfeld limit at theta = r0 mu_ref,
    recomputed per cell and step."""

    def __init__(self, lattice: str = "d2v9", shape=(1, 1, 1), tau: float = 0.6, order: int = 2,
                 r0: float = 0.1, rho_ref: float = 1.0):
        self.lattice = lattice
        self.D = th.lattice_dim(lattice)
        self.e = th.velocity_set(lattice)
        self.Q = self.e.shape[0]
        self.shape = tuple((tuple(shape) + (1, 1, 1))[:3])
        self.cells = int(np.prod(self.shape))
        self.tau, self.order, self.r0, self.rho_ref = tau, order, r0, rho_ref

    def model(self, n: float) -> th.LatticeModel:
        return th.model_from_moments(self.lattice, local_moments(self.D, n / self.rho_ref, self.r0))

    def feq(self, n: float, u0) -> np.ndarray:
        return th.feq_tensor(self.model(n), n, u0, self.order)

    def init(self, n0, u0) -> np.ndarray:
        n0 = np.asarray(n0, dtype=np.float64).reshape(-1)
        u0 = np.asarray(u0, dtype=np.float64).reshape(self.D, -1)
        return np.stack([self.feq(n0[c], u0[:, c]) for c in range(self.cells)], axis=1)

    def moments(self, f: np.ndarray):
        n = f.sum(axis=0)
        u = (self.e.T.astype(np.float64) @ f) / n
        return n, u

    def step(self, f: np.ndarray) -> np.ndarray:
        n, u = self.moments(f)
        feq = np.stack([self.feq(n[c], u[:, c]) for c in range(self.cells)], axis=1)
        post = f - (f - feq) / self.tau
        nx, ny, nz = self.shape
        out = np.empty_like(f)
        for a in range(self.Q):
            ev = list(self.e[a]) + [0] * (3 - self.D)
            plane = post[a].reshape(nz, ny, nx)
            out[a] = np.roll(plane, shift=(ev[2], ev[1], ev[0]), axis=(0, 1, 2)).reshape(-1)
        return out

    def run(self, f: np.ndarray, steps: int) -> np.ndarray:
        for _ in range(steps):
            f = self.step(f)
        return f
