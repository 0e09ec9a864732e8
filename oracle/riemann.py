"""Exact solutions of the one-dimensional Riemann problem for a barotropic gas
(TEST INFRASTRUCTURE ONLY).

Written from the conservation laws of mass and momentum,
    d_t n + d_x (n u) = 0,   d_t (n u) + d_x (n u^2 + P(n)) = 0,
for two pressure laws:

* isothermal, P = a^2 n.  The lattice scheme of the paper has the pressure
  tensor n (J_2 / 3) delta + n u0 u0 in lattice units, i.e. an isothermal gas
  with a^2 = J_2 / 3; the paper compares its Riemann runs with an isothermal
  solver (section "Numerical simulations for electrons in metals").
* gamma law, P = K n^gamma.  The zero-temperature Fermi gas has
  P proportional to n^((D+2)/D), i.e. gamma = 2 in D = 2.

Each side is joined to the middle state by a shock (n* > n_K, Rankine-Hugoniot
jump conditions) or a rarefaction fan (n* <= n_K, constant Riemann invariant
along the fan).  Velocities are in cells per step and positions in cells when
used with lattice runs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.optimize import brentq


@dataclass
class PressureLaw:
    kind: str          # "isothermal" or "gamma"
    a2: float = 0.0    # isothermal: P = a2 n
    K: float = 0.0     # gamma law:  P = K n^gamma
    gamma: float = 2.0

    def P(self, n):
        return self.a2 * n if self.kind == "isothermal" else self.K * np.power(n, self.gamma)

    def c(self, n):
        if self.kind == "isothermal":
            return math.sqrt(self.a2) * np.ones_like(np.asarray(n, dtype=float))
        return np.sqrt(self.gamma * self.K * np.power(n, self.gamma - 1.0))


def isothermal(a2: float) -> PressureLaw:
    return PressureLaw("isothermal", a2=a2)


def gamma_law(K: float, gamma: float) -> PressureLaw:
    return PressureLaw("gamma", K=K, gamma=gamma)


def _wave_function(law: PressureLaw, n: float, nK: float) -> float:
    """Velocity change across the wave joining state K to density n."""
    if n > nK:  # shock
        return math.sqrt((law.P(n) - law.P(nK)) * (n - nK) / (n * nK))
    if law.kind == "isothermal":
        return math.sqrt(law.a2) * math.log(n / nK)
    g = law.gamma
    cK = float(law.c(nK))
    return 2.0 * cK / (g - 1.0) * ((n / nK) ** ((g - 1.0) / 2.0) - 1.0)


@dataclass
class RiemannSolution:
    law: PressureLaw
    nL: float
    uL: float
    nR: float
    uR: float
    n_star: float
    u_star: float

    # wave speeds -----------------------------------------------------------
    def left_speeds(self):
        """(head, tail) of the left fan, or (s, s) for a left shock."""
        if self.n_star > self.nL:
            s = (self.n_star * self.u_star - self.nL * self.uL) / (self.n_star - self.nL)
            return s, s
        return self.uL - float(self.law.c(self.nL)), self.u_star - float(self.law.c(self.n_star))

    def right_speeds(self):
        """(tail, head) of the right fan, or (s, s) for a right shock."""
        if self.n_star > self.nR:
            s = (self.n_star * self.u_star - self.nR * self.uR) / (self.n_star - self.nR)
            return s, s
        return self.u_star + float(self.law.c(self.n_star)), self.uR + float(self.law.c(self.nR))

    # sampling --------------------------------------------------------------
    def sample(self, xi):
        """Density and velocity at the self-similar coordinate xi = x / t."""
        xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
        n = np.empty_like(xi)
        u = np.empty_like(xi)
        law = self.law
        lh, lt = self.left_speeds()
        rt, rh = self.right_speeds()
        for k, s in enumerate(xi):
            if s <= self.u_star:
                if s < lh:
                    n[k], u[k] = self.nL, self.uL
                elif s >= lt:
                    n[k], u[k] = self.n_star, self.u_star
                else:  # inside the left fan, where u - c(n) = s
                    n[k], u[k] = self._fan(s, left=True)
            else:
                if s > rh:
                    n[k], u[k] = self.nR, self.uR
                elif s <= rt:
                    n[k], u[k] = self.n_star, self.u_star
                else:  # inside the right fan, where u + c(n) = s
                    n[k], u[k] = self._fan(s, left=False)
        return n, u

    def _fan(self, s, left: bool):
        law = self.law
        if law.kind == "isothermal":
            a = math.sqrt(law.a2)
            if left:   # u + a ln n is constant
                u = s + a
                return self.nL * math.exp((self.uL - u) / a), u
            u = s - a  # u - a ln n is constant
            return self.nR * math.exp((u - self.uR) / a), u
        g = law.gamma
        if left:       # u + 2 c / (g - 1) is constant
            cL = float(law.c(self.nL))
            c = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * (self.uL - s))
            u = s + c
            return self.nL * (c / cL) ** (2.0 / (g - 1.0)), u
        cR = float(law.c(self.nR))
        c = 2.0 / (g + 1.0) * (cR - 0.5 * (g - 1.0) * (self.uR - s))
        u = s - c
        return self.nR * (c / cR) ** (2.0 / (g - 1.0)), u


def solve(law: PressureLaw, nL: float, uL: float, nR: float, uR: float) -> RiemannSolution:
    """Middle state of the Riemann problem: f_L(n*) + f_R(n*) + uR - uL = 0."""
    F = lambda n: _wave_function(law, n, nL) + _wave_function(law, n, nR) + uR - uL
    lo, hi = 1e-12 * min(nL, nR), 10.0 * max(nL, nR)
    while F(hi) < 0.0:
        hi *= 10.0
    n_star = brentq(F, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500)
    u_star = 0.5 * (uL + uR) + 0.5 * (_wave_function(law, n_star, nR) - _wave_function(law, n_star, nL))
    return RiemannSolution(law, nL, uL, nR, uR, n_star, u_star)
