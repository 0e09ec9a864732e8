"""Pins of the local-weight oracle (Fermi-Dirac weights at theta > 0 recomputed per
cell and step), each against a fact that does not come from the oracle itself:
the exact Fermi-Dirac moments (the truncated Sommerfeld series must agree with
them to the next term of the series), the zero-temperature closed forms, the
constant-weight C oracle at theta = 0, conservation, and the sound speed that
a density-dependent pressure n J_2(n) / 3 implies."""
import math

import numpy as np
import pytest

from oracle import theory as th
from oracle.lbm import Oracle
from oracle.local_weights import LocalOracle, local_moments, mu_of_density


@pytest.mark.parametrize("D", [1, 2, 3])
def test_sommerfeld_moments_at_zero_temperature_are_the_closed_form(D):
    for mu in (0.5, 1.0, 2.5):
        a, b = th.moments_sommerfeld(D, mu, 0.0), th.moments_fd_t0(D, mu)
        for L in a:
            assert a[L] == pytest.approx(b[L], rel=1e-15)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_sommerfeld_moments_agree_with_the_exact_integrals_to_the_next_term(D):
    """Against the radial integral of the Fermi-Dirac weight itself (pinned to the
    polylogarithm elsewhere): the difference is the series' next term
    (7 pi^4 / 360) nu (nu-1) (nu-2) (nu-3) (theta/mu)^4, nu = N + D/2."""
    mu = 1.3
    for r in (1 / 20, 1 / 40):
        theta = r * mu
        exact = th.moments_quantum(D, math.exp(mu / theta), theta=theta, sign=+1)
        somm = th.moments_sommerfeld(D, mu, theta)
        for N in range(5):
            nu = N + D / 2
            nxt = 7 * math.pi ** 4 / 360 * nu * (nu - 1) * (nu - 2) * (nu - 3) * r ** 4
            rem = exact[2 * N] / somm[2 * N] - 1
            assert abs(rem - nxt) <= 0.1 * abs(nxt) + 1e-8, (N, r, rem, nxt)


def test_chemical_potential_is_linear_in_density_in_two_dimensions():
    """D = 2: I_0 = 2 pi mu exactly (nu (nu - 1) = 0 for N = 0), so mu / mu_ref = n / rho_ref."""
    for x in (0.5, 0.97, 1.0, 1.3):
        for r0 in (0.0, 0.1, 0.3):
            assert mu_of_density(2, x, r0) == pytest.approx(x, rel=1e-14)


@pytest.mark.parametrize("D", [1, 3])
def test_chemical_potential_solves_the_density_relation(D):
    for r0 in (0.05, 0.2):
        for x in (0.8, 1.0, 1.25):
            mu = mu_of_density(D, x, r0)
            h = D / 2
            a0 = math.pi ** 2 / 6 * h * (h - 1)
            lhs = mu ** h * (1 + a0 * (r0 / mu) ** 2)
            assert lhs == pytest.approx(x * (1 + a0 * r0 ** 2), rel=1e-13)
        assert mu_of_density(D, 1.0, r0) == pytest.approx(1.0, rel=1e-14)
    assert mu_of_density(D, 1.7, 0.0) == pytest.approx(1.7 ** (2 / D), rel=1e-15)


def test_local_J_at_reference_density_and_its_trend():
    """At theta / mu = r the truncated series gives J_2 = J_2(0) B_1^2 / (B_0 B_2) with
    B_N = 1 + (pi^2/6) nu (nu - 1) r^2; denser cells (larger mu) are colder in units of mu
    and move toward the zero-temperature value 1 + 2/(D + 2)."""
    D, r0 = 2, 0.15
    I = local_moments(D, 1.0, r0)
    B = [1 + math.pi ** 2 / 6 * (N + 1) * N * r0 ** 2 for N in range(3)]
    assert th.J(I, 2) == pytest.approx((1 + 2 / (D + 2)) * B[1] ** 2 / (B[0] * B[2]), rel=1e-14)
    j = [th.J(local_moments(D, x, r0), 2) for x in (0.8, 1.0, 1.5, 4.0)]
    assert j[0] < j[1] < j[2] < j[3] < 1.5


def test_zero_temperature_is_the_constant_weight_run():
    """theta = 0: every cell has the zero-temperature weights, so the run is the C
    oracle's constant-weight run."""
    nx, ny = 8, 6
    rng = np.random.default_rng(0)
    n0 = 1 + 0.02 * rng.standard_normal(nx * ny)
    u0 = 0.03 * rng.standard_normal((2, nx * ny))
    for order in (2, 3):
        loc = LocalOracle("d2v9", (nx, ny, 1), tau=0.7, order=order, r0=0.0)
        f = loc.run(loc.init(n0, u0), 4)
        ref = Oracle("d2v9", shape=(nx, ny, 1), tau=0.7, order=order)
        g = ref.run(ref.init(n0, u0), 4)
        np.testing.assert_allclose(f, g, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("lattice,shape", [("d1v3", (12, 1, 1)), ("d2v9", (8, 6, 1)), ("d3v19", (4, 3, 3))])
def test_local_run_conserves_mass_and_momentum(lattice, shape):
    loc = LocalOracle(lattice, shape, tau=0.8, order=2, r0=0.2)
    rng = np.random.default_rng(1)
    cells = int(np.prod(shape))
    f = loc.init(1 + 0.05 * rng.standard_normal(cells), 0.02 * rng.standard_normal((loc.D, cells)))
    e = loc.e.astype(np.float64)
    m0, p0 = f.sum(), (f.T @ e).sum(axis=0)
    f = loc.run(f, 3)
    assert f.sum() == pytest.approx(m0, rel=1e-14)
    np.testing.assert_allclose((f.T @ e).sum(axis=0), p0, atol=1e-13 * m0)


def test_rest_state_is_stationary():
    loc = LocalOracle("d2v9", (5, 4, 1), tau=0.6, order=3, r0=0.25, rho_ref=1.0)
    f0 = loc.init(np.full(20, 1.3), np.zeros((2, 20)))
    np.testing.assert_allclose(loc.run(f0.copy(), 2), f0, rtol=1e-14, atol=1e-16)


def _J2(x, r0):
    return th.J(local_moments(2, x, r0), 2)


def test_sound_speed_follows_the_local_pressure():
    """A standing sound wave on a uniform state: with weights that follow the local
    density the pressure in lattice units is P(n) = n J_2(n) / 3, so the wave
    travels at c^2 = dP/dn = [J_2 + n dJ_2/dn] / 3, not at the constant-weight
    value J_2 / 3.  Measured from the first zero crossing of the density mode
    (a quarter period)."""
    nx, r0, eps = 64, 0.2, 1e-4
    k = 2 * math.pi / nx
    x = np.arange(nx)
    loc = LocalOracle("d2v9", (nx, 1, 1), tau=0.55, order=2, r0=r0)
    f = loc.init(1 + eps * np.cos(k * x), np.zeros((2, nx)))
    amp = [eps * nx / 2]
    t = 0
    while True:
        f = loc.step(f)
        t += 1
        n, _ = loc.moments(f)
        amp.append(float(np.dot(n - n.mean(), np.cos(k * x))))
        if amp[-1] < 0:
            break
        assert t < 60
    t0 = (t - 1) + amp[-2] / (amp[-2] - amp[-1])
    c_meas = math.pi / (2 * t0) / k
    h = 1e-4
    dJ = (_J2(1 + h, r0) - _J2(1 - h, r0)) / (2 * h)
    c_local = math.sqrt((_J2(1.0, r0) + dJ) / 3)
    c_const = math.sqrt(_J2(1.0, r0) / 3)
    assert abs(c_local / c_const - 1) > 0.04
    assert c_meas == pytest.approx(c_local, rel=5e-3)
