"""Pins of the oracle's obstacles and body force (orc_run_porous), each against a
fact that does not come from the oracle: exact momentum balance, mass
conservation, link reversal at a solid, and the steady channel (Poiseuille)
flow between solid rows, whose curvature is fixed by the lattice viscosity
(pinned independently by the shear-wave test) and whose wall slip vanishes at
the relaxation time known for halfway bounce-back, (tau - 1/2)^2 = 3/16."""
import math

import numpy as np
import pytest

from oracle.lbm import BOUNCE_BACK, Oracle


def test_force_adds_exactly_F_per_cell_per_step_and_no_mass():
    nx, ny, steps = 16, 12, 30
    F = np.array([1e-4, -2.5e-5])
    orc = Oracle("d2v9", shape=(nx, ny, 1), tau=0.7, order=2)
    rng = np.random.default_rng(0)
    n0 = 1 + 0.01 * rng.standard_normal(nx * ny)
    u0 = 0.01 * rng.standard_normal((2, nx * ny))
    f = orc.init(n0, u0)
    e = np.array(orc.model.e)[:, :2]
    m0, p0 = f.sum(), (f.T @ e).sum(axis=0)
    orc.run_porous(f, steps, force=(F[0], F[1]))
    m1, p1 = f.sum(), (f.T @ e).sum(axis=0)
    assert m1 == pytest.approx(m0, rel=1e-14)
    np.testing.assert_allclose(p1 - p0, steps * nx * ny * F, rtol=1e-9, atol=1e-14)


def test_zero_force_without_solids_is_the_plain_run():
    orc = Oracle("d2v9", shape=(10, 8, 1), tau=0.6, order=3)
    rng = np.random.default_rng(1)
    f0 = orc.init(1 + 0.01 * rng.standard_normal(80), 0.02 * rng.standard_normal((2, 80)))
    a, b = f0.copy(), f0.copy()
    orc.run(a, 7)
    orc.run_porous(b, 7)
    np.testing.assert_array_equal(a, b)


def test_solids_conserve_mass_and_stay_untouched():
    nx, ny = 20, 14
    solid = np.zeros((ny, nx), bool)
    solid[4:7, 5:9] = True
    solid[10, 15] = True
    orc = Oracle("d2v9", shape=(nx, ny, 1), tau=0.8, order=2)
    rng = np.random.default_rng(2)
    f = orc.init(1 + 0.02 * rng.standard_normal(nx * ny), 0.02 * rng.standard_normal((2, nx * ny)))
    before = f[:, solid.reshape(-1)].copy()
    fluid_mass = f[:, ~solid.reshape(-1)].sum()
    orc.run_porous(f, 50, solid=solid)
    np.testing.assert_array_equal(f[:, solid.reshape(-1)], before)
    assert f[:, ~solid.reshape(-1)].sum() == pytest.approx(fluid_mass, rel=1e-13)  # rounding of 50 steps


def test_enclosed_cell_reverses_every_moving_population():
    """A fluid cell with solid neighbours on all sides and no relaxation
    (tau -> infinity): each step sends every moving population back reversed."""
    orc = Oracle("d2v9", shape=(3, 3, 1), tau=1e12, order=2)
    solid = np.ones((3, 3), bool)
    solid[1, 1] = False
    f = orc.init(np.ones(9), np.zeros((2, 9)))
    rng = np.random.default_rng(3)
    f[:, 4] = 0.1 + rng.random(9)
    g = f.copy()
    orc.run_porous(g, 1, solid=solid)
    opp = np.array(orc.model.opp)
    np.testing.assert_allclose(g[:, 4], f[opp, 4], rtol=1e-10)


def channel_profile(tau, F=1e-6, H=16, steps=24000):
    nx, ny = 4, H + 2
    solid = np.zeros((ny, nx), bool)
    solid[0] = solid[-1] = True
    orc = Oracle("d2v9", shape=(nx, ny, 1), tau=tau, order=2)
    f = orc.init(np.ones(nx * ny), np.zeros((2, nx * ny)))
    orc.run_porous(f, steps, solid=solid, force=(F, 0.0))
    n, u = orc.moments(f)
    ux = (u[0] * n + F / 2) / n  # physical velocity (j + F/2) / n
    return ux.reshape(ny, nx)[1:-1, 0], F


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2])
def test_channel_flow_is_a_parabola_with_the_lattice_viscosity(tau):
    prof, F = channel_profile(tau)
    nu = (tau - 0.5) / 3.0  # kappa (tau - 1/2), kappa = 1/3 at second order on d2v9 (T = 0)
    d2 = prof[2:] - 2 * prof[1:-1] + prof[:-2]
    np.testing.assert_allclose(d2, -F / nu, rtol=1e-8)
    # halfway walls at y = 1/2 and y = H + 1/2 (row indices of the fluid rows 1..H)
    y = np.arange(1, prof.size + 1)
    parab = F / (2 * nu) * (y - 0.5) * (prof.size + 0.5 - y)
    slip = prof - parab
    assert np.ptp(slip) < 1e-8 * prof.max()  # a constant slip


def test_channel_slip_vanishes_at_the_known_bounce_back_relaxation_time():
    tau0 = 0.5 + math.sqrt(3.0 / 16.0)
    prof, F = channel_profile(tau0)
    nu = (tau0 - 0.5) / 3.0
    y = np.arange(1, prof.size + 1)
    parab = F / (2 * nu) * (y - 0.5) * (prof.size + 0.5 - y)
    assert np.abs(prof - parab).max() < 1e-6 * prof.max()
    prof2, _ = channel_profile(0.8)
    assert np.abs(prof2 - F / (2 * (0.3 / 3)) * (y - 0.5) * (prof.size + 0.5 - y)).max() > 1e-3 * prof2.max()


def test_wall_faces_and_solid_rows_agree():
    """A channel bounded by bounce-back box faces equals one bounded by solid rows."""
    F, tau, H = 2e-6, 0.7, 10
    a = Oracle("d2v9", shape=(4, H, 1), bc=(0, BOUNCE_BACK, 0), tau=tau, order=2)
    fa = a.init(np.ones(4 * H), np.zeros((2, 4 * H)))
    a.run_porous(fa, 300, force=(F, 0.0))
    b = Oracle("d2v9", shape=(4, H + 2, 1), tau=tau, order=2)
    solid = np.zeros((H + 2, 4), bool)
    solid[0] = solid[-1] = True
    fb = b.init(np.ones(4 * (H + 2)), np.zeros((2, 4 * (H + 2))))
    b.run_porous(fb, 300, solid=solid, force=(F, 0.0))
    fb_fluid = fb.reshape(9, H + 2, 4)[:, 1:-1, :].reshape(9, -1)
    np.testing.assert_allclose(fa, fb_fluid, rtol=1e-13, atol=1e-16)
