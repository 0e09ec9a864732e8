"""Pins of the exact Riemann solutions against the conservation laws themselves."""
import math

import numpy as np
import pytest

from oracle import riemann as rs


LAWS = [rs.isothermal(0.5), rs.isothermal(5 / 9), rs.gamma_law(0.25, 2.0), rs.gamma_law(0.3, 5 / 3)]


def flux(law, n, u):
    return np.array([n * u, n * u * u + law.P(n)])


@pytest.mark.parametrize("law", LAWS, ids=lambda l: f"{l.kind}")
@pytest.mark.parametrize("nL,uL,nR,uR", [(1.0, 0.0, 0.8, 0.0), (1.0, 0.0, 0.5, 0.0),
                                          (0.7, 0.0, 1.0, 0.0), (1.0, 0.3, 0.9, -0.2),
                                          (1.0, -0.2, 1.0, 0.2)])
def test_waves_satisfy_conservation(law, nL, uL, nR, uR):
    sol = rs.solve(law, nL, uL, nR, uR)
    ns, us = sol.n_star, sol.u_star
    for side, (nK, uK) in (("L", (nL, uL)), ("R", (nR, uR))):
        if ns > nK:
            # Rankine-Hugoniot: F(star) - F(K) = s (U(star) - U(K)) for both equations
            s = (sol.left_speeds() if side == "L" else sol.right_speeds())[0]
            jump_F = flux(law, ns, us) - flux(law, nK, uK)
            jump_U = np.array([ns - nK, ns * us - nK * uK])
            np.testing.assert_allclose(jump_F, s * jump_U, rtol=1e-10, atol=1e-12)
            # Lax entropy condition: characteristics run into the shock
            cK, cs = float(law.c(nK)), float(law.c(ns))
            if side == "L":
                assert uK - cK > s > us - cs
            else:
                assert uK + cK < s < us + cs
        else:
            # rarefaction: the fan is continuous at its edges and u -/+ c = x/t inside
            head, tail = sol.left_speeds() if side == "L" else sol.right_speeds()[::-1]
            for xi in np.linspace(min(head, tail), max(head, tail), 7):
                n, u = sol.sample(xi)
                c = float(law.c(n[0]))
                assert (u[0] - c if side == "L" else u[0] + c) == pytest.approx(xi, abs=1e-12)
            eps = 1e-9
            a_out, a_in = sol.sample(head - eps if side == "L" else head + eps), sol.sample(head)
            assert a_out[0][0] == pytest.approx(nK, abs=1e-7) and a_in[0][0] == pytest.approx(nK, abs=1e-7)
            t_in = sol.sample(tail)
            assert t_in[0][0] == pytest.approx(ns, abs=1e-7) and t_in[1][0] == pytest.approx(us, abs=1e-7)


def test_symmetric_collision_has_zero_middle_velocity():
    sol = rs.solve(rs.isothermal(0.5), 1.0, 0.2, 1.0, -0.2)
    assert sol.u_star == pytest.approx(0.0, abs=1e-14)
    assert sol.n_star > 1.0


def test_isothermal_rarefaction_profile_closed_form():
    """Inside an isothermal left fan, n = n_L exp(-(u - u_L)/a) and u = x/t + a."""
    a2 = 0.5
    sol = rs.solve(rs.isothermal(a2), 1.0, 0.0, 0.8, 0.0)
    a = math.sqrt(a2)
    head, tail = sol.left_speeds()
    xi = 0.5 * (head + tail)
    n, u = sol.sample(xi)
    assert u[0] == pytest.approx(xi + a, abs=1e-14)
    assert n[0] == pytest.approx(math.exp(-u[0] / a), rel=1e-14)
