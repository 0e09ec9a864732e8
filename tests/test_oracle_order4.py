"""Pins of the oracle's fourth-order pieces (P_4 of eq. H4, A_4 of eq. A4, the
expansion to N = 4) and of the 41-velocity set it runs on, each against a fact
that does not come from the oracle's own formulas: orthonormality under the
weight by exact quadrature over the Fermi disk and by Gauss-Hermite quadrature,
the Gaussian-limit values the paper states, A as the projection of the shifted
weight, the moment conditions of eq. i2n-disc, and the moments of the shifted
Fermi disk.  A last test records a finding: beyond second order the
zero-temperature expansion is linearly unstable on this set too."""
import itertools
import math

import numpy as np
import pytest

from oracle import theory as th
from oracle.lbm import Oracle
from test_oracle_theory import ball_nodes, kron_sym


def indices(D, order=4):
    for N in range(order + 1):
        yield from itertools.product(range(D), repeat=N)


@pytest.mark.parametrize("D", [1, 2])
def test_continuous_orthonormality_through_fourth_order(D):
    """Eq. omeg-feq for P_0..P_4 under the zero-temperature weight, by exact
    quadrature over the Fermi disk (ball): P_4 with the printed d_4, d'_4, dbar_4."""
    co = th.coefficients(th.moments_fd_t0(D, 1.0), D, kmax=4)
    pts, wts = ball_nodes(D)
    idx = list(indices(D))
    vals = {i: np.array([th.P(co, i, p) for p in pts]) for i in idx}
    for i in idx:
        for j in idx:
            assert float(np.sum(wts * vals[i] * vals[j])) == pytest.approx(kron_sym(i, j), abs=1e-10), (i, j)


def test_continuous_orthonormality_through_fourth_order_gaussian():
    co = th.coefficients(th.moments_mb(2, 1.0, 1.0), 2, kmax=4)
    x, w = np.polynomial.hermite_e.hermegauss(14)
    w = w / math.sqrt(2 * math.pi)
    pts = [(a, b) for a in x for b in x]
    wts = np.array([wa * wb for wa in w for wb in w])
    idx = list(indices(2))
    vals = {i: np.array([th.P(co, i, p) for p in pts]) for i in idx}
    for i in idx:
        for j in idx:
            assert float(np.sum(wts * vals[i] * vals[j])) == pytest.approx(kron_sym(i, j), abs=1e-11)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_gaussian_limit_of_the_fourth_order_coefficients(D):
    """Remark after eq. sommerfeld: with I_2N = 1, c_4 = 1, |c'_4| = 1, cbar_4 = 0,
    |d_4| = 1, dbar_4 = 0 and d'_4 = 0."""
    co = th.coefficients(th.moments_mb(D, 1.0, 1.0), D, kmax=4)
    assert co.c[4] == pytest.approx(1.0) and abs(co.cp[4]) == pytest.approx(1.0)
    assert co.cb[4] == pytest.approx(0.0, abs=1e-15)
    assert abs(co.d["d4"]) == pytest.approx(1.0, rel=1e-14)
    assert co.d["db4"] == pytest.approx(0.0, abs=1e-14) and co.d["dp4"] == pytest.approx(0.0, abs=1e-14)


def _other_root(I, D, co):
    """The coefficients of P_4 taken with d_4 = -sqrt(d_4^2)."""
    dl = {L: 2.0 * I[L + 2] * I[L - 2] / th.Delta_sq(I, D, L) for L in (2, 4, 6)}
    D6 = math.sqrt(th.Delta_sq(I, D, 6))
    d4 = -co.d["d4"]
    return {"d4": d4,
            "dp4": -(d4 / D) * (I[0] / I[2] + I[4] * dl[2] / (I[2] * dl[4])) + 2 * co.c[4] * I[6] * D6 / (D * I[4]),
            "db4": d4 * dl[2] / (D * (D + 2) * dl[4]) + co.c[4] * (D - 2 * (D + 2) * D6) / (D * (D + 2) * (D + 4))}


@pytest.mark.parametrize("D", [1, 2, 3])
def test_the_sign_of_d4_is_fixed_by_the_gaussian_limit(D):
    """d_4 is printed through d_4^2, and both roots make P_4 orthonormal; the paper's
    Gaussian limit (dbar_4 = 0, d'_4 = 0, i.e. the Hermite polynomial) holds only for
    the positive root: there dbar_4 = (d_4 - 1) / (D (D + 2))."""
    I = th.moments_mb(D, 1.0, 1.0)
    co = th.coefficients(I, D, kmax=4)
    other = _other_root(I, D, co)
    assert co.d["d4"] > 0 and co.d["db4"] == pytest.approx(0.0, abs=1e-14)
    assert other["db4"] == pytest.approx(-2.0 / (D * (D + 2)), rel=1e-12)


@pytest.mark.parametrize("D", [1, 2])
def test_A4_is_the_projection_of_the_shifted_weight(D):
    """Eq. expansao1 for N = 4, by direct integration; checks the printed A_4 with
    its sixth pair term read as u_i2 u_i4 delta_i1i3."""
    co = th.coefficients(th.moments_fd_t0(D, 1.0), D, kmax=4)
    pts, wts = ball_nodes(D)
    rng = np.random.default_rng(6)
    for _ in range(3):
        u = 0.3 * rng.standard_normal(D)
        for i in itertools.product(range(D), repeat=4):
            direct = float(np.sum(wts * np.array([th.P(co, i, p + u) for p in pts])))
            assert th.A(co, i, u) == pytest.approx(direct, abs=1e-11), i


def test_A4_as_printed_is_not_the_projection():
    """Taken literally (u_i2 u_i4 delta_i2i3 in place of delta_i1i3) A_4 differs from
    the projection for an index tuple where the two deltas differ."""
    co = th.coefficients(th.moments_fd_t0(2, 1.0), 2, kmax=4)
    pts, wts = ball_nodes(2)
    u = np.array([0.21, -0.13])
    i = (0, 1, 1, 0)
    direct = float(np.sum(wts * np.array([th.P(co, i, p + u) for p in pts])))
    assert th.A(co, i, u) == pytest.approx(direct, abs=1e-11)
    # literal form: replace the pair term u_1 u_3 delta_12 (indices as printed) by u_1 u_3 delta_11
    lit = th.A(co, i, u) + co.I0 * ((1 - co.J2 * co.J4) * co.cp[4] + co.cb[4] * float(u @ u)) * (
        u[i[1]] * u[i[3]] * (float(i[1] == i[2]) - float(i[0] == i[2])))
    assert abs(lit - direct) > 1e-4


def test_A4_vanishes_at_zero_velocity():
    for D in (1, 2, 3):
        co = th.coefficients(th.moments_fd_t0(D, 1.7), D, kmax=4)
        for i in itertools.product(range(D), repeat=4):
            assert th.A(co, i, np.zeros(D)) == pytest.approx(0.0, abs=1e-15)


# --------------------------------------------------------------------------
# the 41-velocity set
# --------------------------------------------------------------------------

def test_d2v41_meets_the_moment_conditions_through_degree_nine():
    m = th.make_model("d2v41")
    I = th.moments_fd_t0(2, 1.0)
    assert m.Q == 41 and (m.w_hat > 0).all()
    xi = m.cvel * m.e.astype(float)
    w = m.w_hat * I[0]
    for deg in range(10):
        for mono in itertools.product(range(deg + 1), repeat=2):
            if sum(mono) != deg:
                continue
            lhs = float(np.sum(w * xi[:, 0] ** mono[0] * xi[:, 1] ** mono[1]))
            rhs = th.isotropic_moment(I, mono)
            assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-12 * I[min(deg + deg % 2, 8)]), mono
    shell = np.array([int(v @ v) for v in m.e])
    assert m.w_hat[shell == 1][0] == pytest.approx(m.w_hat[shell == 16][0], rel=1e-12)
    # the scale is the largest smallest weight: nearby scales have a smaller minimum
    c_gq = math.sqrt(3 * I[4] / I[2])
    for dc in (-1e-3, 1e-3):
        w2, _ = th.quadrature_weights(I, "d2v41", cvel=m.cvel + dc * c_gq, max_degree=8)
        assert w2.min() < (m.w_hat * I[0]).min()


def test_d2v41_discrete_orthonormality_through_fourth_order():
    """Every pair P_M, P_N with M, N <= 4 (degree <= 8) is orthonormal on the set:
    the discrete sums equal the continuous ones."""
    m = th.make_model("d2v41")
    co = m.co
    xi = m.cvel * m.e.astype(float)
    w = m.w_hat * co.I0
    idx = list(indices(2))
    vals = {i: np.array([th.P(co, i, x) for x in xi]) for i in idx}
    for i in idx:
        for j in idx:
            assert float(np.sum(w * vals[i] * vals[j])) == pytest.approx(kron_sym(i, j), abs=1e-9), (i, j)


def test_fourth_order_equilibrium_has_the_moments_of_the_shifted_fermi_disk():
    """At N = 4 on d2v41 the discrete equilibrium reproduces every moment of order
    <= 4 of f_eq(xi - u), the Fermi disk moved by u (density, momentum, pressure
    tensor, energy flux and the fourth moments), computed by exact quadrature
    over the moved disk.  At N = 2 the third moments are off."""
    m = th.make_model("d2v41")
    pts, wts = ball_nodes(2)
    xi = m.cvel * m.e.astype(float)
    u0 = np.array([0.031, -0.017])
    u = m.cvel * u0
    n = m.co.I0
    feq4 = th.feq_tensor(m, n, u0, 4)
    feq2 = th.feq_tensor(m, n, u0, 2)
    for deg in range(5):
        for mono in itertools.product(range(deg + 1), repeat=2):
            if sum(mono) != deg:
                continue
            cont = float(np.sum(wts * (pts[:, 0] + u[0]) ** mono[0] * (pts[:, 1] + u[1]) ** mono[1]))
            disc = float(np.sum(feq4 * xi[:, 0] ** mono[0] * xi[:, 1] ** mono[1]))
            assert disc == pytest.approx(cont, rel=1e-11, abs=1e-13), mono
    cont3 = float(np.sum(wts * (pts[:, 0] + u[0]) ** 3))
    assert abs(float(np.sum(feq2 * xi[:, 0] ** 3)) - cont3) > 1e-4 * abs(cont3)


def growth_factors(model, order, tau, ks):
    """Largest |eigenvalue| of the collide-and-stream map linearised about rest
    (n = 1, u = 0) for each wave vector in ks (numerical Jacobian of f_eq)."""
    e = model.e.astype(float)
    f0 = th.feq_tensor(model, 1.0, [0.0, 0.0], order)

    def feq_of(f):
        n = f.sum()
        return th.feq_tensor(model, n, (f[:, None] * e).sum(axis=0) / n, order)

    Q, h = model.Q, 1e-7
    Jac = np.zeros((Q, Q))
    for b in range(Q):
        d = np.zeros(Q)
        d[b] = h
        Jac[:, b] = (feq_of(f0 + d) - feq_of(f0 - d)) / (2 * h)
    M = (1 - 1 / tau) * np.eye(Q) + Jac / tau
    out = {}
    for k in ks:
        ph = np.exp(-1j * (e @ np.asarray(k, dtype=float)))
        out[k] = float(np.max(np.abs(np.linalg.eigvals(ph[:, None] * M))))
    return out


def test_beyond_second_order_the_expansion_is_linearly_unstable_on_d2v41():
    """Finding: on the degree-9 set too, the zero-temperature expansion beyond
    second order grows at rest (the c'_3 (1 - J_2) term of A_3 is linear in u),
    while the second-order truncation does not.  The oracle's growth of a tiny
    perturbation matches the linear analysis of its own equilibrium."""
    m = th.make_model("d2v41")
    tau, nx = 0.8, 16
    ks = [(2 * math.pi * a / nx, 2 * math.pi * b / nx) for a in range(nx // 2 + 1) for b in range(nx // 2 + 1)
          if (a, b) != (0, 0)]
    g3 = growth_factors(m, 3, tau, ks)
    kbest = max(g3, key=g3.get)
    assert g3[kbest] > 1.05
    assert max(growth_factors(m, 2, tau, ks).values()) < 1 + 1e-9
    assert growth_factors(m, 4, tau, [kbest])[kbest] == pytest.approx(g3[kbest], rel=1e-6)
    o = Oracle(m, shape=(nx, nx, 1), tau=tau, order=3)
    rng = np.random.default_rng(12)
    f = o.init(1 + 1e-10 * rng.standard_normal(nx * nx), 1e-10 * rng.standard_normal((2, nx * nx)))
    x = np.arange(nx)
    X, Y = np.meshgrid(x, x)
    mode = np.exp(-1j * (kbest[0] * X + kbest[1] * Y)).reshape(-1)
    o.run(f, 40)
    na, _ = o.moments(f)
    o.run(f, 20)
    nb, _ = o.moments(f)
    rate = (abs(np.sum(nb * mode)) / abs(np.sum(na * mode))) ** (1 / 20)
    assert rate == pytest.approx(g3[kbest], rel=5e-3)
