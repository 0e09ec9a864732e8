"""Pins of the oracle's theory module against what the paper and the mathematics fix.

None of these retypes the oracle's own formula: each compares it with a direct
integral, a closed form the paper prints in a different place, the textbook
Hermite equilibrium, or the paper's second (geometric-space) form of the
discrete equilibrium.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import theory as th


# --------------------------------------------------------------------------
# exact quadrature over the zero-temperature Fermi ball (|xi|^2 < 2 mu)
# --------------------------------------------------------------------------

def ball_nodes(D, mu=1.0, nr=24, nphi=48):
    """Nodes and weights that integrate polynomials of degree < 2*nr - D over the
    ball of radius sqrt(2 mu) exactly (Gauss-Legendre in r, uniform in angle)."""
    R = math.sqrt(2.0 * mu)
    x, w = np.polynomial.legendre.leggauss(nr)
    r = 0.5 * R * (x + 1.0)
    wr = 0.5 * R * w
    if D == 1:
        return np.concatenate([r, -r])[:, None], np.concatenate([wr, wr])
    if D == 2:
        phi = 2 * math.pi * np.arange(nphi) / nphi
        pts = np.array([[ri * math.cos(p), ri * math.sin(p)] for ri in r for p in phi])
        wts = np.array([wi * ri * 2 * math.pi / nphi for ri, wi in zip(r, wr) for _ in phi])
        return pts, wts
    raise ValueError(D)


def ball_integral(D, fn, mu=1.0):
    pts, wts = ball_nodes(D, mu)
    return sum(w * fn(p) for p, w in zip(pts, wts))


@pytest.mark.parametrize("D", [1, 2, 3])
@pytest.mark.parametrize("mu", [1.0, 2.5])
def test_fd_t0_moments_equal_radial_integral(D, mu):
    """Sommerfeld closed form at theta = 0 versus the radial integral formula."""
    I = th.moments_fd_t0(D, mu)
    R = math.sqrt(2 * mu)
    Ir = th.moments_radial(D, lambda r: 1.0 if r < R else 0.0, xi_max=R, nmax=4)
    for L in I:
        assert I[L] == pytest.approx(Ir[L], rel=1e-12)


@pytest.mark.parametrize("D", [1, 2])
def test_fd_t0_moment_tensor_structure(D):
    """int omega xi_x^{2N} = I_{2N} (2N-1)!! and int omega xi_x^2 xi_y^2 = I_4 (direct
    integration over the Fermi ball)."""
    I = th.moments_fd_t0(D, 1.0)
    for N in range(4):
        direct = ball_integral(D, lambda p: p[0] ** (2 * N))
        assert direct == pytest.approx(I[2 * N] * math.prod(range(2 * N - 1, 0, -2)), rel=1e-12)
    if D == 2:
        assert ball_integral(2, lambda p: p[0] ** 2 * p[1] ** 2) == pytest.approx(I[4], rel=1e-12)
        assert ball_integral(2, lambda p: p[0] ** 3 * p[1]) == pytest.approx(0.0, abs=1e-13)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_t0_ratios_closed_forms(D):
    """The zero-temperature paragraph: J_N = 1 + 2/(N + D), Delta_N^2 = (D + N)/2,
    I_0 = (2 pi mu)^{D/2} / Gamma(D/2 + 1), c_0 = sqrt(6 mu / (D + 4))."""
    for mu in (1.0, 3.0):
        I = th.moments_fd_t0(D, mu)
        for L in (2, 4):
            assert th.J(I, L) == pytest.approx(1 + 2 / (L + D), rel=1e-13)
            assert th.Delta_sq(I, D, L) == pytest.approx((D + L) / 2, rel=1e-12)
        assert I[0] == pytest.approx((2 * math.pi * mu) ** (D / 2) / math.gamma(D / 2 + 1), rel=1e-14)
        co = th.coefficients(I, D)
        assert co.c0_lattice == pytest.approx(math.sqrt(6 * mu / (D + 4)), rel=1e-14)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_gaussian_limit_coefficients(D):
    """Remark after eq. sommerfeld: with I_{2N} = 1, c_K = 1, |c'_K| = 1, cbar_K = 0."""
    co = th.coefficients(th.moments_mb(D, 1.0, 1.0), D)
    for K in range(4):
        assert co.c[K] == pytest.approx(1.0)
    for K in (2, 3):
        assert abs(co.cp[K]) == pytest.approx(1.0)
        assert co.cb[K] == pytest.approx(0.0, abs=1e-15)
    assert th.J(co.I, 2) == 1.0 and th.Delta_sq(co.I, D, 4) == 1.0


def all_indices(D, order=3):
    for N in range(order + 1):
        yield from itertools.product(range(D), repeat=N)


def kron_sym(i, j):
    """delta_{i1..iN | j1..jN}: sum over permutations of j of the delta products."""
    if len(i) != len(j):
        return 0.0
    return float(sum(all(a == b for a, b in zip(i, p)) for p in itertools.permutations(j)))


@pytest.mark.parametrize("D", [1, 2])
def test_continuous_orthonormality_fd_t0(D):
    """Eq. omeg-feq under the zero-temperature weight, by direct integration."""
    co = th.coefficients(th.moments_fd_t0(D, 1.0), D)
    pts, wts = ball_nodes(D)
    idx = list(all_indices(D))
    vals = {i: np.array([th.P(co, i, p) for p in pts]) for i in idx}
    for i in idx:
        for j in idx:
            g = float(np.sum(wts * vals[i] * vals[j]))
            assert g == pytest.approx(kron_sym(i, j), abs=1e-11), (i, j)


def test_continuous_orthonormality_mb():
    """Eq. omeg-feq under the Gaussian weight of unit density and theta = 1 (D = 2),
    by tensor Gauss-Hermite quadrature."""
    co = th.coefficients(th.moments_mb(2, 1.0, 1.0), 2)
    x, w = np.polynomial.hermite_e.hermegauss(12)
    w = w / math.sqrt(2 * math.pi)
    pts = [(a, b) for a in x for b in x]
    wts = np.array([wa * wb for wa in w for wb in w])
    idx = list(all_indices(2))
    for i in idx:
        for j in idx:
            g = float(np.sum(wts * np.array([th.P(co, i, p) * th.P(co, j, p) for p in pts])))
            assert g == pytest.approx(kron_sym(i, j), abs=1e-12)


@pytest.mark.parametrize("D", [1, 2])
def test_A_is_projection_of_shifted_equilibrium(D):
    """Eq. expansao1: A_{i..}(u) = int omega(eta) P_{i..}(eta + u) d eta, by direct
    integration (checks the printed A0-A3, including c'_3 (1 - J_2))."""
    co = th.coefficients(th.moments_fd_t0(D, 1.0), D)
    pts, wts = ball_nodes(D)
    rng = np.random.default_rng(5)
    for _ in range(3):
        u = 0.3 * rng.standard_normal(D)
        for i in all_indices(D):
            direct = float(np.sum(wts * np.array([th.P(co, i, p + u) for p in pts])))
            assert th.A(co, i, u) == pytest.approx(direct, abs=1e-11), i


def test_A_vanishes_at_zero_velocity():
    """Eq. expansao2: A_{i..}(0) = 0 for N > 0 and A_0 P_0 = 1."""
    for D in (1, 2, 3):
        co = th.coefficients(th.moments_fd_t0(D, 1.3), D)
        for i in all_indices(D):
            if len(i) > 0:
                assert th.A(co, i, np.zeros(D)) == pytest.approx(0.0, abs=1e-15)
        assert th.A(co, (), np.zeros(D)) * th.P(co, (), np.zeros(D)) == pytest.approx(1.0, rel=1e-15)


@pytest.mark.parametrize("lat", ["d1v3", "d2v9"])
def test_weights_match_printed_formulas(lat):
    """Section on the Gaussian quadrature: d1v3 w0 = I0 (1 - J2/3), w1 = I0 J2/6;
    d2v9 w0 = I0 (1 - 5 J2/9), w_long = I0 J2/36, w_short = I0 J2/9; c0 = sqrt(3 I4/I2).
    The oracle solves the moment conditions instead of using these."""
    for family in (th.FD_T0, th.MB):
        m = th.make_model(lat, family)
        J2 = m.co.J2
        e2 = (m.e ** 2).sum(axis=1)
        if lat == "d1v3":
            want = np.where(e2 == 0, 1 - J2 / 3, J2 / 6)
        else:
            want = np.where(e2 == 0, 1 - 5 * J2 / 9, np.where(e2 == 1, J2 / 9, J2 / 36))
        np.testing.assert_allclose(m.w_hat, want, rtol=1e-14, atol=0)
        assert m.cvel == pytest.approx(math.sqrt(3 * m.co.I[4] / m.co.I[2]))


def test_t0_weights_values():
    """Exact rational weights at theta = 0 implied by the formulas (the printed
    numerical values in the zero-temperature paragraph are inconsistent; the
    formulas are followed)."""
    np.testing.assert_allclose(th.make_model("d1v3").w_hat, [4 / 9, 5 / 18, 5 / 18], rtol=1e-14)
    np.testing.assert_allclose(th.make_model("d2v9").w_hat[[0, 1, 5]], [1 / 6, 1 / 6, 1 / 24], rtol=1e-14)
    np.testing.assert_allclose(th.make_model("d3v19").w_hat[[0, 1, 7]], [1 / 15, 7 / 90, 7 / 180], rtol=1e-14)


def lattice_P(m, i):
    return np.array([th.P(m.co, i, m.cvel * e) for e in m.e])


@pytest.mark.parametrize("lat", ["d1v3", "d2v9", "d3v19"])
def test_discrete_orthonormality_up_to_degree_five(lat):
    """Eq. i2n-disc makes sum_a w_a P_i P_j equal the continuous integral for every
    pair of total degree <= 5, so eq. omeg-feq holds on the lattice for them."""
    m = th.make_model(lat)
    w = m.w_hat * m.co.I0
    idx = list(all_indices(m.D))
    for i in idx:
        for j in idx:
            if len(i) + len(j) > 5:
                continue
            g = float(np.sum(w * lattice_P(m, i) * lattice_P(m, j)))
            assert g == pytest.approx(kron_sym(i, j), abs=1e-12), (i, j)


def test_third_order_not_orthonormal_on_lattice():
    """P_111 P_111 is of degree 6, beyond what d2v9 integrates: its lattice norm is
    not 1 (and on d1v3 P_111 vanishes at every node)."""
    m = th.make_model("d2v9")
    w = m.w_hat * m.co.I0
    assert abs(float(np.sum(w * lattice_P(m, (0, 0, 0)) ** 2)) - 6.0) > 1.0
    m1 = th.make_model("d1v3")
    np.testing.assert_allclose(lattice_P(m1, (0, 0, 0)), 0.0, atol=1e-14)


def hermite_textbook(e, u):
    """Third-order Hermite equilibrium with c_s^2 = 1/3, over the weight:
    1 + e.u/cs2 + (e.u)^2/(2 cs2^2) - u^2/(2 cs2) + (e.u)^3/(6 cs2^3) - (e.u) u^2/(2 cs2^2)."""
    cs2 = 1.0 / 3.0
    eu, u2 = float(e @ u), float(u @ u)
    return (1 + eu / cs2 + eu ** 2 / (2 * cs2 ** 2) - u2 / (2 * cs2)
            + eu ** 3 / (6 * cs2 ** 3) - eu * u2 / (2 * cs2 ** 2))


@pytest.mark.parametrize("lat,w", [("d1v3", [2 / 3, 1 / 6, 1 / 6]),
                                   ("d2v9", [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)])
def test_gaussian_subcase_is_hermite(lat, w):
    """Remark after eq. sommerfeld: for the Maxwell-Boltzmann weight the polynomials
    are the Hermite ones, so the expansion is the textbook Hermite equilibrium
    (theta = 1/3 puts c_0 = 1, the standard lattice units)."""
    m = th.make_model(lat, th.MB, theta=1.0 / 3.0)
    assert m.cvel == pytest.approx(1.0)
    np.testing.assert_allclose(m.w_hat, w, rtol=1e-14)
    rng = np.random.default_rng(1)
    for _ in range(5):
        u = 0.2 * rng.standard_normal(m.D)
        f = th.feq_tensor(m, 1.3, u)
        want = np.array([1.3 * w[a] * hermite_textbook(m.e[a].astype(float), u) for a in range(m.Q)])
        if lat == "d1v3":  # on three nodes (e.u)^3 = e.u u^2, so the textbook cubic terms cancel too
            pass
        np.testing.assert_allclose(f, want, rtol=1e-13, atol=1e-15)


def geometric_form(m, u0):
    """The discrete third-order equilibrium in geometric space as the paper prints it
    after "becomes in the geometrical space", per population, over w_a."""
    D = m.D
    J2, J4 = m.co.J2, m.co.J4
    d2, d4 = th.Delta_sq(m.co.I, D, 2), th.Delta_sq(m.co.I, D, 4)
    out = []
    for e in m.e.astype(float):
        eu, u2, e2 = float(e @ u0), float(u0 @ u0), float(e @ e)
        br = ((1 - J2) * J4 * (D + 2) * d4 - 3 * (1 - J2) * J4 * d4 * e2 - 3 * J4 * d4 * u2
              + 9 * J4 * (d4 - 1) / (D + 2) * u2 * e2 + 3 * J4 * eu ** 2)
        out.append(1 + 3 / J2 * eu + 9 / (2 * J2) * eu ** 2 + 4.5 * (d2 - 1) / (J2 * D) * u2 * e2
                   - 1.5 * d2 * u2 + 3 / (2 * J2) * eu * br)
    return np.array(out)


@pytest.mark.parametrize("lat", ["d1v3", "d2v9", "d3v19"])
@pytest.mark.parametrize("family", [th.FD_T0, th.MB])
def test_tensor_expansion_equals_geometric_form(lat, family):
    m = th.make_model(lat, family)
    rng = np.random.default_rng(2)
    for _ in range(6):
        u0 = 0.15 * rng.standard_normal(m.D)
        f = th.feq_tensor(m, 0.9, u0)
        np.testing.assert_allclose(f, 0.9 * m.w_hat * geometric_form(m, u0), rtol=1e-12, atol=1e-15)


def xi_form(m, u):
    """The discrete third-order equilibrium in xi-space as the paper prints it before
    the change to geometric velocities (u in the xi units), over w_a."""
    I, D = m.co.I, m.D
    I0, I2, I4, I6 = I[0], I[2], I[4], I[6]
    J2, J4 = m.co.J2, m.co.J4
    d2, d4 = th.Delta_sq(I, D, 2), th.Delta_sq(I, D, 4)
    out = []
    for e in m.e.astype(float):
        xi = m.cvel * e
        xu, u2, x2 = float(xi @ u), float(u @ u), float(xi @ xi)
        br = (3 * (1 - J2) * J4 / I2 * (D + 2) * d4 - 3 * (1 - J2) * J4 / I4 * d4 * x2
              - 3 * J4 / I4 * d4 * u2 + 3 * (d4 - 1) / (I6 * (D + 2)) * x2 * u2 + xu ** 2 / I6)
        out.append(1 + I0 / I2 * xu + I0 / (2 * I4) * xu ** 2 + I0 * (d2 - 1) / (2 * I4 * D) * u2 * x2
                   - I2 / (2 * I4) * d2 * u2 + I0 / 6 * xu * br)
    return np.array(out)


@pytest.mark.parametrize("lat", ["d1v3", "d2v9", "d3v19"])
def test_tensor_expansion_equals_xi_form(lat):
    """The xi-space form of the third-order discrete equilibrium, as printed, equals
    the tensor expansion (u in xi units, u = c_0 u0)."""
    m = th.make_model(lat)
    rng = np.random.default_rng(6)
    for _ in range(6):
        u0 = 0.15 * rng.standard_normal(m.D)
        f = th.feq_tensor(m, 1.0, u0, order=3) / m.w_hat
        np.testing.assert_allclose(f, xi_form(m, m.cvel * u0), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("lat", ["d1v3", "d2v9", "d3v19"])
@pytest.mark.parametrize("order", [2, 3])
def test_equilibrium_moments(lat, order):
    """Collision invariants: sum_a f_eq = n and sum_a f_eq e_a = n u0, and at u0 = 0
    f_eq = n w_a (eq. expansao2)."""
    m = th.make_model(lat)
    rng = np.random.default_rng(3)
    for _ in range(5):
        n = 1 + 0.2 * rng.random()
        u0 = 0.1 * rng.standard_normal(m.D)
        f = th.feq_tensor(m, n, u0, order)
        assert f.sum() == pytest.approx(n, rel=1e-14)
        np.testing.assert_allclose((f[:, None] * m.e).sum(axis=0), n * u0, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(th.feq_tensor(m, 1.7, np.zeros(m.D), order), 1.7 * m.w_hat, rtol=1e-14)


def test_pressure_tensor_is_isothermal():
    """Second moment of the T = 0 d2v9 equilibrium: n (J2/3 delta + u0 u0), exactly
    (the isothermal closure the Riemann checks rely on)."""
    m = th.make_model("d2v9")
    rng = np.random.default_rng(4)
    for order in (2, 3):
        for _ in range(4):
            n, u0 = 1.1, 0.1 * rng.standard_normal(2)
            f = th.feq_tensor(m, n, u0, order)
            Pi = np.einsum("a,ai,aj->ij", f, m.e.astype(float), m.e.astype(float))
            np.testing.assert_allclose(Pi, n * (m.co.J2 / 3 * np.eye(2) + np.outer(u0, u0)), rtol=1e-12, atol=1e-15)


def test_chemical_potential_cancels():
    """The equilibrium over n w_a in lattice units does not depend on the reference
    chemical potential (every coefficient is a ratio of the I_{2N})."""
    a, b = th.make_model("d2v9", mu=1.0), th.make_model("d2v9", mu=2.7)
    u0 = np.array([0.05, -0.02])
    np.testing.assert_allclose(th.feq_tensor(a, 1.0, u0), th.feq_tensor(b, 1.0, u0), rtol=1e-13)


# -- Fermi-Dirac at theta > 0 and Bose-Einstein weights ------------------------

def _g_polylog(nu, z, sign):
    """Complete Fermi-Dirac / Bose-Einstein integral through mpmath's polylogarithm:
    g_nu(z) = -Li_nu(-z) (Fermi-Dirac), Li_nu(z) (Bose-Einstein)."""
    import mpmath

    mpmath.mp.dps = 30
    v = -mpmath.polylog(nu, -mpmath.mpf(z)) if sign > 0 else mpmath.polylog(nu, mpmath.mpf(z))
    return float(mpmath.re(v))


@pytest.mark.parametrize("D", [1, 2, 3])
@pytest.mark.parametrize("sign,z", [(1, 0.05), (1, 1.0), (1, 148.4131591025766), (1, 2.3e17), (-1, 0.2), (-1, 0.9)])
def test_quantum_moments_equal_polylog(D, sign, z):
    """I_2N = (2 pi)^(D/2) theta^(N + D/2) g_(N + D/2)(z) (paragraph before eq.
    sommerfeld), g through the polylogarithm, against the oracle's radial
    integral of the weight itself."""
    theta = 0.7
    I = th.moments_quantum(D, z, theta=theta, sign=sign)
    for N in range(5):
        ref = (2 * math.pi) ** (D / 2) * theta ** (N + D / 2) * _g_polylog(N + D / 2, z, sign)
        assert I[2 * N] == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_fd_moments_follow_the_sommerfeld_expansion(D):
    """eq. sommerfeld: I_2N = (2 pi)^(D/2) mu^nu / Gamma(nu + 1) [1 + pi^2/6 nu (nu - 1)
    (theta/mu)^2 + ...], nu = N + D/2.  What remains is the series' next term,
    (7 pi^4 / 360) nu (nu-1) (nu-2) (nu-3) (theta/mu)^4 (zero for nu = 1, 2, 3,
    where the series ends and only exponentially small terms are left)."""
    mu = 1.0
    for r in (1 / 20, 1 / 40):
        theta = r * mu
        I = th.moments_quantum(D, math.exp(mu / theta), theta=theta, sign=+1)
        for N in range(5):
            nu = N + D / 2
            somm = (2 * math.pi) ** (D / 2) * mu ** nu / math.gamma(nu + 1) * (1 + math.pi ** 2 / 6 * nu * (nu - 1) * r * r)
            rem = I[2 * N] / somm - 1
            nxt = 7 * math.pi ** 4 / 360 * nu * (nu - 1) * (nu - 2) * (nu - 3) * r ** 4
            assert abs(rem - nxt) <= 0.1 * abs(nxt) + 1e-8, (N, r, rem, nxt)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_quantum_weights_reach_their_limits(D):
    """z -> 0: both reduce to the Maxwell-Boltzmann weight (J_L -> 1); Fermi-Dirac at
    z -> infinity reaches the zero-temperature ratios J_L = 1 + 2/(L + D)."""
    for sign in (1, -1):
        I = th.moments_quantum(D, 1e-7, theta=0.5, sign=sign)
        assert abs(th.J(I, 2) - 1) < 1e-6 and abs(th.J(I, 4) - 1) < 1e-6
    I = th.moments_quantum(D, math.exp(400.0), theta=1e-3, sign=1)
    assert th.J(I, 2) == pytest.approx(1 + 2 / (2 + D), rel=1e-4)
    assert th.J(I, 4) == pytest.approx(1 + 2 / (4 + D), rel=1e-4)
    # Fermi statistics push J above the Gaussian value, Bose statistics below
    assert th.J(th.moments_quantum(D, 2.0, sign=1), 2) > 1 > th.J(th.moments_quantum(D, 0.5, sign=-1), 2)


@pytest.mark.parametrize("lat", ["d1v3", "d2v9", "d3v19"])
@pytest.mark.parametrize("family,z", [(th.FD, 148.4131591025766), (th.BE, 0.6)])
def test_quantum_models_meet_the_quadrature_conditions(lat, family, z):
    """The lattice weights solve eq. i2n-disc for the new weights too, and the
    discrete equilibrium keeps mass and momentum."""
    m = th.make_model(lat, family, z=z, theta=0.9)
    assert m.w_hat.sum() == pytest.approx(1.0, abs=1e-13)
    rng = np.random.default_rng(4)
    for _ in range(3):
        u0 = 0.05 * rng.standard_normal(m.D)
        f = th.feq_tensor(m, 1.3, u0, order=3)
        assert f.sum() == pytest.approx(1.3, rel=1e-13)
        np.testing.assert_allclose(f @ m.e[:, :m.D], 1.3 * u0, rtol=1e-12, atol=1e-15)
