"""FP64 reference theory of the generalized-polynomial lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Nothing under ``oracle/`` belongs to the product
path: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import it.  It shares no code, tables or constants with the
HIP library; the two meet only through seeded input arrays.

Everything here is written from the paper (Coelho, Ilha, Doria, arXiv:1510.07328)
in its own notation, plain and slow, in float64:

* weight families and their moment integrals I_N
  (section "Generalized polynomials in D dimensions", eqs. i2n-cont, i2n-cont2,
  sommerfeld, and the Maxwell-Boltzmann remark that follows it);
* the ratios J_L and Delta_L and the polynomial coefficients c_K, c'_K, cbar_K
  (same section, the paragraph after eq. H4);
* the polynomials P_0..P_3 as tensors (eqs. H0-H3);
* the shifted-argument coefficients A_0..A_3 (section "The EDF expansion in
  generalized polynomials", eqs. A0-A3) and the truncated expansion of the
  equilibrium (eq. expansao0);
* the velocity sets and their weights, found by solving the discrete moment
  conditions (section "The Gaussian quadrature", eq. i2n-disc) rather than by
  copying printed weight values.

Readings taken where the text is garbled or silent (each is also listed in the
design notes of the repository):

* c'_K and cbar_K are used for K = 2, 3 (4) only; P_1 has no such terms.
* The d2v9 long vectors are (1,1), (-1,1), (-1,-1), (1,-1) (the printed list
  repeats (1,-1)).
* Delta_L is the positive square root of the printed Delta_L^2.
* The D=3 velocity set (not given in the paper) is the 19-velocity set whose
  weights solve the same moment conditions with c_0^2 = 3 I_4 / I_2.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Weight families and their isotropic moments I_N  (eqs. i2n-cont, i2n-cont2)
# ---------------------------------------------------------------------------

FD_T0 = "fd_t0"   # Fermi-Dirac at theta = 0: a step of height 1 inside |xi|^2 < 2 mu
MB = "mb"         # Maxwell-Boltzmann: rho0 exp(-xi^2 / 2 theta) / (2 pi theta)^(D/2)
FD = "fd"         # Fermi-Dirac at theta > 0: 1 / (z^-1 exp(xi^2 / 2 theta) + 1), z = e^(mu/theta)
BE = "be"         # Bose-Einstein: 1 / (z^-1 exp(xi^2 / 2 theta) - 1), 0 < z < 1


def moments_fd_t0(D: int, mu: float = 1.0, nmax: int = 4) -> dict:
    """I_{2N} of the zero-temperature Fermi-Dirac weight.

    The Sommerfeld form (eq. sommerfeld) with theta = 0, which the section on
    electrons in metals uses: I_{2N} = (2 pi)^{D/2} mu^{N + D/2} / Gamma(N + D/2 + 1).
    Returned as {L: I_L} for even L = 0 .. 2 nmax; odd moments vanish.
    """
    return {2 * N: (2.0 * math.pi) ** (D / 2.0) * mu ** (N + D / 2.0)
            / math.gamma(N + D / 2.0 + 1.0) for N in range(nmax + 1)}


def moments_sommerfeld(D: int, mu: float, theta: float, nmax: int = 4) -> dict:
    """I_{2N} of the Fermi-Dirac weight in the Sommerfeld limit, eq. sommerfeld with
    the series cut after the (theta/mu)^2 term, as the paper does:
    I_{2N} = (2 pi)^{D/2} mu^nu / Gamma(nu + 1) [1 + (pi^2 / 6) nu (nu - 1) (theta/mu)^2],
    nu = N + D/2.  Returned as {L: I_L} for even L = 0 .. 2 nmax."""
    r2 = (theta / mu) ** 2
    out = {}
    for N in range(nmax + 1):
        nu = N + D / 2.0
        out[2 * N] = ((2.0 * math.pi) ** (D / 2.0) * mu ** nu / math.gamma(nu + 1.0)
                      * (1.0 + math.pi ** 2 / 6.0 * nu * (nu - 1.0) * r2))
    return out


def moments_mb(D: int, rho0: float = 1.0, theta: float = 1.0, nmax: int = 4) -> dict:
    """I_{2N} = I_0 theta^N of the Maxwell-Boltzmann weight (remark after eq. sommerfeld)."""
    return {2 * N: rho0 * theta ** N for N in range(nmax + 1)}


def moments_radial(D: int, omega, xi_max: float, nmax: int = 4, breakpoints=()) -> dict:
    """I_{2N} of an isotropic weight omega(|xi|) from the radial integral, eq. i2n-cont2:

        I_{2N} = pi^{D/2} / (2^{N-1} Gamma(N + D/2)) * int_0^inf omega(xi) xi^{2N+D-1} dxi.
    """
    from scipy import integrate

    out = {}
    for N in range(nmax + 1):
        pts = [0.0] + sorted(b for b in breakpoints if 0.0 < b < xi_max) + [xi_max]
        total = 0.0
        for a, b in zip(pts[:-1], pts[1:]):
            val, _ = integrate.quad(lambda r: omega(r) * r ** (2 * N + D - 1), a, b,
                                    epsabs=0.0, epsrel=1e-13, limit=200)
            total += val
        out[2 * N] = math.pi ** (D / 2.0) / (2.0 ** (N - 1) * math.gamma(N + D / 2.0)) * total
    return out


def moments_quantum(D: int, z: float, theta: float = 1.0, sign: int = +1, nmax: int = 4) -> dict:
    """I_{2N} of the Fermi-Dirac (sign +1) or Bose-Einstein (sign -1) weight
    omega(xi) = 1 / (z^-1 exp(|xi|^2 / 2 theta) + sign), i.e. the distribution at
    u = 0 (section on generalized polynomials: the weight is the equilibrium
    at rest), from the radial integral of eq. i2n-cont2, split at the Fermi
    edge |xi| = sqrt(2 theta ln z) when z > 1."""
    if sign > 0 and not z > 0:
        raise ValueError("fugacity must be > 0")
    if sign < 0 and not 0 < z < 1:
        raise ValueError("Bose-Einstein fugacity must be in (0, 1)")
    eta = math.log(z)

    def omega(r):
        a = r * r / (2.0 * theta) - eta
        if a > 700.0:
            return 0.0
        return 1.0 / (math.exp(a) + sign)

    edge = math.sqrt(2.0 * theta * eta) if eta > 0 else 0.0
    xi_max = math.sqrt(2.0 * theta * (max(eta, 0.0) + 80.0))
    breaks = [edge * f for f in (0.5, 0.9, 0.97, 1.0, 1.03, 1.1, 1.5)] if edge > 0 else [math.sqrt(2 * theta)]
    return moments_radial(D, omega, xi_max, nmax, breakpoints=breaks)


# ---------------------------------------------------------------------------
# Ratios and polynomial coefficients (paragraph after eq. H4)
# ---------------------------------------------------------------------------

def J(I: dict, L: int) -> float:
    """J_L = I_L^2 / (I_{L+2} I_{L-2}), L even."""
    return I[L] ** 2 / (I[L + 2] * I[L - 2])


def Delta_sq(I: dict, D: int, L: int) -> float:
    """Delta_L^2 = 2 / [(D + L) - J_L (D + L - 2)], L even."""
    return 2.0 / ((D + L) - J(I, L) * (D + L - 2))


@dataclass
class Coefficients:
    """The coefficients of P_0..P_3 for one weight and dimension, plus what the
    expansion needs.  c[K] = c_K, cp[K] = c'_K, cb[K] = cbar_K."""

    D: int
    I: dict
    c: dict = field(default_factory=dict)
    cp: dict = field(default_factory=dict)
    cb: dict = field(default_factory=dict)
    d: dict = field(default_factory=dict)  # d_4, d'_4, dbar_4 (keys d4, dp4, db4)

    @property
    def I0(self) -> float:
        return self.I[0]

    @property
    def J2(self) -> float:
        return J(self.I, 2)

    @property
    def J4(self) -> float:
        return J(self.I, 4)

    @property
    def c0_lattice(self) -> float:
        """Velocity scale of the d1v3 / d2v9 lattices: c_0 = sqrt(3 I_4 / I_2)
        (section "The Gaussian quadrature")."""
        return math.sqrt(3.0 * self.I[4] / self.I[2])


def coefficients(I: dict, D: int, kmax: int = 3) -> Coefficients:
    """c_K = 1/sqrt(I_{2K}); for K >= 2
    c'_K = -c_K (I_{2K-2} / I_{2K-4}) Delta_{2K-2},
    cbar_K = c_K (Delta_{2K-2} - 1) / (D + 2K - 4);
    and for K = 4 the coefficients of the isotropic term of P_4 (after eq. H4),
    with delta_L = 2 I_{L+2} I_{L-2} / Delta_L^2:
    d_4^2 = 8 delta_4^2 I_4 / (delta_2 [delta_2 delta_6 (D + 4) - delta_4^2 D]),
    d'_4 = -(d_4 / D) [I_0 / I_2 + I_4 delta_2 / (I_2 delta_4)] + 2 c_4 I_6 Delta_6 / (D I_4),
    dbar_4 = d_4 delta_2 / (D (D + 2) delta_4) + c_4 [D - 2 (D + 2) Delta_6] / (D (D + 2) (D + 4)).
    K = 4 (kmax = 4, for the fourth-order expansion) needs I up to I_8."""
    if 2 * kmax > max(I):
        kmax = max(I) // 2
    co = Coefficients(D=D, I=dict(I))
    for K in range(kmax + 1):
        co.c[K] = 1.0 / math.sqrt(I[2 * K])
        co.cp[K] = 0.0
        co.cb[K] = 0.0
    for K in range(2, kmax + 1):
        dlt = math.sqrt(Delta_sq(I, D, 2 * K - 2))
        co.cp[K] = -co.c[K] * (I[2 * K - 2] / I[2 * K - 4]) * dlt
        co.cb[K] = co.c[K] * (dlt - 1.0) / (D + 2 * K - 4)
    if kmax >= 4:
        dl = {L: 2.0 * I[L + 2] * I[L - 2] / Delta_sq(I, D, L) for L in (2, 4, 6)}
        D6 = math.sqrt(Delta_sq(I, D, 6))
        c4 = co.c[4]
        d4 = math.sqrt(8.0 * dl[4] ** 2 * I[4] / (dl[2] * (dl[2] * dl[6] * (D + 4) - dl[4] ** 2 * D)))
        co.d = {
            "d4": d4,
            "dp4": -(d4 / D) * (I[0] / I[2] + I[4] * dl[2] / (I[2] * dl[4])) + 2.0 * c4 * I[6] * D6 / (D * I[4]),
            "db4": d4 * dl[2] / (D * (D + 2) * dl[4]) + c4 * (D - 2 * (D + 2) * D6) / (D * (D + 2) * (D + 4)),
        }
    return co


# ---------------------------------------------------------------------------
# Polynomials P_{i1..iN}(xi)  (eqs. H0-H3) and coefficients A_{i1..iN}(u)  (eqs. A0-A3)
# ---------------------------------------------------------------------------

def _kd(i: int, j: int) -> float:
    return 1.0 if i == j else 0.0


def _sym6(a, idx) -> float:
    """a_i a_j delta_kl summed over the six ways to split (i, j, k, l) into two pairs."""
    i, j, k, l = idx
    return (a[i] * a[j] * _kd(k, l) + a[i] * a[k] * _kd(j, l) + a[i] * a[l] * _kd(j, k)
            + a[j] * a[k] * _kd(i, l) + a[j] * a[l] * _kd(i, k) + a[k] * a[l] * _kd(i, j))


def _delta4(idx) -> float:
    """delta_{i1 i2 i3 i4}, read as the isotropic four-index delta
    delta_ij delta_kl + delta_ik delta_jl + delta_il delta_jk (the tensor whose
    contraction with four vectors gives the isotropic moments of eq. i2n-cont)."""
    i, j, k, l = idx
    return _kd(i, j) * _kd(k, l) + _kd(i, k) * _kd(j, l) + _kd(i, l) * _kd(j, k)


def P(co: Coefficients, idx: tuple, xi) -> float:
    """The generalized polynomial with indices idx evaluated at the vector xi."""
    N = len(idx)
    xi = np.asarray(xi, dtype=np.float64)
    x2 = float(xi @ xi)
    if N == 0:
        return co.c[0]
    if N == 1:
        return co.c[1] * xi[idx[0]]
    if N == 2:
        i, j = idx
        return co.c[2] * xi[i] * xi[j] + (co.cb[2] * x2 + co.cp[2]) * _kd(i, j)
    if N == 3:
        i, j, k = idx
        sym = xi[i] * _kd(j, k) + xi[j] * _kd(i, k) + xi[k] * _kd(i, j)
        return co.c[3] * xi[i] * xi[j] * xi[k] + (co.cb[3] * x2 + co.cp[3]) * sym
    if N == 4:
        i, j, k, l = idx
        return (co.c[4] * xi[i] * xi[j] * xi[k] * xi[l]
                + (co.cb[4] * x2 + co.cp[4]) * _sym6(xi, idx)
                + (co.d["db4"] * x2 * x2 + co.d["dp4"] * x2 + co.d["d4"]) * _delta4(idx))
    raise ValueError("polynomials above fourth order are not part of this reference")


def A(co: Coefficients, idx: tuple, u) -> float:
    """A_{i1..iN}(u) = I_0 P'_{i1..iN}(u): the projection of f_eq(xi - u) on P_{i1..iN}."""
    N = len(idx)
    u = np.asarray(u, dtype=np.float64)
    u2 = float(u @ u)
    I0 = co.I0
    if N == 0:
        return I0 * co.c[0]
    if N == 1:
        return I0 * co.c[1] * u[idx[0]]
    if N == 2:
        i, j = idx
        return I0 * (co.c[2] * u[i] * u[j] + co.cb[2] * u2 * _kd(i, j))
    if N == 3:
        i, j, k = idx
        sym = u[i] * _kd(j, k) + u[j] * _kd(i, k) + u[k] * _kd(i, j)
        return I0 * (co.c[3] * u[i] * u[j] * u[k]
                     + (co.cp[3] * (1.0 - co.J2) + co.cb[3] * u2) * sym)
    if N == 4:
        # eq. A4; its sixth pair term is printed u_i2 u_i4 delta_i2i3 and read as
        # u_i2 u_i4 delta_i1i3 (the symmetric sum over the six pairings)
        c4, cb4, cp4 = co.c[4], co.cb[4], co.cp[4]
        db4, dp4 = co.d["db4"], co.d["dp4"]
        iso = (2.0 * co.I[2] / I0 * (cb4 + (co.D + 2) * db4) + dp4) * u2 + db4 * u2 * u2
        return I0 * (c4 * u[idx[0]] * u[idx[1]] * u[idx[2]] * u[idx[3]]
                     + ((1.0 - co.J2 * co.J4) * cp4 + cb4 * u2) * _sym6(u, idx)
                     + iso * _delta4(idx))
    raise ValueError("coefficients above fourth order are not part of this reference")


def S(co: Coefficients, xi, u, order: int = 3) -> float:
    """Truncated expansion of eq. expansao0 divided by the weight:
    S(xi, u) = sum_{N=0}^{order} (1/N!) sum_{i1..iN} A_{i1..iN}(u) P_{i1..iN}(xi),
    so that f_eq(xi - u) = omega(xi) S(xi, u)."""
    total = 0.0
    for N in range(order + 1):
        acc = 0.0
        for idx in itertools.product(range(co.D), repeat=N):
            acc += A(co, idx, u) * P(co, idx, xi)
        total += acc / math.factorial(N)
    return total


# ---------------------------------------------------------------------------
# Velocity sets and quadrature weights (eq. i2n-disc)
# ---------------------------------------------------------------------------

def velocity_set(name: str) -> np.ndarray:
    """Geometric velocities e_alpha (integer vectors), in a fixed order."""
    if name == "d1v3":
        return np.array([[0], [1], [-1]], dtype=np.int64)
    if name == "d2v9":
        return np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
                         [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.int64)
    if name == "d3v19":
        vs = [[0, 0, 0]]
        for a in range(3):
            for s in (1, -1):
                v = [0, 0, 0]
                v[a] = s
                vs.append(v)
        for a, b in ((0, 1), (0, 2), (1, 2)):
            for sa in (1, -1):
                for sb in (1, -1):
                    v = [0, 0, 0]
                    v[a], v[b] = sa, sb
                    vs.append(v)
        return np.array(vs, dtype=np.int64)
    if name == "d2v41":
        vs = []
        for E in D2V41_SHELLS:
            shell = [(x, y) for x in range(-4, 5) for y in range(-4, 5) if x * x + y * y == E]
            shell.sort(key=lambda v: math.atan2(v[1], v[0]) % (2 * math.pi))
            vs.extend(shell)
        return np.array(vs, dtype=np.int64)
    raise ValueError(name)


# The 41-velocity set for the fourth-order expansion (the paper gives none): the
# shells |e|^2 = 0, 1, 2, 4, 8, 9, 10, 13, 16 of the square lattice.  Its nine
# shell weights are fixed by the nine isotropic moment conditions of eq. i2n-disc
# through degree 8 (degree 9 holds by symmetry), which the fourth-order expansion
# needs (products P_4 P_4); with the zero-temperature Fermi-Dirac weight they are
# all positive for c_0 / sqrt(3 I_4 / I_2) in about [0.388, 0.395], and no smaller
# set of up to nine shells reaching three cells has positive weights.
D2V41_SHELLS = (0, 1, 2, 4, 8, 9, 10, 13, 16)


def lattice_dim(name: str) -> int:
    return {"d1v3": 1, "d2v9": 2, "d3v19": 3, "d2v41": 2}[name]


def lattice_scale(I: dict, lattice: str) -> float:
    """c_0 of a velocity set, xi_alpha = c_0 e_alpha.  d1v3, d2v9, d3v19:
    sqrt(3 I_4 / I_2) (section "The Gaussian quadrature").  d2v41: the scale with
    the largest smallest weight.  For the zero-temperature Fermi-Dirac weight that
    is where the weights of the shells |e|^2 = 1 (rising there) and |e|^2 = 16
    (falling) are equal, at c_0 / sqrt(3 I_4 / I_2) in [0.385, 0.3915]: a root
    found by bisection."""
    c_gq = math.sqrt(3.0 * I[4] / I[2])
    if lattice != "d2v41":
        return c_gq
    e = velocity_set("d2v41")
    shell = np.array([int(v @ v) for v in e])

    def gap(c):
        w, _ = quadrature_weights(I, "d2v41", cvel=c * c_gq, max_degree=8)
        return w[shell == 1][0] - w[shell == 16][0], w

    lo, hi = 0.385, 0.3915
    glo, _ = gap(lo)
    ghi, _ = gap(hi)
    if not glo * ghi < 0:
        raise ArithmeticError("d2v41: no scale with equal |e|^2 = 1 and 16 weights in the window")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        gm, _ = gap(mid)
        if gm * glo > 0:
            lo, glo = mid, gm
        else:
            hi = mid
        if hi - lo < 1e-16:
            break
    c = 0.5 * (lo + hi)
    _, w = gap(c)
    if not (w > 0).all():
        raise ArithmeticError("d2v41: weights not positive at the chosen scale")
    return c * c_gq


def isotropic_moment(I: dict, m) -> float:
    """int omega xi^m for a monomial with exponents m (eq. i2n-cont):
    I_{|m|} times the number of ways to pair equal indices, zero if any m_i is odd."""
    if any(k % 2 for k in m):
        return 0.0
    npair = 1
    for k in m:
        npair *= math.prod(range(k - 1, 0, -2)) if k > 1 else 1
    return I[sum(m)] * npair


def monomials(D: int, max_degree: int):
    for deg in range(max_degree + 1):
        for m in itertools.product(range(deg + 1), repeat=D):
            if sum(m) == deg:
                yield m


def quadrature_weights(I: dict, lattice: str, cvel: float | None = None,
                       max_degree: int = 5):
    """Weights w_alpha that make sum_alpha w_alpha xi_alpha^m equal the continuous
    moments for every monomial with |m| <= max_degree (eq. i2n-disc), with
    xi_alpha = c_0 e_alpha.  Velocities of equal |e|^2 share one weight (the
    symmetry of the sets used here).  Returns (w, residual): the residual is the
    largest violation of the moment conditions, relative to the moment scale."""
    e = velocity_set(lattice)
    D = e.shape[1]
    if cvel is None:
        cvel = math.sqrt(3.0 * I[4] / I[2])
    xi = cvel * e.astype(np.float64)
    shells = sorted(set(int(v @ v) for v in e))
    cls = np.array([shells.index(int(v @ v)) for v in e])
    rows, rhs, scale = [], [], []
    for m in monomials(D, max_degree):
        mono = np.prod(xi ** np.array(m), axis=1)
        rows.append([mono[cls == s].sum() for s in range(len(shells))])
        rhs.append(isotropic_moment(I, m))
        scale.append(I[min(sum(m) + (sum(m) % 2), max(I))])
    Am, b, sc = np.array(rows), np.array(rhs), np.array(scale)
    An, bn = Am / sc[:, None], b / sc
    wc, *_ = np.linalg.lstsq(An, bn, rcond=None)
    # iterative refinement with the residual formed in extended precision, so the
    # weights meet the conditions to the last bit (mass conservation of the
    # collision depends on sum_alpha w_alpha = I_0 holding exactly)
    ld = np.longdouble
    wl = wc.astype(ld)
    for _ in range(4):
        r = bn.astype(ld) - An.astype(ld) @ wl
        dw, *_ = np.linalg.lstsq(An, r.astype(np.float64), rcond=None)
        wl = wl + dw.astype(ld)
    wc = wl.astype(np.float64)
    resid = float(np.max(np.abs(Am @ wc - b) / sc))
    return wc[cls], resid


# ---------------------------------------------------------------------------
# A complete lattice model: what the LBM oracle needs
# ---------------------------------------------------------------------------

@dataclass
class LatticeModel:
    name: str
    D: int
    e: np.ndarray          # (Q, D) integer velocities
    w_hat: np.ndarray      # (Q,) normalized weights w_alpha / I_0
    opp: np.ndarray        # (Q,) index of -e_alpha
    co: Coefficients
    cvel: float            # c_0: xi_alpha = c_0 e_alpha, u = c_0 u0

    @property
    def Q(self) -> int:
        return self.e.shape[0]


def make_model(lattice: str = "d2v9", family: str = FD_T0, **kw) -> LatticeModel:
    """Build a lattice model for the zero-temperature Fermi-Dirac weight (the case of
    the section on electrons in metals), the Maxwell-Boltzmann weight, or the
    Fermi-Dirac / Bose-Einstein weights at fugacity z (keyword z, optional theta)."""
    D = lattice_dim(lattice)
    if family == FD_T0:
        I = moments_fd_t0(D, mu=kw.get("mu", 1.0))
    elif family == MB:
        I = moments_mb(D, rho0=kw.get("rho0", 1.0), theta=kw.get("theta", 1.0 / 3.0))
    elif family in (FD, BE):
        I = moments_quantum(D, kw["z"], theta=kw.get("theta", 1.0), sign=+1 if family == FD else -1)
    else:
        raise ValueError(family)
    return model_from_moments(lattice, I)


def model_from_moments(lattice: str, I: dict) -> LatticeModel:
    """The lattice model of a weight given by its moments I_L: polynomial
    coefficients, the scale c_0 (lattice_scale) and quadrature weights solving
    eq. i2n-disc (through degree 5 for the sets of the paper and the d3v19 set,
    through degree 9 for d2v41)."""
    D = lattice_dim(lattice)
    co = coefficients(I, D, kmax=4 if lattice == "d2v41" else 3)
    cvel = lattice_scale(I, lattice)
    w, resid = quadrature_weights(I, lattice, cvel=cvel, max_degree=9 if lattice == "d2v41" else 5)
    if resid > 1e-12:
        raise ArithmeticError(f"{lattice}: moment conditions not met (residual {resid:.3e})")
    e = velocity_set(lattice)
    opp = np.array([int(np.flatnonzero((e == -v).all(axis=1))[0]) for v in e])
    return LatticeModel(lattice, D, e, w / I[0], opp, co, cvel)


def feq_tensor(model: LatticeModel, n: float, u0, order: int = 3) -> np.ndarray:
    """Discrete equilibrium f_eq,alpha = n w_hat_alpha S(c_0 e_alpha, c_0 u0) by the
    tensor expansion (eq. expansao0 with A0-A3 and H0-H3), one population at a time."""
    u = model.cvel * np.asarray(u0, dtype=np.float64)
    return np.array([n * model.w_hat[a] * S(model.co, model.cvel * model.e[a], u, order)
                     for a in range(model.Q)])
