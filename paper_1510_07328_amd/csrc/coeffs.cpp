// Host (float64) construction of the collapsed per-class equilibrium: row a0 of
// the hot path, done once per configuration.
//
// Ratios of the weight's moments: at zero temperature the paper's closed forms
// J_L = 1 + 2/(L + D) and Delta_L^2 = (D + L)/2 (they follow from eq. sommerfeld
// at theta = 0 and the definitions after eq. H4); for the Gaussian weight every
// J and Delta is 1; for the Fermi-Dirac and Bose-Einstein weights at fugacity z,
// J_L from the complete integrals g_nu(z); for custom J_2, J_4 as given;
// Delta_L^2 = 2 / [(D + L) - J_L (D + L - 2)].
// The per-class equilibrium coefficients follow from J_2 and J_4 (lbm_model.h).
#include <cmath>
#include <sstream>
#include <utility>

#include "lbm_internal.h"
#include "lbm_model.h"

namespace lbm {

namespace {

// 20-point Gauss-Legendre nodes and weights on [-1, 1] (positive half; the rule
// is symmetric), computed once by Newton iteration on P_20.
struct GaussLegendre20 {
    double x[10], w[10];
    GaussLegendre20() {
        const int n = 20;
        for (int i = 0; i < n / 2; ++i) {
            double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                const double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

// Complete Fermi-Dirac (s = +1) or Bose-Einstein (s = -1) integral
//   g_nu(z) = (1 / Gamma(nu)) int_0^inf x^(nu-1) / (z^-1 e^x + s) dx,  eta = ln z,
// the function that gives the weight's moments I_2N = (2 pi)^(D/2) theta^(N+D/2)
// g_(N+D/2)(z) (the paragraph before eq. sommerfeld; the 1/Gamma(nu) is the factor
// the paper's own Sommerfeld and Maxwell-Boltzmann limits require).  With x = t^2
// the integrand 2 t^(2 nu - 1) / (e^(t^2 - eta) + s) is smooth for 2 nu - 1 a
// non-negative integer (nu = N + D/2); composite 20-point Gauss-Legendre on panels
// fine enough to resolve the Fermi edge at t = sqrt(eta), up to where the
// integrand is below e^-60 of its scale.
double g_nu(double nu, double eta, int s) {
    static const GaussLegendre20 gl;
    const double t_edge = eta > 0.0 ? std::sqrt(eta) : 0.0;
    const double T = std::sqrt((eta > 0.0 ? eta : 0.0) + 60.0);
    const double h = std::fmin(0.25, 0.125 / std::fmax(t_edge, 1.0));
    const int panels = (int)std::ceil(T / h);
    const double hp = T / panels;
    double sum = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double c = (p + 0.5) * hp, r = 0.5 * hp;
        double acc = 0.0;
        for (int i = 0; i < 10; ++i)
            for (int sg = -1; sg <= 1; sg += 2) {
                const double t = c + sg * r * gl.x[i];
                const double e = std::exp(t * t - eta);
                acc += gl.w[i] * 2.0 * std::pow(t, 2.0 * nu - 1.0) / (e + s);
            }
        sum += r * acc;
    }
    return sum / std::tgamma(nu);
}

}  // namespace

// ---------------------------------------------------------------------------
// The 41-velocity set and the fourth-order expansion (row f3).
//
// Velocities: the shells |e|^2 = 0, 1, 2, 4, 8, 9, 10, 13, 16.  Their nine
// weights solve eq. i2n-disc for the nine even monomials x^a y^b (a >= b,
// a + b <= 8) of the zero-temperature Fermi-Dirac weight, rows scaled by
// I_(a+b):  sum_s w_s sum_(v in s) (c v_x)^a (c v_y)^b = I_(a+b) (a-1)!! (b-1)!!
// (odd degrees vanish by symmetry, so the set is exact through degree 9).
// The scale c: where the weights of the shells |e|^2 = 1 and 16 are equal, the
// largest smallest weight, c / sqrt(3 I_4 / I_2) in [0.385, 0.3915].
//
// Equilibrium: S = sum_(N <= order) (1/N!) A_N : P_N with P_N of eqs. H0-H4 and
// A_N of eqs. A0-A4, contracted in closed form in a = u.xi, U = u^2, X = xi^2
// (delta_ijkl the isotropic four-index delta; Sym3(v) = v_i delta_jk + 2 more,
// S6(v) = v_i v_j delta_kl + 5 more):
//   A1.P1 = I0 c1^2 a
//   A2:P2 = I0 [c2^2 a^2 + U (X (2 c2 cb2 + D cb2^2) + cp2 (c2 + D cb2))]
//   A3:P3 = I0 a [c3^2 a^2 + U (3 c3 (cb3 X + cp3) + 3 c3 cb3 X + (3D+6) cb3 (cb3 X + cp3))
//                 + (1 - J2) cp3 (3 c3 X + (3D+6) (cb3 X + cp3))]
//   A4:P4 = I0 [c4^2 a^4 + a^2 U (6 c4 G + 6 c4 X y1 + (6D+24) G y1) + a^2 (6 c4 X y0 + (6D+24) G y0)
//               + U^2 (3 c4 H + 6 G X y1 + 6 (D+2) H y1 + W z2) + U (6 G X y0 + 6 (D+2) H y0 + W z1)]
// with G = cb4 X + cp4, H = db4 X^2 + dp4 X + d4, y0 = (1 - J2 J4) cp4, y1 = cb4,
// z1 = 2 (I2/I0) (cb4 + (D+2) db4) + dp4, z2 = db4, W = 3 c4 X^2 + 6 (D+2) G X + 3 D (D+2) H,
// from u(x)u(x)u(x)u : xi(x)xi(x)xi(x)xi = a^4, u^4 : S6(xi) = 6 a^2 U, u^4 : delta = 3 U^2,
// S6(u) : S6(xi) = (6D+24) a^2 + 6 U X, S6(u) : delta = 6 (D+2) U, delta : delta = 3 D (D+2),
// Sym3(u) : Sym3(xi) = (3D+6) a.  With xi = c e and u = c u0 this collapses per shell.
namespace {

constexpr int kShells41[9] = {0, 1, 2, 4, 8, 9, 10, 13, 16};
constexpr int kMono41[9][2] = {{0, 0}, {2, 0}, {4, 0}, {2, 2}, {6, 0}, {4, 2}, {8, 0}, {6, 2}, {4, 4}};

double dfact(int k) {  // (k - 1)!! for even k
    double r = 1.0;
    for (int j = k - 1; j > 1; j -= 2) r *= j;
    return r;
}

// Gaussian elimination with partial pivoting, n <= 9.
bool solve9(double A[9][9], double *b, int n) {
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0) return false;
        if (piv != col) {
            for (int k = 0; k < n; ++k) std::swap(A[piv][k], A[col][k]);
            std::swap(b[piv], b[col]);
        }
        for (int r = col + 1; r < n; ++r) {
            const double f = A[r][col] / A[col][col];
            for (int k = col; k < n; ++k) A[r][k] -= f * A[col][k];
            b[r] -= f * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double acc = b[r];
        for (int k = r + 1; k < n; ++k) acc -= A[r][k] * b[k];
        b[r] = acc / A[r][r];
    }
    return true;
}

// per-velocity shell weights at scale c; I[N] = I_(2N)
bool weights41(const double *I, double c, double *w) {
    double A[9][9], b[9];
    for (int r = 0; r < 9; ++r) {
        const int ax = kMono41[r][0], ay = kMono41[r][1];
        const double scale = I[(ax + ay) / 2];
        for (int k = 0; k < 9; ++k) {
            double sum = 0.0;
            for (int x = -4; x <= 4; ++x)
                for (int y = -4; y <= 4; ++y)
                    if (x * x + y * y == kShells41[k]) sum += std::pow(c * x, ax) * std::pow(c * y, ay);
            A[r][k] = sum / scale;
        }
        b[r] = I[(ax + ay) / 2] * dfact(ax) * dfact(ay) / scale;
    }
    if (!solve9(A, b, 9)) return false;
    for (int k = 0; k < 9; ++k) w[k] = b[k];
    return true;
}

lbm_status build_d2v41(const lbm_config *cfg, Model *m, std::string *err) {
    if (cfg->weight != LBM_W_FD_T0) {
        if (err) *err = "d2v41 is built for the zero-temperature Fermi-Dirac weight only";
        return LBM_ERR_UNSUPPORTED;
    }
    if (cfg->order < 2 || cfg->order > 4) {
        if (err) *err = "d2v41: order must be 2, 3 or 4";
        return LBM_ERR_UNSUPPORTED;
    }
    const int D = 2;
    double I[5];  // I_(2N) at mu = 1: (2 pi)^(D/2) mu^(N + D/2) / Gamma(N + D/2 + 1) = 2 pi / (N + 1)!
    {
        double fac = 1.0;
        for (int N = 0; N < 5; ++N) {
            fac *= (N + 1);
            I[N] = 2.0 * M_PI / fac;
        }
    }
    auto J = [&](int L) { return I[L / 2] * I[L / 2] / (I[L / 2 + 1] * I[L / 2 - 1]); };
    auto Dsq = [&](int L) { return 2.0 / ((D + L) - J(L) * (D + L - 2)); };
    double c[5], cp[5] = {0, 0, 0, 0, 0}, cb[5] = {0, 0, 0, 0, 0};
    for (int K = 0; K < 5; ++K) c[K] = 1.0 / std::sqrt(I[K]);
    for (int K = 2; K < 5; ++K) {
        const double dl = std::sqrt(Dsq(2 * K - 2));
        cp[K] = -c[K] * (I[K - 1] / I[K - 2]) * dl;
        cb[K] = c[K] * (dl - 1.0) / (D + 2 * K - 4);
    }
    double del[8];  // delta_L = 2 I_(L+2) I_(L-2) / Delta_L^2, L = 2, 4, 6
    for (int L = 2; L <= 6; L += 2) del[L] = 2.0 * I[L / 2 + 1] * I[L / 2 - 1] / Dsq(L);
    const double D6 = std::sqrt(Dsq(6));
    const double d4 = std::sqrt(8.0 * del[4] * del[4] * I[2] / (del[2] * (del[2] * del[6] * (D + 4) - del[4] * del[4] * D)));
    const double dp4 = -(d4 / D) * (I[0] / I[1] + I[2] * del[2] / (I[1] * del[4])) + 2.0 * c[4] * I[3] * D6 / (D * I[2]);
    const double db4 = d4 * del[2] / (D * (D + 2) * del[4]) + c[4] * (D - 2 * (D + 2) * D6) / (D * (D + 2) * (D + 4));
    const double J2 = J(2), J4 = J(4);

    // scale: bisection on w(|e|^2 = 1) - w(|e|^2 = 16)
    const double cgq = std::sqrt(3.0 * I[2] / I[1]);
    double w[9];
    auto gap = [&](double s) {
        if (!weights41(I, s * cgq, w)) return std::nan("");
        return w[1] - w[8];
    };
    double lo = 0.385, hi = 0.3915, glo = gap(lo);
    if (!(glo * gap(hi) < 0.0)) {
        if (err) *err = "d2v41: no scale with equal |e|^2 = 1 and 16 weights";
        return LBM_ERR_ARG;
    }
    for (int it = 0; it < 200 && hi - lo > 1e-16; ++it) {
        const double mid = 0.5 * (lo + hi), gm = gap(mid);
        if (gm * glo > 0.0) {
            lo = mid;
            glo = gm;
        } else {
            hi = mid;
        }
    }
    const double scale = 0.5 * (lo + hi);
    gap(scale);
    for (int k = 0; k < 9; ++k)
        if (!(w[k] > 0.0)) {
            if (err) *err = "d2v41: a weight is not positive";
            return LBM_ERR_ARG;
        }

    const double cv = scale * cgq, c2v = cv * cv;
    const int order = cfg->order;
    m->D = D;
    m->Q = 41;
    m->ncls = 9;
    m->J2 = J2;
    m->J4 = J4;
    m->d2sq = Dsq(2);
    m->d4sq = Dsq(4);
    m->scale = scale;
    const double I0 = I[0];
    for (int k = 0; k < 9; ++k) {
        const double E = kShells41[k], X = c2v * E;
        ClassCoef cc{};
        cc.w = w[k] / I0;
        // order 1 and 2
        cc.l1 = I0 * c[1] * c[1] * c2v;
        cc.q = 0.5 * I0 * c[2] * c[2] * c2v * c2v;
        cc.s = 0.5 * I0 * c2v * (X * (2.0 * c[2] * cb[2] + D * cb[2] * cb[2]) + cp[2] * (c[2] + D * cb[2]));
        if (order >= 3) {
            const double f = I0 / 6.0 * c2v;
            cc.k4 = f * c[3] * c[3] * c2v * c2v;
            cc.c3 = f * c2v *
                    (3.0 * c[3] * (cb[3] * X + cp[3]) + 3.0 * c[3] * cb[3] * X + (3.0 * D + 6.0) * cb[3] * (cb[3] * X + cp[3]));
            cc.l1 += f * (1.0 - J2) * cp[3] * (3.0 * c[3] * X + (3.0 * D + 6.0) * (cb[3] * X + cp[3]));
        }
        if (order >= 4) {
            const double G = cb[4] * X + cp[4], H = db4 * X * X + dp4 * X + d4;
            const double y0 = (1.0 - J2 * J4) * cp[4], y1 = cb[4];
            const double z1 = 2.0 * (I[1] / I0) * (cb[4] + (D + 2) * db4) + dp4, z2 = db4;
            const double W = 3.0 * c[4] * X * X + 6.0 * (D + 2) * G * X + 3.0 * D * (D + 2) * H;
            const double f = I0 / 24.0;
            const double c4v = c2v * c2v;
            cc.p4 = f * c[4] * c[4] * c4v * c4v;
            cc.r4 = f * c4v * c2v * (6.0 * c[4] * G + 6.0 * c[4] * X * y1 + (6.0 * D + 24.0) * G * y1);
            cc.q += f * c4v * (6.0 * c[4] * X * y0 + (6.0 * D + 24.0) * G * y0);
            cc.t4 = f * c4v * (3.0 * c[4] * H + 6.0 * G * X * y1 + 6.0 * (D + 2) * H * y1 + W * z2);
            cc.s += f * c2v * (6.0 * G * X * y0 + 6.0 * (D + 2) * H * y0 + W * z1);
        }
        m->cls[k] = cc;
    }
    return LBM_OK;
}

}  // namespace

lbm_status build_model(const lbm_config *cfg, Model *m, std::string *err) {
    std::ostringstream os;
    if (!cfg || !m) {
        if (err) *err = "null argument";
        return LBM_ERR_ARG;
    }
    int D = 0, Q = 0;
    m->lattice = cfg->lattice;
    m->scale = 1.0;
    switch (cfg->lattice) {
    case LBM_D1V3: D = 1; Q = 3; break;
    case LBM_D2V9: D = 2; Q = 9; break;
    case LBM_D3V19: D = 3; Q = 19; break;
    case LBM_D2V41: D = 2; Q = 41; break;
    default:
        if (err) *err = "unknown lattice";
        return LBM_ERR_ARG;
    }
    if (cfg->lattice == LBM_D2V41) {
        if (!(cfg->tau > 0.5) || !std::isfinite(cfg->tau)) {
            if (err) *err = "tau must be finite and > 1/2";
            return LBM_ERR_ARG;
        }
        return build_d2v41(cfg, m, err);
    }
    if (cfg->order != 2 && cfg->order != 3) {
        if (err) *err = cfg->order == 4 ? "order 4 needs the 41-velocity set (LBM_D2V41)" : "order must be 2 or 3";
        return LBM_ERR_UNSUPPORTED;
    }
    if (!(cfg->tau > 0.5) || !std::isfinite(cfg->tau)) {
        if (err) *err = "tau must be finite and > 1/2";
        return LBM_ERR_ARG;
    }
    double J2, J4;
    if (cfg->weight == LBM_W_FD_T0) {
        J2 = 1.0 + 2.0 / (2 + D);
        J4 = 1.0 + 2.0 / (4 + D);
    } else if (cfg->weight == LBM_W_MB) {
        J2 = 1.0;
        J4 = 1.0;
    } else if (cfg->weight == LBM_W_FD || cfg->weight == LBM_W_BE) {
        const double z = cfg->fugacity;
        const int sgn = cfg->weight == LBM_W_FD ? 1 : -1;
        if (!(z > 0.0) || !std::isfinite(z) || (sgn < 0 && !(z < 1.0))) {
            if (err) *err = sgn > 0 ? "fugacity must be finite and > 0" : "Bose-Einstein fugacity must be in (0, 1)";
            return LBM_ERR_ARG;
        }
        if (sgn > 0 && std::log(z) > 1e4) {
            if (err) *err = "fugacity too large (use LBM_W_FD_T0 for the zero-temperature limit)";
            return LBM_ERR_ARG;
        }
        const double eta = std::log(z), h = 0.5 * D;
        double g[4];  // g_(N + D/2), N = 0..3
        for (int N = 0; N < 4; ++N) g[N] = g_nu(N + h, eta, sgn);
        J2 = g[1] * g[1] / (g[2] * g[0]);  // J_L = I_L^2 / (I_(L+2) I_(L-2)); theta cancels
        J4 = g[2] * g[2] / (g[3] * g[1]);
    } else if (cfg->weight == LBM_W_FD_LOCAL) {
        const double r0 = cfg->theta_over_mu;
        if (!(r0 >= 0.0 && r0 <= 0.5)) {
            if (err) *err = "theta_over_mu must be in [0, 0.5] (Sommerfeld limit)";
            return LBM_ERR_ARG;
        }
        if (cfg->obstacles || cfg->force[0] != 0.0 || cfg->force[1] != 0.0 || cfg->force[2] != 0.0) {
            if (err) *err = "per-cell weights are not supported with obstacles or a body force";
            return LBM_ERR_UNSUPPORTED;
        }
        // the reference cell (n = rho_ref, mu = mu_ref): J_L of eq. sommerfeld at theta/mu = r0
        const SommerfeldJ sj = sommerfeld_j(D);
        J2 = sj.J2z * (1.0 + sj.b[1] * r0 * r0) * (1.0 + sj.b[1] * r0 * r0) /
             ((1.0 + sj.b[0] * r0 * r0) * (1.0 + sj.b[2] * r0 * r0));
        J4 = sj.J4z * (1.0 + sj.b[2] * r0 * r0) * (1.0 + sj.b[2] * r0 * r0) /
             ((1.0 + sj.b[1] * r0 * r0) * (1.0 + sj.b[3] * r0 * r0));
        m->local = 1;
        m->r0 = r0;
    } else if (cfg->weight == LBM_W_CUSTOM) {
        J2 = cfg->J2;
        J4 = cfg->J4;
        if (!(J2 > 0) || !(J4 > 0) || !std::isfinite(J2) || !std::isfinite(J4)) {
            if (err) *err = "custom J2, J4 must be finite and positive";
            return LBM_ERR_ARG;
        }
    } else {
        if (err) *err = "unknown weight family";
        return LBM_ERR_ARG;
    }
    const double den2 = (D + 2) - J2 * D, den4 = (D + 4) - J4 * (D + 2);
    if (!(den2 > 0) || !(den4 > 0)) {
        if (err) *err = "J2/J4 give a non-positive Delta^2";
        return LBM_ERR_ARG;
    }
    ClassSet<double> cs;
    class_coefs<double>(D, J2, J4, cfg->order == 3, cs);
    m->D = D;
    m->Q = Q;
    m->ncls = D == 1 ? 2 : 3;
    m->J2 = J2;
    m->J4 = J4;
    m->d2sq = cs.d2sq;
    m->d4sq = cs.d4sq;
    for (int k = 0; k < 3; ++k)
        m->cls[k] = ClassCoef{cs.w[k], cs.l1[k], cs.q[k], cs.s[k], cs.c3[k], cs.k4[k], 0.0, 0.0, 0.0};
    return LBM_OK;
}

}  // namespace lbm
