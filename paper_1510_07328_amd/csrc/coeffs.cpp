// Host (float64) construction of the collapsed per-class equilibrium: row a0 of
// the hot path, done once per configuration.
//
// Ratios of the weight's moments: at zero temperature the paper's closed forms
// J_L = 1 + 2/(L + D) and Delta_L^2 = (D + L)/2 (they follow from eq. sommerfeld
// at theta = 0 and the definitions after eq. H4); for the Gaussian weight every
// J and Delta is 1; for the Fermi-Dirac and Bose-Einstein weights at fugacity z,
// J_L from the complete integrals g_nu(z); for custom J_2, J_4 as given;
// Delta_L^2 = 2 / [(D + L) - J_L (D + L - 2)].
// Equilibrium: the geometric-space form of the discrete third-order
// equilibrium (section "The Gaussian quadrature"), whose terms split by
// truncation order as
//   order <= 2: 1 + (3/J2) eu + (9/(2 J2)) eu^2 + (9 (Delta2^2 - 1)/(2 J2 D)) e^2 u^2
//               - (3/2) Delta2^2 u^2
//   order 3:    + (3/(2 J2)) eu [ (1 - J2) J4 (D+2) Delta4^2 - 3 (1 - J2) J4 Delta4^2 e^2
//               - 3 J4 Delta4^2 u^2 + 9 J4 (Delta4^2 - 1)/(D + 2) e^2 u^2 + 3 J4 eu^2 ]
// and collapse on each shell |e|^2 = E to S - 1 = eu (l1 + c3 u^2 + k4 eu^2) + q eu^2 + s u^2.
// Weights: d1v3 (1 - J2/3, J2/6), d2v9 (1 - 5 J2/9, J2/9, J2/36) as printed with
// the quadrature; d3v19 (1 - 2 J2/3, J2/18, J2/36), from the same moment
// conditions through fourth order with c_0^2 = 3 I_4 / I_2.
#include <cmath>
#include <sstream>

#include "lbm_internal.h"

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

lbm_status build_model(const lbm_config *cfg, Model *m, std::string *err) {
    std::ostringstream os;
    if (!cfg || !m) {
        if (err) *err = "null argument";
        return LBM_ERR_ARG;
    }
    int D = 0, Q = 0;
    switch (cfg->lattice) {
    case LBM_D1V3: D = 1; Q = 3; break;
    case LBM_D2V9: D = 2; Q = 9; break;
    case LBM_D3V19: D = 3; Q = 19; break;
    default:
        if (err) *err = "unknown lattice";
        return LBM_ERR_ARG;
    }
    if (cfg->order != 2 && cfg->order != 3) {
        if (err) *err = "order must be 2 or 3";
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
    const double d2 = 2.0 / den2, d4 = 2.0 / den4;

    const double a1 = 3.0 / J2, a2 = 4.5 / J2, b1 = 4.5 * (d2 - 1.0) / (J2 * D), b0 = -1.5 * d2;
    double k0 = 0, k1 = 0, k2 = 0, k3 = 0, k4 = 0;
    if (cfg->order == 3) {
        const double K = 1.5 / J2;
        k0 = K * (1.0 - J2) * J4 * (D + 2) * d4;
        k1 = -3.0 * K * (1.0 - J2) * J4 * d4;
        k2 = -3.0 * K * J4 * d4;
        k3 = 9.0 * K * J4 * (d4 - 1.0) / (D + 2);
        k4 = 3.0 * K * J4;
    }
    double w[3];
    int ncls;
    if (D == 1) {
        w[0] = 1.0 - J2 / 3.0; w[1] = J2 / 6.0; w[2] = 0.0; ncls = 2;
    } else if (D == 2) {
        w[0] = 1.0 - 5.0 * J2 / 9.0; w[1] = J2 / 9.0; w[2] = J2 / 36.0; ncls = 3;
    } else {
        w[0] = 1.0 - 2.0 * J2 / 3.0; w[1] = J2 / 18.0; w[2] = J2 / 36.0; ncls = 3;
    }
    m->D = D;
    m->Q = Q;
    m->ncls = ncls;
    m->J2 = J2;
    m->J4 = J4;
    m->d2sq = d2;
    m->d4sq = d4;
    for (int k = 0; k < 3; ++k) {
        const double E = k;  // |e|^2 of shell k
        m->cls[k] = ClassCoef{w[k], a1 + k0 + k1 * E, a2, b1 * E + b0, k2 + k3 * E, k4};
    }
    return LBM_OK;
}

}  // namespace lbm
