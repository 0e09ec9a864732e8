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
    for (int k = 0; k < 3; ++k) m->cls[k] = ClassCoef{cs.w[k], cs.l1[k], cs.q[k], cs.s[k], cs.c3[k], cs.k4[k]};
    return LBM_OK;
}

}  // namespace lbm
