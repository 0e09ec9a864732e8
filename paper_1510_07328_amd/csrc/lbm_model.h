// Per-class equilibrium coefficients from the moment ratios J_2 and J_4, for
// the host set-up (float64, once per configuration) and for the per-cell
// weights of LBM_W_FD_LOCAL (in the kernels' precision, every cell and step).
//
// Geometric-space form of the discrete third-order equilibrium (section "The
// Gaussian quadrature"), split by truncation order:
//   order <= 2: 1 + (3/J2) eu + (9/(2 J2)) eu^2 + (9 (Delta2^2 - 1)/(2 J2 D)) e^2 u^2
//               - (3/2) Delta2^2 u^2
//   order 3:    + (3/(2 J2)) eu [ (1 - J2) J4 (D+2) Delta4^2 - 3 (1 - J2) J4 Delta4^2 e^2
//               - 3 J4 Delta4^2 u^2 + 9 J4 (Delta4^2 - 1)/(D + 2) e^2 u^2 + 3 J4 eu^2 ],
// Delta_L^2 = 2 / [(D + L) - J_L (D + L - 2)] (paragraph after eq. H4), collapsed
// on each shell |e|^2 = E to S - 1 = eu (l1 + c3 u^2 + k4 eu^2) + q eu^2 + s u^2.
// Weights: d1v3 (1 - J2/3, J2/6), d2v9 (1 - 5 J2/9, J2/9, J2/36) as printed with
// the quadrature; d3v19 (1 - 2 J2/3, J2/18, J2/36), from the same moment
// conditions through fourth order with c_0^2 = 3 I_4 / I_2.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

// Constants of the Sommerfeld moments cut after (theta/mu)^2 (eq. sommerfeld):
// I_2N ~ mu^nu / Gamma(nu + 1) [1 + b_N (theta/mu)^2], b_N = (pi^2/6) nu (nu - 1),
// nu = N + D/2.  The powers of mu and the Gamma functions cancel in
// J_L = I_L^2 / (I_(L+2) I_(L-2)), leaving the zero-temperature values
// J2z = 1 + 2/(D + 2), J4z = 1 + 2/(D + 4) times ratios of the brackets.
struct SommerfeldJ {
    double b[4];
    double J2z, J4z;
};

inline SommerfeldJ sommerfeld_j(int D) {
    SommerfeldJ s{};
    const double pi2_6 = 1.6449340668482264;  // pi^2 / 6
    for (int N = 0; N < 4; ++N) {
        const double nu = N + 0.5 * D;
        s.b[N] = pi2_6 * nu * (nu - 1.0);
    }
    s.J2z = 1.0 + 2.0 / (D + 2);
    s.J4z = 1.0 + 2.0 / (D + 4);
    return s;
}

template <typename T>
struct ClassSet {
    T w[3], l1[3], q[3], s[3], c3[3], k4[3];
    T d2sq, d4sq;
};

template <typename T>
__host__ __device__ inline void class_coefs(int D, T J2, T J4, bool order3, ClassSet<T> &o) {
    const T d2 = T(2) / (T(D + 2) - J2 * T(D));
    const T d4 = T(2) / (T(D + 4) - J4 * T(D + 2));
    const T a1 = T(3) / J2, a2 = T(4.5) / J2, b1 = T(4.5) * (d2 - T(1)) / (J2 * T(D)), b0 = T(-1.5) * d2;
    T k0 = T(0), k1 = T(0), k2 = T(0), k3 = T(0), k4 = T(0);
    if (order3) {
        const T K = T(1.5) / J2;
        k0 = K * (T(1) - J2) * J4 * T(D + 2) * d4;
        k1 = T(-3) * K * (T(1) - J2) * J4 * d4;
        k2 = T(-3) * K * J4 * d4;
        k3 = T(9) * K * J4 * (d4 - T(1)) / T(D + 2);
        k4 = T(3) * K * J4;
    }
    if (D == 1) {
        o.w[0] = T(1) - J2 / T(3); o.w[1] = J2 / T(6); o.w[2] = T(0);
    } else if (D == 2) {
        o.w[0] = T(1) - T(5) * J2 / T(9); o.w[1] = J2 / T(9); o.w[2] = J2 / T(36);
    } else {
        o.w[0] = T(1) - T(2) * J2 / T(3); o.w[1] = J2 / T(18); o.w[2] = J2 / T(36);
    }
    for (int k = 0; k < 3; ++k) {
        const T E = T(k);  // |e|^2 of shell k
        o.l1[k] = a1 + k0 + k1 * E;
        o.q[k] = a2;
        o.s[k] = b1 * E + b0;
        o.c3[k] = k2 + k3 * E;
        o.k4[k] = k4;
    }
    o.d2sq = d2;
    o.d4sq = d4;
}

}  // namespace lbm
