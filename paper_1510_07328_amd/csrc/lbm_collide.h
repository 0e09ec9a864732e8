// The fused collision shared by every step kernel (plain field steps and the
// batched tube sweep): moments, equilibrium from the per-class polynomial,
// BGK relaxation.  Included by the kernel sources only.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"
#include "lbm_model.h"

namespace lbm {

// ---------------------------------------------------------------------------
// The kernels are compiled without floating-point contraction and every fused
// multiply-add is written out, so the arithmetic is fixed by the source and
// identical in every kernel that inlines it.
//
// The relaxation is applied as increments d_a = (g_eq,a - g_a) / tau.  In exact
// arithmetic the equilibrium has the cell's mass and momentum, so
// sum_a d_a = 0 and sum_a d_a e_a = 0; those identities are used to form d for
// the +e_d populations (momentum) and for the rest population (mass) from the
// others.  The collision then conserves mass and momentum up to the final
// rounding of g_a + d_a, instead of inheriting the rounding of the moment sums
// and of the weights (which in float32 drifts the conserved fields by about
// 1e-8 relative per step).
//
// The conserved moments dn = sum_a g_a and j = sum_a g_a e_a are accumulated in
// float64, where the sum of float32 populations is exact, and rounded once:
// summed in float32, their partial sums carry rounding errors of the size of
// the populations (|g| ~ w dn), which the equilibrium passes on to every
// population each step; relative to a small velocity that was the largest
// float32 error of the step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class L>
struct PlusAxis;  // population index of +e_d for d < D
template <>
struct PlusAxis<D1Q3> { static constexpr int p[3] = {1, -1, -1}; };
template <>
struct PlusAxis<D2Q9> { static constexpr int p[3] = {1, 2, -1}; };
template <>
struct PlusAxis<D3Q19> { static constexpr int p[3] = {1, 3, 5}; };
template <>
struct PlusAxis<D2Q41> { static constexpr int p[3] = {1, 3, -1}; };

// Population pairs (a, -a) of each set: the equilibrium polynomial is
// evaluated once per pair, since e_-a . u = -(e_a . u) exactly (the results are
// identical to evaluating each population on its own).
template <class L>
struct Pairs;
template <>
struct Pairs<D1Q3> { static constexpr int n = 1; static constexpr int p[1] = {1}; };
template <>
struct Pairs<D2Q9> { static constexpr int n = 4; static constexpr int p[4] = {1, 2, 5, 6}; };
template <>
struct Pairs<D3Q19> {
    static constexpr int n = 9;
    static constexpr int p[9] = {1, 3, 5, 7, 9, 11, 13, 15, 17};
};
template <>
struct Pairs<D2Q41> {
    static constexpr int n = 20;
    static constexpr int p[20] = {1, 3, 5, 7, 9, 11, 13, 15, 17, 19, 21, 23, 25, 27, 29, 31, 33, 35, 37, 39};
};

// acc + e g for an integer link component e (exact add or subtract for e = +-1,
// as every set with one-cell links uses; a multiply-add for longer links)
// (e is a compile-time constant after the callers' loops are unrolled)
template <typename T>
__device__ __forceinline__ T add_e(T acc, T g, int e) {
    if (e == 0) return acc;
    if (e == 1) return acc + g;
    if (e == -1) return acc - g;
    return fmaT(T(e), g, acc);
}

// Accumulates e v into acc, where the first term (started = false) sets acc
// instead of being added to zero: the value is that of the sum from zero (only
// the sign of a zero can differ), without the add of 0 that the compiler must
// otherwise keep for signed zeros.
template <typename T>
__device__ __forceinline__ void acc_e(T &acc, bool &started, T v, int e) {
    if (e == 0) return;
    if (!started) {
        acc = e == 1 ? v : e == -1 ? -v : T(e) * v;
        started = true;
        return;
    }
    acc = add_e(acc, v, e);
}

// 1 / n.  float: the hardware reciprocal (1 ulp) refined by one Newton-Raphson
// step, r + r (1 - n r), within one ulp of the rounded quotient at a third of
// the cost of the correctly rounded division; double: the division.
__device__ __forceinline__ float recip(float n) {
    const float r = __builtin_amdgcn_rcpf(n);
    return fmaT(fmaT(-n, r, 1.0f), r, r);
}
__device__ __forceinline__ double recip(double n) { return 1.0 / n; }

// Per-class coefficients as the collision reads them (NC classes).
template <typename T, int NC>
struct Classes {
    T w[NC], l1[NC], q[NC], s[NC], c3[NC], k4[NC], p4[NC], r4[NC], t4[NC];
};

// Per-cell weights (LBM_W_FD_LOCAL): J_2, J_4 of a cell of density n = rho_ref + dn
// from the Sommerfeld moments at its chemical potential, then its coefficients;
// dJ2 = J_2 - J_2,ref is returned on its own (the weights shift by dJ2 times a
// constant per class).  D = 2: mu / mu_ref = n / rho_ref exactly.  D = 1, 3:
// s = sqrt(mu / mu_ref) solves s^D + b_0 r2 s^(D-4) = x rhs (the I_0 relation
// multiplied out), by four Newton steps from the zero-temperature root x^(1/D).
template <class L, typename T>
__device__ __forceinline__ void local_classes(const LocalW<T> &p, T n, T dn, bool order3, ClassSet<T> &cs,
                                              T &dJ2) {
    T dm;  // mu / mu_ref - 1
    if constexpr (L::D == 2) {
        dm = dn * p.inv_rho;
    } else {
        const T x = n * p.inv_rho;
        const T a = p.b[0] * p.r2, y = x * p.rhs;
        T sq = L::D == 1 ? x : cbrt(x);
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const T is = T(1) / sq, is2 = is * is;
            T F, dF;
            if constexpr (L::D == 1) {
                F = fmaT(a * is2, is, sq) - y;
                dF = fmaT(T(-3) * a, is2 * is2, T(1));
            } else {
                F = fmaT(sq * sq, sq, a * is) - y;
                dF = fmaT(T(3) * sq, sq, -a * is2);
            }
            sq = sq - F / dF;
        }
        dm = (sq - T(1)) * (sq + T(1));
    }
    const T m = T(1) + dm;
    const T dt = -p.r2 * dm * (T(2) + dm) / (m * m);  // r2 / m^2 - r2
    const T B0 = fmaT(p.b[0], dt, p.Br[0]), B1 = fmaT(p.b[1], dt, p.Br[1]);
    const T B2 = fmaT(p.b[2], dt, p.Br[2]), B3 = fmaT(p.b[3], dt, p.Br[3]);
    dJ2 = p.J2z * dt * fmaT(p.P2, dt, p.P1) * p.inv_br02 / (B0 * B2);
    const T J4 = p.J4z * B2 * B2 / (B1 * B3);
    class_coefs<T>(L::D, p.J2r + dJ2, J4, order3, cs);
}

// dw_a / dJ_2 per class (the weights are linear in J_2)
template <class L>
struct WeightSlope;
template <>
struct WeightSlope<D1Q3> { static constexpr double v[3] = {-1.0 / 3.0, 1.0 / 6.0, 0.0}; };
template <>
struct WeightSlope<D2Q9> { static constexpr double v[3] = {-5.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0}; };
template <>
struct WeightSlope<D3Q19> { static constexpr double v[3] = {-2.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0}; };

// ORDER3 = false skips the third-order terms (their coefficients are zero at
// second order, so the result is the same).
//
// FORCE = true adds a constant body force F (force density per cell and step)
// by the exact difference of equilibria, d_a += g_eq,a(n, u + F/n) - g_eq,a(n, u).
// The difference is formed from the polynomial itself, with a = e.u, b = e.F/n
// and w2 = |u + F/n|^2 - |u|^2 = (F/n).(2u + F/n):
//   S(u + F/n) - S(u) = [q b (2a + b) + s w2]                               (even in e)
//                     + [l1 b + c3 (u^2 b + w2 (a + b)) + k4 b (3a^2 + 3ab + b^2)]   (odd in e),
// so no two nearly equal equilibria are subtracted.  Its mass is zero and its
// momentum is F; the exact-moment step below sets sum_a d_a e_a = F.
//
// LOCAL = true takes the weights and coefficients of each cell from its density
// (local_classes); the populations stay deviations from the reference weights
// c.w times rho_ref, so g_eq,a = w_a(n) [dn + n (S_a - 1)] + dw_a rho_ref with
// w_a(n) = w_a,ref + dw_a and dw_a = dJ2 dw/dJ_2.
template <class L, typename T, bool ORDER3 = true, bool FORCE = false, bool LOCAL = false>
__device__ __forceinline__ void collide(T (&g)[L::Q], const Coef<T> &c, const T *F = nullptr) {
    static_assert(!(FORCE && LOCAL), "body force and per-cell weights are not combined");
    static_assert(!(L::O4 && (FORCE || LOCAL)), "the fourth-order set runs without force and local weights");
    // conserved moments accumulated in float64 (exact for float32 populations),
    // each rounded once to T
    double dnA = double(g[0]), jA[3] = {0.0, 0.0, 0.0};
    bool js[3] = {false, false, false};
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const double gq = double(g[q]);
        if (q > 0) dnA += gq;
#pragma unroll
        for (int d = 0; d < L::D; ++d) acc_e(jA[d], js[d], gq, L::e[q][d]);
    }
    const T dn = T(dnA);
    const T n = T(double(c.rho_ref) + dnA);
    const T inv_n = recip(n);
    T u[3] = {T(0), T(0), T(0)};
    T u2 = T(0);
#pragma unroll
    for (int d = 0; d < L::D; ++d) {
        u[d] = T(jA[d]) * inv_n;
        u2 = fmaT(u[d], u[d], u2);
    }
    Classes<T, L::NC> K;
    T dw[L::NC] = {};
    if constexpr (LOCAL) {
        T dJ2;
        ClassSet<T> loc;
        local_classes<L, T>(c.loc, n, dn, ORDER3, loc, dJ2);
#pragma unroll
        for (int k = 0; k < L::NC; ++k) {
            dw[k] = dJ2 * T(WeightSlope<L>::v[k]);
            K.w[k] = c.w[k] + dw[k];
            K.l1[k] = loc.l1[k];
            K.q[k] = loc.q[k];
            K.s[k] = loc.s[k];
            K.c3[k] = loc.c3[k];
            K.k4[k] = loc.k4[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < L::NC; ++k) {
            K.w[k] = c.w[k];
            K.l1[k] = c.l1[k];
            K.q[k] = c.q[k];
            K.s[k] = c.s[k];
            K.c3[k] = c.c3[k];
            K.k4[k] = c.k4[k];
            if constexpr (L::O4) {
                K.p4[k] = c.p4[k];
                K.r4[k] = c.r4[k];
                K.t4[k] = c.t4[k];
            }
        }
    }
    T dl[3] = {T(0), T(0), T(0)}, w2 = T(0);
    if constexpr (FORCE) {
#pragma unroll
        for (int d = 0; d < L::D; ++d) {
            dl[d] = F[d] * inv_n;
            w2 = fmaT(dl[d], fmaT(T(2), u[d], dl[d]), w2);
        }
    }
    T inc[L::Q];
    {  // rest population: eu = 0, S - 1 = s u^2 (its increment is set from the others below)
        const T sm1 = K.s[0] * u2;
        const T geq = K.w[0] * fmaT(n, sm1, dn);
        inc[0] = c.omega * (geq - g[0]);
    }
#pragma unroll
    for (int i = 0; i < Pairs<L>::n; ++i) {
        const int q = Pairs<L>::p[i], qb = L::opp[q];
        const int k = L::cls[q];
        T eu = T(0);
        bool es = false;
#pragma unroll
        for (int d = 0; d < L::D; ++d) acc_e(eu, es, u[d], L::e[q][d]);
        const T eu2 = eu * eu;
        // S - 1 = eu (l1 + c3 u^2 + k4 eu^2) + q eu^2 + s u^2 [+ p4 eu^4 + r4 eu^2 u^2 + t4 u^4]
        const T odd = ORDER3 ? fmaT(K.k4[k], eu2, fmaT(K.c3[k], u2, K.l1[k])) : K.l1[k];
        T even = fmaT(K.q[k], eu2, K.s[k] * u2);
        if constexpr (L::O4) even = fmaT(eu2, fmaT(K.p4[k], eu2, K.r4[k] * u2), fmaT(K.t4[k] * u2, u2, even));
        const T sm1 = fmaT(eu, odd, even);
        const T sm1b = fmaT(-eu, odd, even);
        if constexpr (LOCAL) {
            const T shift = dw[k] * c.rho_ref;
            const T geq = K.w[k] * fmaT(n, sm1, dn) + shift;
            const T geqb = K.w[k] * fmaT(n, sm1b, dn) + shift;
            inc[q] = c.omega * (geq - g[q]);
            inc[qb] = c.omega * (geqb - g[qb]);
        } else {  // g_eq - g with one rounding: w X - g fused
            inc[q] = c.omega * fmaT(K.w[k], fmaT(n, sm1, dn), -g[q]);
            inc[qb] = c.omega * fmaT(K.w[k], fmaT(n, sm1b, dn), -g[qb]);
        }
        if constexpr (FORCE) {
            T b = T(0);
#pragma unroll
            for (int d = 0; d < L::D; ++d) {
                if (L::e[q][d] == 1) b += dl[d];
                if (L::e[q][d] == -1) b -= dl[d];
            }
            const T deven = fmaT(K.q[k] * b, fmaT(T(2), eu, b), K.s[k] * w2);
            T dodd = K.l1[k] * b;
            if (ORDER3) {
                const T cub = b * fmaT(T(3) * eu, eu + b, b * b);
                dodd = fmaT(K.k4[k], cub, fmaT(K.c3[k], fmaT(u2, b, w2 * (eu + b)), dodd));
            }
            const T wn = K.w[k] * n;
            inc[q] = fmaT(wn, deven + dodd, inc[q]);
            inc[qb] = fmaT(wn, deven - dodd, inc[qb]);
        }
    }
#pragma unroll
    for (int d = 0; d < L::D; ++d) {
        const int p = PlusAxis<L>::p[d];
        T acc = FORCE ? F[d] : T(0);
        bool started = FORCE;
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            if (q == p) continue;
            acc_e(acc, started, inc[q], -L::e[q][d]);
        }
        inc[p] = acc;
    }
    {
        T acc = -inc[1];
#pragma unroll
        for (int q = 2; q < L::Q; ++q) acc -= inc[q];
        inc[0] = acc;
    }
#pragma unroll
    for (int q = 0; q < L::Q; ++q) g[q] += inc[q];
}

// Weights in precision T whose zeroth and second moments are exact as real
// numbers: w_short = fl(J2/9 or the shell value), w_long = (c_s^2 - m1 w_short)/m2,
// w_rest = 1 - n1 w_short - n2 w_long.  Shell sizes n1, n2 and second moments
// along x m1, m2: d1v3 2 / 2; d2v9 4, 4 / 2, 4; d3v19 6, 12 / 2, 8.
// The 41-velocity set takes its weights rounded one by one.
template <typename T>
inline void consistent_weights(const Model &m, T *w) {
    if (m.ncls > 3) {
        for (int k = 0; k < m.ncls; ++k) w[k] = T(m.cls[k].w);
        return;
    }
    const double cs2 = m.J2 / 3.0;
    const int n1 = m.D == 1 ? 2 : m.D == 2 ? 4 : 6;
    const int n2 = m.D == 1 ? 0 : m.D == 2 ? 4 : 12;
    const int m1 = 2, m2 = m.D == 2 ? 4 : 8;
    w[1] = T(m.cls[1].w);
    if (n2 > 0) {
        w[2] = (T(cs2) - T(m1) * w[1]) / T(m2);
        w[0] = T(1.0 - n1 * double(w[1]) - n2 * double(w[2]));
    } else {
        w[2] = T(0);
        w[0] = T(1.0 - n1 * double(w[1]));
    }
}

// true when any third-order coefficient is non-zero
inline bool has_third_order(const Model &m) {
    for (int k = 0; k < m.ncls; ++k)
        if (m.cls[k].c3 != 0.0 || m.cls[k].k4 != 0.0) return true;
    return false;
}

template <typename T>
inline Coef<T> make_coef(const Model &m, double tau, double rho_ref) {
    Coef<T> c{};
    consistent_weights<T>(m, c.w);
    for (int k = 0; k < kMaxClasses; ++k) {
        c.l1[k] = T(m.cls[k].l1);
        c.q[k] = T(m.cls[k].q);
        c.s[k] = T(m.cls[k].s);
        c.c3[k] = T(m.cls[k].c3);
        c.k4[k] = T(m.cls[k].k4);
        c.p4[k] = T(m.cls[k].p4);
        c.r4[k] = T(m.cls[k].r4);
        c.t4[k] = T(m.cls[k].t4);
    }
    c.omega = T(1.0 / tau);
    c.rho_ref = T(rho_ref);
    if (m.local) {
        const SommerfeldJ sj = sommerfeld_j(m.D);
        const double r2 = m.r0 * m.r0;
        double Br[4];
        for (int N = 0; N < 4; ++N) Br[N] = 1.0 + sj.b[N] * r2;
        c.loc.r2 = T(r2);
        for (int N = 0; N < 4; ++N) {
            c.loc.b[N] = T(sj.b[N]);
            c.loc.Br[N] = T(Br[N]);
        }
        c.loc.J2z = T(sj.J2z);
        c.loc.J4z = T(sj.J4z);
        c.loc.rhs = T(1.0 + sj.b[0] * r2);
        c.loc.inv_rho = T(1.0 / rho_ref);
        c.loc.J2r = T(m.J2);
        // B1^2 B0r B2r - B1r^2 B0 B2 with B = Br + b dt, divided by dt
        c.loc.P1 = T(2.0 * Br[1] * sj.b[1] * Br[0] * Br[2] - Br[1] * Br[1] * (sj.b[0] * Br[2] + sj.b[2] * Br[0]));
        c.loc.P2 = T(sj.b[1] * sj.b[1] * Br[0] * Br[2] - Br[1] * Br[1] * sj.b[0] * sj.b[2]);
        c.loc.inv_br02 = T(1.0 / (Br[0] * Br[2]));
    }
    return c;
}

}  // namespace lbm
