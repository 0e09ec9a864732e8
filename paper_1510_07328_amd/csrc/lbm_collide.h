// The fused collision shared by every step kernel (plain field steps and the
// batched tube sweep): moments, equilibrium from the per-class polynomial,
// BGK relaxation.  Included by the kernel sources only.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"

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
template <class L, typename T, bool ORDER3 = true, bool FORCE = false>
__device__ __forceinline__ void collide(T (&g)[L::Q], const Coef<T> &c, const T *F = nullptr) {
    T dn = T(0), j[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        dn += g[q];
#pragma unroll
        for (int d = 0; d < L::D; ++d) {
            if (L::e[q][d] == 1) j[d] += g[q];
            if (L::e[q][d] == -1) j[d] -= g[q];
        }
    }
    const T n = c.rho_ref + dn;
    const T inv_n = T(1) / n;
    T u[3] = {T(0), T(0), T(0)};
    T u2 = T(0);
#pragma unroll
    for (int d = 0; d < L::D; ++d) {
        u[d] = j[d] * inv_n;
        u2 = fmaT(u[d], u[d], u2);
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
        const T sm1 = c.s[0] * u2;
        const T geq = c.w[0] * fmaT(n, sm1, dn);
        inc[0] = c.omega * (geq - g[0]);
    }
#pragma unroll
    for (int i = 0; i < Pairs<L>::n; ++i) {
        const int q = Pairs<L>::p[i], qb = L::opp[q];
        const int k = L::cls[q];
        T eu = T(0);
#pragma unroll
        for (int d = 0; d < L::D; ++d) {
            if (L::e[q][d] == 1) eu += u[d];
            if (L::e[q][d] == -1) eu -= u[d];
        }
        const T eu2 = eu * eu;
        // S - 1 = eu (l1 + c3 u^2 + k4 eu^2) + q eu^2 + s u^2
        const T odd = ORDER3 ? fmaT(c.k4[k], eu2, fmaT(c.c3[k], u2, c.l1[k])) : c.l1[k];
        const T even = fmaT(c.q[k], eu2, c.s[k] * u2);
        const T sm1 = fmaT(eu, odd, even);
        const T sm1b = fmaT(-eu, odd, even);
        const T geq = c.w[k] * fmaT(n, sm1, dn);
        const T geqb = c.w[k] * fmaT(n, sm1b, dn);
        inc[q] = c.omega * (geq - g[q]);
        inc[qb] = c.omega * (geqb - g[qb]);
        if constexpr (FORCE) {
            T b = T(0);
#pragma unroll
            for (int d = 0; d < L::D; ++d) {
                if (L::e[q][d] == 1) b += dl[d];
                if (L::e[q][d] == -1) b -= dl[d];
            }
            const T deven = fmaT(c.q[k] * b, fmaT(T(2), eu, b), c.s[k] * w2);
            T dodd = c.l1[k] * b;
            if (ORDER3) {
                const T cub = b * fmaT(T(3) * eu, eu + b, b * b);
                dodd = fmaT(c.k4[k], cub, fmaT(c.c3[k], fmaT(u2, b, w2 * (eu + b)), dodd));
            }
            const T wn = c.w[k] * n;
            inc[q] = fmaT(wn, deven + dodd, inc[q]);
            inc[qb] = fmaT(wn, deven - dodd, inc[qb]);
        }
    }
#pragma unroll
    for (int d = 0; d < L::D; ++d) {
        const int p = PlusAxis<L>::p[d];
        T acc = FORCE ? F[d] : T(0);
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            if (q == p) continue;
            if (L::e[q][d] == 1) acc -= inc[q];
            if (L::e[q][d] == -1) acc += inc[q];
        }
        inc[p] = acc;
    }
    {
        T acc = T(0);
#pragma unroll
        for (int q = 1; q < L::Q; ++q) acc -= inc[q];
        inc[0] = acc;
    }
#pragma unroll
    for (int q = 0; q < L::Q; ++q) g[q] += inc[q];
}

// Weights in precision T whose zeroth and second moments are exact as real
// numbers: w_short = fl(J2/9 or the shell value), w_long = (c_s^2 - m1 w_short)/m2,
// w_rest = 1 - n1 w_short - n2 w_long.  Shell sizes n1, n2 and second moments
// along x m1, m2: d1v3 2 / 2; d2v9 4, 4 / 2, 4; d3v19 6, 12 / 2, 8.
template <typename T>
inline void consistent_weights(const Model &m, T (&w)[3]) {
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
    for (int k = 0; k < 3; ++k)
        if (m.cls[k].c3 != 0.0 || m.cls[k].k4 != 0.0) return true;
    return false;
}

template <typename T>
inline Coef<T> make_coef(const Model &m, double tau, double rho_ref) {
    Coef<T> c{};
    consistent_weights<T>(m, c.w);
    for (int k = 0; k < 3; ++k) {
        c.l1[k] = T(m.cls[k].l1);
        c.q[k] = T(m.cls[k].q);
        c.s[k] = T(m.cls[k].s);
        c.c3[k] = T(m.cls[k].c3);
        c.k4[k] = T(m.cls[k].k4);
    }
    c.omega = T(1.0 / tau);
    c.rho_ref = T(rho_ref);
    return c;
}

}  // namespace lbm
