/*
 * Plain FP64 CPU lattice Boltzmann oracle for the generalized-polynomial method
 * of Coelho, Ilha and Doria (arXiv:1510.07328).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or constant with the HIP library: the model description (velocities,
 * weights, polynomial coefficients) is handed in by oracle/theory.py.
 *
 * Order 4 uses P_4 (eq. H4) with delta_{ijkl} read as the isotropic four-index
 * delta (delta_ij delta_kl + delta_ik delta_jl + delta_il delta_jk) and A_4
 * (eq. A4) with its sixth pair term read as u_i2 u_i4 delta_i1i3.
 *
 * What it computes, step by step, in the paper's order:
 *   1. moments of the populations, I_0 = n = sum_a f_a and
 *      u0 = sum_a f_a e_a / n  (section "The Gaussian quadrature", moment update
 *      after the lattice BGK equation; the printed "I_0 = sum f e" is read as
 *      sum_a f_a);
 *   2. the discrete equilibrium by the tensor expansion of eq. expansao0,
 *      f_eq,a = n w_a sum_{N<=order} (1/N!) sum_{i1..iN} A_{i1..iN}(u) P_{i1..iN}(xi_a)
 *      with u = c_0 u0 and xi_a = c_0 e_a (eqs. H0-H3 and A0-A3);
 *   3. BGK relaxation f*_a = f_a - (f_a - f_eq,a) / tau (lattice BGK equation);
 *   4. streaming f_a(x + e_a, t + 1) = f*_a(x, t); periodic axes wrap, and on a
 *      bounce-back axis a link leaving the box returns to its cell reversed,
 *      f_abar(x, t + 1) = f*_a(x, t) (halfway bounce-back; the paper names
 *      bounce-back for obstacles without fixing its form).
 *
 * orc_run_porous adds the two ingredients of the paper's porous-media runs
 * (section "Numerical simulations for electrons in metals", flow through rigid
 * obstacles under a constant external force):
 *   - solid cells (a mask): they take no part in the step; a link that would
 *     stream into a solid cell returns to its cell reversed (halfway
 *     bounce-back, as at a wall);
 *   - a constant body force F per cell (force density, lattice units).  The
 *     paper does not say how the force enters; here by the exact difference of
 *     equilibria: after relaxation each fluid cell receives
 *     f_eq,a(n, u0 + F / n) - f_eq,a(n, u0), which adds F to its momentum and
 *     nothing to its mass.  The physical velocity is then (j + F / 2) / n.
 *
 * Build with -ffp-contract=off: every sum runs in a fixed order (populations
 * ascending, tensor indices lexicographic, cells x fastest).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

#define ORC_MAXT 40 /* 1 + 3 + 9 + 27 tuples for D = 3, order 3; 1 + 2 + 4 + 8 + 16 for D = 2, order 4 */

/* Tensor index tuples (i1..iN) for N = 0..order, lexicographic. */
typedef struct {
    int T;
    int N[ORC_MAXT];
    int idx[ORC_MAXT][4];
    double P[ORC_MAXT][ORC_MAXQ]; /* P_t(xi_a) */
} orc_tensors;

static double kd(int i, int j) { return i == j ? 1.0 : 0.0; }

/* a_i a_j delta_kl over the six ways to split (i, j, k, l) into two pairs */
static double sym6(const double *a, const int *id)
{
    const int i = id[0], j = id[1], k = id[2], l = id[3];
    return a[i] * a[j] * kd(k, l) + a[i] * a[k] * kd(j, l) + a[i] * a[l] * kd(j, k)
         + a[j] * a[k] * kd(i, l) + a[j] * a[l] * kd(i, k) + a[k] * a[l] * kd(i, j);
}

static double delta4(const int *id)
{
    return kd(id[0], id[1]) * kd(id[2], id[3]) + kd(id[0], id[2]) * kd(id[1], id[3])
         + kd(id[0], id[3]) * kd(id[1], id[2]);
}

/* eqs. H0-H3 */
static double poly_P(const orc_model *m, int N, const int *id, const double *xi)
{
    double x2 = 0.0;
    for (int d = 0; d < m->D; ++d) x2 += xi[d] * xi[d];
    switch (N) {
    case 0: return m->c[0];
    case 1: return m->c[1] * xi[id[0]];
    case 2:
        return m->c[2] * xi[id[0]] * xi[id[1]] + (m->cb[2] * x2 + m->cp[2]) * kd(id[0], id[1]);
    case 3: {
        double sym = xi[id[0]] * kd(id[1], id[2]) + xi[id[1]] * kd(id[0], id[2])
                   + xi[id[2]] * kd(id[0], id[1]);
        return m->c[3] * xi[id[0]] * xi[id[1]] * xi[id[2]] + (m->cb[3] * x2 + m->cp[3]) * sym;
    }
    case 4:
        return m->c[4] * xi[id[0]] * xi[id[1]] * xi[id[2]] * xi[id[3]] + (m->cb[4] * x2 + m->cp[4]) * sym6(xi, id)
             + (m->db4 * x2 * x2 + m->dp4 * x2 + m->d4) * delta4(id);
    }
    return 0.0;
}

/* eqs. A0-A3 */
static double coef_A(const orc_model *m, int N, const int *id, const double *u)
{
    double u2 = 0.0;
    for (int d = 0; d < m->D; ++d) u2 += u[d] * u[d];
    switch (N) {
    case 0: return m->I0 * m->c[0];
    case 1: return m->I0 * m->c[1] * u[id[0]];
    case 2: return m->I0 * (m->c[2] * u[id[0]] * u[id[1]] + m->cb[2] * u2 * kd(id[0], id[1]));
    case 3: {
        double sym = u[id[0]] * kd(id[1], id[2]) + u[id[1]] * kd(id[0], id[2])
                   + u[id[2]] * kd(id[0], id[1]);
        return m->I0 * (m->c[3] * u[id[0]] * u[id[1]] * u[id[2]]
                        + (m->cp[3] * (1.0 - m->J2) + m->cb[3] * u2) * sym);
    }
    case 4: {
        const double iso = (2.0 * m->I2 / m->I0 * (m->cb[4] + (m->D + 2) * m->db4) + m->dp4) * u2 + m->db4 * u2 * u2;
        return m->I0 * (m->c[4] * u[id[0]] * u[id[1]] * u[id[2]] * u[id[3]]
                        + ((1.0 - m->J2 * m->J4) * m->cp[4] + m->cb[4] * u2) * sym6(u, id) + iso * delta4(id));
    }
    }
    return 0.0;
}

static void build_tensors(const orc_model *m, orc_tensors *t)
{
    t->T = 0;
    for (int N = 0; N <= m->order; ++N) {
        int count = 1;
        for (int k = 0; k < N; ++k) count *= m->D;
        for (int c = 0; c < count; ++c) {
            int rem = c, id[4] = {0, 0, 0, 0};
            for (int k = N - 1; k >= 0; --k) { id[k] = rem % m->D; rem /= m->D; }
            t->N[t->T] = N;
            memcpy(t->idx[t->T], id, sizeof id);
            for (int a = 0; a < m->Q; ++a) {
                double xi[3];
                for (int d = 0; d < m->D; ++d) xi[d] = m->cvel * m->e[a][d];
                t->P[t->T][a] = poly_P(m, N, id, xi);
            }
            t->T++;
        }
    }
}

static const double inv_fact[5] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0};

/* f_eq,a = n w_a S_a by the tensor expansion */
static void feq_cell(const orc_model *m, const orc_tensors *t, double n, const double *u0, double *feq)
{
    double u[3] = {0, 0, 0}, Av[ORC_MAXT];
    for (int d = 0; d < m->D; ++d) u[d] = m->cvel * u0[d];
    for (int k = 0; k < t->T; ++k) Av[k] = coef_A(m, t->N[k], t->idx[k], u);
    for (int a = 0; a < m->Q; ++a) {
        double S = 0.0;
        int k = 0;
        for (int N = 0; N <= m->order; ++N) {
            double acc = 0.0;
            for (; k < t->T && t->N[k] == N; ++k) acc += Av[k] * t->P[k][a];
            S += inv_fact[N] * acc;
        }
        feq[a] = n * m->w_hat[a] * S;
    }
}

static int check_model(const orc_model *m)
{
    if (m->D < 1 || m->D > 3 || m->Q < 1 || m->Q > ORC_MAXQ) return -1;
    if (m->order < 0 || m->order > 4) return -1;
    int tcount = 0, p = 1;
    for (int N = 0; N <= m->order; ++N) { tcount += p; p *= m->D; }
    if (tcount > ORC_MAXT) return -1;
    if (m->nx < 1 || m->ny < 1 || m->nz < 1) return -1;
    if (!(m->tau > 0.0)) return -1;
    return 0;
}

int orc_feq(const orc_model *m, double n, const double *u0, double *feq)
{
    if (check_model(m)) return -1;
    orc_tensors t;
    build_tensors(m, &t);
    feq_cell(m, &t, n, u0, feq);
    return 0;
}

/* f[a][z][y][x] = f_eq(n0[cell], u0[d][cell]) */
int orc_init(const orc_model *m, const double *n0, const double *u0, double *f)
{
    if (check_model(m)) return -1;
    orc_tensors t;
    build_tensors(m, &t);
    const long cells = (long)m->nx * m->ny * m->nz;
    for (long c = 0; c < cells; ++c) {
        double u[3] = {0, 0, 0}, feq[ORC_MAXQ];
        for (int d = 0; d < m->D; ++d) u[d] = u0[(long)d * cells + c];
        feq_cell(m, &t, n0[c], u, feq);
        for (int a = 0; a < m->Q; ++a) f[(long)a * cells + c] = feq[a];
    }
    return 0;
}

int orc_moments(const orc_model *m, const double *f, double *n, double *u0)
{
    if (check_model(m)) return -1;
    const long cells = (long)m->nx * m->ny * m->nz;
    for (long c = 0; c < cells; ++c) {
        double rho = 0.0, j[3] = {0, 0, 0};
        for (int a = 0; a < m->Q; ++a) {
            double fa = f[(long)a * cells + c];
            rho += fa;
            for (int d = 0; d < m->D; ++d) j[d] += fa * m->e[a][d];
        }
        n[c] = rho;
        for (int d = 0; d < m->D; ++d) u0[(long)d * cells + c] = j[d] / rho;
    }
    return 0;
}

/* One collide-and-stream step from f into g (push form). */
static void step(const orc_model *m, const orc_tensors *t, const double *f, double *g)
{
    const int nx = m->nx, ny = m->ny, nz = m->nz, D = m->D;
    const long cells = (long)nx * ny * nz;
    const int dims[3] = {nx, ny, nz};
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long c = ((long)z * ny + y) * nx + x;
                double fa[ORC_MAXQ], feq[ORC_MAXQ], rho = 0.0, j[3] = {0, 0, 0}, u0[3] = {0, 0, 0};
                for (int a = 0; a < m->Q; ++a) {
                    fa[a] = f[(long)a * cells + c];
                    rho += fa[a];
                    for (int d = 0; d < D; ++d) j[d] += fa[a] * m->e[a][d];
                }
                for (int d = 0; d < D; ++d) u0[d] = j[d] / rho;
                feq_cell(m, t, rho, u0, feq);
                const int pos[3] = {x, y, z};
                for (int a = 0; a < m->Q; ++a) {
                    const double fs = fa[a] - (fa[a] - feq[a]) / m->tau;
                    int tgt[3] = {x, y, z}, bounced = 0;
                    for (int d = 0; d < 3; ++d) {
                        int s = pos[d] + (d < D ? m->e[a][d] : 0);
                        if (s < 0 || s >= dims[d]) {
                            if (m->bc[d] == 1) bounced = 1;
                            else s = (s + dims[d]) % dims[d];
                        }
                        tgt[d] = s;
                    }
                    if (bounced)
                        g[(long)m->opp[a] * cells + c] = fs;
                    else
                        g[(long)a * cells + ((long)tgt[2] * ny + tgt[1]) * nx + tgt[0]] = fs;
                }
            }
}

/* One step with solid cells and a body force (push form).  Solid cells copy
 * their populations through unchanged. */
static void step_porous(const orc_model *m, const orc_tensors *t, const unsigned char *solid, const double *force,
                        const double *f, double *g)
{
    const int nx = m->nx, ny = m->ny, nz = m->nz, D = m->D;
    const long cells = (long)nx * ny * nz;
    const int dims[3] = {nx, ny, nz};
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long c = ((long)z * ny + y) * nx + x;
                if (solid && solid[c]) {
                    for (int a = 0; a < m->Q; ++a) g[(long)a * cells + c] = f[(long)a * cells + c];
                    continue;
                }
                double fa[ORC_MAXQ], feq[ORC_MAXQ], feqF[ORC_MAXQ];
                double rho = 0.0, j[3] = {0, 0, 0}, u0[3] = {0, 0, 0}, uF[3] = {0, 0, 0};
                for (int a = 0; a < m->Q; ++a) {
                    fa[a] = f[(long)a * cells + c];
                    rho += fa[a];
                    for (int d = 0; d < D; ++d) j[d] += fa[a] * m->e[a][d];
                }
                for (int d = 0; d < D; ++d) {
                    u0[d] = j[d] / rho;
                    uF[d] = u0[d] + force[d] / rho;
                }
                feq_cell(m, t, rho, u0, feq);
                feq_cell(m, t, rho, uF, feqF);
                const int pos[3] = {x, y, z};
                for (int a = 0; a < m->Q; ++a) {
                    const double fs = fa[a] - (fa[a] - feq[a]) / m->tau + (feqF[a] - feq[a]);
                    int tgt[3] = {x, y, z}, bounced = 0;
                    for (int d = 0; d < 3; ++d) {
                        int s = pos[d] + (d < D ? m->e[a][d] : 0);
                        if (s < 0 || s >= dims[d]) {
                            if (m->bc[d] == 1) bounced = 1;
                            else s = (s + dims[d]) % dims[d];
                        }
                        tgt[d] = s;
                    }
                    const long tc = ((long)tgt[2] * ny + tgt[1]) * nx + tgt[0];
                    if (!bounced && solid && solid[tc]) bounced = 1;
                    if (bounced)
                        g[(long)m->opp[a] * cells + c] = fs;
                    else
                        g[(long)a * cells + tc] = fs;
                }
            }
}

/* Advance f by `steps` steps with a solid mask (cells, nonzero = solid; may be
 * NULL) and a body force force[3] (components beyond D ignored). */
int orc_run_porous(const orc_model *m, const unsigned char *solid, const double *force, double *f, long steps)
{
    if (check_model(m) || steps < 0 || !force) return -1;
    orc_tensors t;
    build_tensors(m, &t);
    const long cells = (long)m->nx * m->ny * m->nz;
    double *g = (double *)malloc(sizeof(double) * cells * m->Q);
    if (!g) return -2;
    for (long s = 0; s < steps; ++s) {
        step_porous(m, &t, solid, force, f, g);
        memcpy(f, g, sizeof(double) * cells * m->Q);
    }
    free(g);
    return 0;
}

/* Advance f (layout [Q][nz][ny][nx]) by `steps` steps in place. */
int orc_run(const orc_model *m, double *f, long steps)
{
    if (check_model(m) || steps < 0) return -1;
    orc_tensors t;
    build_tensors(m, &t);
    const long cells = (long)m->nx * m->ny * m->nz;
    double *g = (double *)malloc(sizeof(double) * cells * m->Q);
    if (!g) return -2;
    for (long s = 0; s < steps; ++s) {
        step(m, &t, f, g);
        memcpy(f, g, sizeof(double) * cells * m->Q);
    }
    free(g);
    return 0;
}
