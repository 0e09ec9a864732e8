/*
 * The lbm_* call surface over the FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  It lets the tests exercise the library's calling
 * conventions -- argument checks, error codes, checkpoint and restore, fault
 * injection through lbm_set_state -- on a machine without a GPU, against the
 * plain float64 iteration of lbm_oracle.c.  It shares no code or header with
 * the HIP library: the configuration record below is laid out like the
 * library's (a test compares the layouts field by field), and the lattice
 * model is built here from the paper's formulas.
 *
 * The model, from the configuration (section "Generalized polynomials in D
 * dimensions" and the paragraph after eq. H4; section "The Gaussian
 * quadrature"):
 *   - moments of the weight I_2N: zero-temperature Fermi-Dirac,
 *     I_2N = (2 pi)^(D/2) mu^(N + D/2) / Gamma(N + D/2 + 1) at mu = 1 (eq.
 *     sommerfeld at theta = 0); Maxwell-Boltzmann, I_2N = I_0 theta^N with
 *     theta = 1/3 (c_0 = 1); or given J_2, J_4, with I_0 = I_2 = 1,
 *     I_4 = I_2^2 / (J_2 I_0), I_6 = I_4^2 / (J_4 I_2);
 *   - J_L = I_L^2 / (I_(L+2) I_(L-2)), Delta_L^2 = 2 / [(D + L) - J_L (D + L - 2)]
 *     (positive root);
 *   - c_K = I_2K^(-1/2); c'_K = -c_K (I_(2K-2) / I_(2K-4)) Delta_(2K-2) and
 *     cbar_K = c_K (Delta_(2K-2) - 1) / (D + 2K - 4) for K = 2, 3;
 *   - c_0 = sqrt(3 I_4 / I_2) and the normalised weights of the d1v3 and d2v9
 *     sets, (1 - J_2/3, J_2/6) and (1 - 5 J_2/9, J_2/9, J_2/36), and of the
 *     19-velocity set that solves the same moment conditions in D = 3,
 *     (1 - 2 J_2/3, J_2/18, J_2/36).
 *
 * Differences from the GPU library, all by design of a CPU stand-in: every
 * pointer is host memory (the "workspace" holds the float64 populations, the
 * stream is ignored), every call is synchronous, storage is float64 only
 * (LBM_FP32_DEV is LBM_ERR_UNSUPPORTED), the weight families are the three
 * above, and there are no obstacles, body force or per-cell weights.  The
 * streaming scheme field is accepted and ignored (the oracle streams by push;
 * both schemes give the same populations).  Populations are in the oracle's
 * velocity order (lbm_velocities reports it).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

/* status codes, as the library numbers them */
enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_UNSUPPORTED = -2, ORC_ERR_NUMERIC = -4, ORC_ERR_STATE = -5 };
/* configuration values, as the library numbers them */
enum { ORC_D1V3 = 1, ORC_D2V9 = 2, ORC_D3V19 = 3 };
enum { ORC_W_MB = 0, ORC_W_FD_T0 = 1, ORC_W_CUSTOM = 2 };
enum { ORC_FP32_DEV = 0, ORC_FP64 = 1 };

typedef struct {
    int lattice;
    int nx, ny, nz;
    int bc[3];
    int weight;
    double J2, J4;
    int order;
    double tau;
    int precision;
    double rho_ref;
    int scheme;
    int block;
    int graph_steps;
    int obstacles;
    double force[3];
    double fugacity;
    double theta_over_mu;
} orc_api_config;

typedef struct {
    orc_model m;
    double *f;      /* [Q][cells] full populations, in the caller's workspace */
    long cells;
    double rho_ref;
    int64_t steps;
} orc_api_ctx;

static _Thread_local char g_err[256];

static int fail(int status, const char *msg)
{
    snprintf(g_err, sizeof g_err, "%s", msg);
    return status;
}

const char *lbm_last_error(void) { return g_err; }

/* layout of the configuration record, for the test that compares it with the library's */
size_t orc_api_config_size(void) { return sizeof(orc_api_config); }
size_t orc_api_config_offset(int field)
{
    switch (field) {
    case 0: return offsetof(orc_api_config, lattice);
    case 1: return offsetof(orc_api_config, bc);
    case 2: return offsetof(orc_api_config, J2);
    case 3: return offsetof(orc_api_config, tau);
    case 4: return offsetof(orc_api_config, rho_ref);
    case 5: return offsetof(orc_api_config, force);
    case 6: return offsetof(orc_api_config, theta_over_mu);
    }
    return (size_t)-1;
}

static void set_velocities(orc_model *m, int lattice)
{
    static const int d1[3][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}};
    static const int d2[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                                 {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    if (lattice == ORC_D1V3) {
        m->D = 1;
        m->Q = 3;
        memcpy(m->e, d1, sizeof d1);
    } else if (lattice == ORC_D2V9) {
        m->D = 2;
        m->Q = 9;
        memcpy(m->e, d2, sizeof d2);
    } else {
        /* rest; the six faces +-x, +-y, +-z; the twelve edges in the xy, xz, yz planes */
        int q = 0;
        m->D = 3;
        memset(m->e[q++], 0, sizeof m->e[0]);
        for (int a = 0; a < 3; ++a)
            for (int s = 1; s >= -1; s -= 2) {
                memset(m->e[q], 0, sizeof m->e[q]);
                m->e[q++][a] = s;
            }
        static const int planes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int p = 0; p < 3; ++p)
            for (int sa = 1; sa >= -1; sa -= 2)
                for (int sb = 1; sb >= -1; sb -= 2) {
                    memset(m->e[q], 0, sizeof m->e[q]);
                    m->e[q][planes[p][0]] = sa;
                    m->e[q][planes[p][1]] = sb;
                    q++;
                }
        m->Q = q;
    }
    for (int a = 0; a < m->Q; ++a)
        for (int b = 0; b < m->Q; ++b)
            if (m->e[b][0] == -m->e[a][0] && m->e[b][1] == -m->e[a][1] && m->e[b][2] == -m->e[a][2]) m->opp[a] = b;
}

/* The lattice model of a configuration (see the file comment). */
static int build_model(const orc_api_config *cfg, orc_model *m)
{
    memset(m, 0, sizeof *m);
    if (cfg->lattice != ORC_D1V3 && cfg->lattice != ORC_D2V9 && cfg->lattice != ORC_D3V19)
        return fail(ORC_ERR_UNSUPPORTED, "the oracle surface runs d1v3, d2v9 and d3v19");
    set_velocities(m, cfg->lattice);
    const int D = m->D;
    double I[4]; /* I_0, I_2, I_4, I_6 */
    if (cfg->weight == ORC_W_FD_T0) {
        for (int N = 0; N < 4; ++N) I[N] = pow(2.0 * acos(-1.0), D / 2.0) / tgamma(N + D / 2.0 + 1.0);
    } else if (cfg->weight == ORC_W_MB) {
        const double theta = 1.0 / 3.0;
        for (int N = 0; N < 4; ++N) I[N] = pow(theta, N);
    } else if (cfg->weight == ORC_W_CUSTOM) {
        if (!(cfg->J2 > 0.0) || !(cfg->J4 > 0.0)) return fail(ORC_ERR_ARG, "custom weight needs J2, J4 > 0");
        I[0] = 1.0;
        I[1] = 1.0;
        I[2] = I[1] * I[1] / (cfg->J2 * I[0]);
        I[3] = I[2] * I[2] / (cfg->J4 * I[1]);
    } else {
        return fail(ORC_ERR_UNSUPPORTED, "the oracle surface takes the MB, FD_T0 and custom weights");
    }
    const double J2 = I[1] * I[1] / (I[2] * I[0]);
    const double J4 = I[2] * I[2] / (I[3] * I[1]);
    const double d2sq = 2.0 / ((D + 2) - J2 * D);
    const double d4sq = 2.0 / ((D + 4) - J4 * (D + 2));
    if (!(d2sq > 0.0) || !(d4sq > 0.0)) return fail(ORC_ERR_ARG, "Delta_L^2 must be positive");
    const double d2 = sqrt(d2sq), d4 = sqrt(d4sq);
    for (int K = 0; K < 4; ++K) m->c[K] = 1.0 / sqrt(I[K]);
    m->cp[2] = -m->c[2] * (I[1] / I[0]) * d2;
    m->cb[2] = m->c[2] * (d2 - 1.0) / D;
    m->cp[3] = -m->c[3] * (I[2] / I[1]) * d4;
    m->cb[3] = m->c[3] * (d4 - 1.0) / (D + 2);
    m->cvel = sqrt(3.0 * I[2] / I[1]);
    m->I0 = I[0];
    m->J2 = J2;
    m->J4 = J4;
    m->I2 = I[1];
    double w0, w1, w2;
    if (D == 1) {
        w0 = 1.0 - J2 / 3.0, w1 = J2 / 6.0, w2 = 0.0;
    } else if (D == 2) {
        w0 = 1.0 - 5.0 * J2 / 9.0, w1 = J2 / 9.0, w2 = J2 / 36.0;
    } else {
        w0 = 1.0 - 2.0 * J2 / 3.0, w1 = J2 / 18.0, w2 = J2 / 36.0;
    }
    for (int a = 0; a < m->Q; ++a) {
        const int e2 = m->e[a][0] * m->e[a][0] + m->e[a][1] * m->e[a][1] + m->e[a][2] * m->e[a][2];
        m->w_hat[a] = e2 == 0 ? w0 : e2 == 1 ? w1 : w2;
    }
    m->order = cfg->order;
    m->nx = cfg->nx;
    m->ny = cfg->ny;
    m->nz = cfg->nz;
    for (int d = 0; d < 3; ++d) m->bc[d] = cfg->bc[d];
    m->tau = cfg->tau;
    return ORC_OK;
}

static int check_config(const orc_api_config *cfg, orc_model *m)
{
    if (!cfg) return fail(ORC_ERR_ARG, "null config");
    int s = build_model(cfg, m);
    if (s != ORC_OK) return s;
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return fail(ORC_ERR_ARG, "box sizes must be >= 1");
    if (m->D < 2 && cfg->ny != 1) return fail(ORC_ERR_ARG, "d1v3 needs ny = 1");
    if (m->D < 3 && cfg->nz != 1) return fail(ORC_ERR_ARG, "2D lattices need nz = 1");
    for (int d = 0; d < 3; ++d)
        if (cfg->bc[d] != 0 && cfg->bc[d] != 1) return fail(ORC_ERR_ARG, "bad bc");
    if (cfg->order != 2 && cfg->order != 3) return fail(ORC_ERR_ARG, "order must be 2 or 3");
    if (!(cfg->tau > 0.5)) return fail(ORC_ERR_ARG, "tau must be > 1/2");
    if (cfg->precision != ORC_FP32_DEV && cfg->precision != ORC_FP64) return fail(ORC_ERR_ARG, "bad precision");
    if (cfg->precision != ORC_FP64) return fail(ORC_ERR_UNSUPPORTED, "the oracle stores float64 populations only");
    if (cfg->scheme != 0 && cfg->scheme != 1) return fail(ORC_ERR_ARG, "bad scheme");
    if (cfg->obstacles || cfg->force[0] != 0.0 || cfg->force[1] != 0.0 || cfg->force[2] != 0.0)
        return fail(ORC_ERR_UNSUPPORTED, "the oracle surface has no obstacles or body force");
    return ORC_OK;
}

/* (the exported calls use static helpers for each other's work, so that no call
 * inside this library can bind to a same-named symbol of another library) */
static int workspace_bytes(const orc_api_config *cfg, size_t *bytes)
{
    orc_model m;
    if (!bytes) return fail(ORC_ERR_ARG, "null argument");
    int s = check_config(cfg, &m);
    if (s != ORC_OK) return s;
    *bytes = sizeof(double) * (size_t)m.Q * (size_t)cfg->nx * cfg->ny * cfg->nz;
    return ORC_OK;
}

int lbm_workspace_bytes(const orc_api_config *cfg, size_t *bytes) { return workspace_bytes(cfg, bytes); }

int lbm_init(const orc_api_config *cfg, void *workspace, size_t bytes, void *stream, const double *n0,
             const double *u0, orc_api_ctx **out)
{
    (void)stream;
    if (!out) return fail(ORC_ERR_ARG, "null argument");
    *out = NULL;
    if (!workspace || !n0 || !u0) return fail(ORC_ERR_ARG, "null argument");
    size_t need = 0;
    int s = workspace_bytes(cfg, &need);
    if (s != ORC_OK) return s;
    if (bytes < need) return fail(ORC_ERR_ARG, "workspace smaller than lbm_workspace_bytes()");
    if ((uintptr_t)workspace % sizeof(double)) return fail(ORC_ERR_ARG, "workspace must be 8-byte aligned");
    orc_api_ctx *c = (orc_api_ctx *)calloc(1, sizeof *c);
    if (!c) return fail(ORC_ERR_ARG, "out of host memory");
    check_config(cfg, &c->m);
    c->f = (double *)workspace;
    c->cells = (long)cfg->nx * cfg->ny * cfg->nz;
    c->rho_ref = cfg->rho_ref > 0.0 ? cfg->rho_ref : 1.0;
    if (orc_init(&c->m, n0, u0, c->f)) {
        free(c);
        return fail(ORC_ERR_ARG, "the oracle rejected the model");
    }
    *out = c;
    return ORC_OK;
}

int lbm_step(orc_api_ctx *c, int64_t nsteps)
{
    if (!c) return fail(ORC_ERR_ARG, "null context");
    if (nsteps < 0) return fail(ORC_ERR_ARG, "nsteps must be >= 0");
    if (orc_run(&c->m, c->f, (long)nsteps)) return fail(ORC_ERR_ARG, "the oracle rejected the run");
    c->steps += nsteps;
    return ORC_OK;
}

static int moments(orc_api_ctx *c, double *n_host, double *u_host)
{
    if (!c || !n_host || !u_host) return fail(ORC_ERR_ARG, "null argument");
    orc_moments(&c->m, c->f, n_host, u_host);
    return ORC_OK;
}

int lbm_moments(orc_api_ctx *c, double *n_host, double *u_host) { return moments(c, n_host, u_host); }

/* no device here: the same host moments */
int lbm_moments_device(orc_api_ctx *c, double *n, double *u) { return moments(c, n, u); }

int lbm_totals(orc_api_ctx *c, double *out_host)
{
    if (!c || !out_host) return fail(ORC_ERR_ARG, "null argument");
    const orc_model *m = &c->m;
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    long bad = 0;
    for (long x = 0; x < c->cells; ++x) {
        double n = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < m->Q; ++a) {
            const double fa = c->f[(long)a * c->cells + x];
            n += fa;
            for (int d = 0; d < m->D; ++d) j[d] += m->e[a][d] * fa;
        }
        if (!(n > 0.0) || !isfinite(n)) bad++;
        tot[0] += n;
        for (int d = 0; d < m->D; ++d) tot[1 + d] += j[d];
    }
    for (int d = 0; d <= m->D; ++d) out_host[d] = tot[d];
    for (int d = 0; d <= m->D; ++d)
        if (!isfinite(tot[d])) return fail(ORC_ERR_NUMERIC, "non-finite total");
    if (bad) return fail(ORC_ERR_NUMERIC, "cells with non-positive or non-finite density");
    return ORC_OK;
}

/* populations as deviations g = f - w rho_ref at their natural slots, float64 */
int lbm_get_state(orc_api_ctx *c, void *host, size_t bytes)
{
    if (!c || !host) return fail(ORC_ERR_ARG, "null argument");
    if (bytes != sizeof(double) * (size_t)c->m.Q * (size_t)c->cells) return fail(ORC_ERR_ARG, "state size mismatch");
    double *g = (double *)host;
    for (int a = 0; a < c->m.Q; ++a)
        for (long x = 0; x < c->cells; ++x)
            g[(long)a * c->cells + x] = c->f[(long)a * c->cells + x] - c->m.w_hat[a] * c->rho_ref;
    return ORC_OK;
}

int lbm_set_state(orc_api_ctx *c, const void *host, size_t bytes)
{
    if (!c || !host) return fail(ORC_ERR_ARG, "null argument");
    if (bytes != sizeof(double) * (size_t)c->m.Q * (size_t)c->cells) return fail(ORC_ERR_ARG, "state size mismatch");
    const double *g = (const double *)host;
    for (int a = 0; a < c->m.Q; ++a)
        for (long x = 0; x < c->cells; ++x)
            c->f[(long)a * c->cells + x] = g[(long)a * c->cells + x] + c->m.w_hat[a] * c->rho_ref;
    return ORC_OK;
}

int lbm_steps_done(orc_api_ctx *c, int64_t *steps)
{
    if (!c || !steps) return fail(ORC_ERR_ARG, "null argument");
    *steps = c->steps;
    return ORC_OK;
}

int lbm_info(orc_api_ctx *c, int64_t *cells, int *Q, int64_t *bytes_per_step)
{
    if (!c || !cells || !Q || !bytes_per_step) return fail(ORC_ERR_ARG, "null argument");
    *cells = c->cells;
    *Q = c->m.Q;
    *bytes_per_step = 2 * (int64_t)c->m.Q * c->cells * (int64_t)sizeof(double);
    return ORC_OK;
}

int lbm_velocities(int lattice, int *e_out, int cap, int *Q)
{
    if (!e_out || !Q) return fail(ORC_ERR_ARG, "null argument");
    if (lattice != ORC_D1V3 && lattice != ORC_D2V9 && lattice != ORC_D3V19)
        return fail(ORC_ERR_UNSUPPORTED, "the oracle surface runs d1v3, d2v9 and d3v19");
    orc_model m;
    memset(&m, 0, sizeof m);
    set_velocities(&m, lattice);
    if (cap < 3 * m.Q) return fail(ORC_ERR_ARG, "e_out too small");
    for (int a = 0; a < m.Q; ++a)
        for (int d = 0; d < 3; ++d) e_out[3 * a + d] = m.e[a][d];
    *Q = m.Q;
    return ORC_OK;
}

/* the model the surface builds, for the test against the Python oracle's */
int orc_api_model(const orc_api_config *cfg, orc_model *out)
{
    if (!out) return fail(ORC_ERR_ARG, "null argument");
    return check_config(cfg, out);
}

int lbm_free(orc_api_ctx *c)
{
    free(c);
    return ORC_OK;
}
