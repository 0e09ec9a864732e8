/*
 * lbm.h -- C ABI of the MI355X (gfx950) generalized-polynomial lattice
 * Boltzmann library, liblbm.so.
 *
 * The method is that of Coelho, Ilha and Doria, "A lattice Boltzmann method
 * based on generalized polynomials and its application for electrons in
 * metals" (arXiv:1510.07328): the equilibrium is expanded in polynomials that
 * are orthonormal under the equilibrium itself (section "Generalized
 * polynomials in D dimensions", eqs. omeg-feq, H0-H3), truncated at second or
 * third order (section "The EDF expansion in generalized polynomials",
 * eqs. expansao0, A0-A3), evaluated on a velocity set whose weights solve the
 * discrete moment conditions (section "The Gaussian quadrature", eq. i2n-disc
 * and the d1v3 / d2v9 sets), and advanced by the lattice BGK equation with the
 * moment update that follows it.  The zero-temperature Fermi-Dirac weight is
 * the one of the section "Numerical simulations for electrons in metals".
 *
 * Conventions for every entry point:
 *   - Every call returns lbm_status: 0 on success, a negative code on error.
 *     No exception or abort crosses the ABI.  lbm_last_error() returns a
 *     thread-local message about the last failing call of the calling thread.
 *   - Device memory is never allocated by the library (no hipMalloc): the
 *     caller passes a workspace of at least lbm_workspace_bytes() bytes and
 *     keeps it alive until lbm_free().  The context itself is host memory.
 *   - Work is enqueued on the HIP stream given to lbm_init (NULL = the null
 *     stream); calls are asynchronous unless documented as synchronizing.
 *   - Populations are stored structure-of-arrays, g[alpha][z][y][x] with x
 *     fastest, as deviations g = f - w_alpha rho_ref from the reference state
 *     (float32 for LBM_FP32_DEV, float64 for LBM_FP64).
 *   - Velocities are in lattice units, u0 = u / c_0 (cells per step), where
 *     c_0 = sqrt(3 I_4 / I_2) is the velocity scale of the section on the
 *     Gaussian quadrature.
 *   - One context may not be used by two threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_ERR_ARG = -1,         /* invalid argument (shape, tau <= 1/2, null pointer, size) */
    LBM_ERR_UNSUPPORTED = -2, /* valid but not implemented combination */
    LBM_ERR_HIP = -3,         /* a HIP runtime call failed; text in lbm_last_error() */
    LBM_ERR_NUMERIC = -4,     /* non-finite or non-positive density found */
    LBM_ERR_STATE = -5        /* call not valid for this context */
} lbm_status;

/* Velocity sets.  d1v3 and d2v9 are the sets of section "The Gaussian
 * quadrature"; d3v19 solves the same moment conditions (eq. i2n-disc) through
 * degree 5 in D = 3.  LBM_D2V41 carries the fourth-order expansion (order = 4,
 * P_4 and A_4 of eqs. H4, A4, with delta_{i1i2i3i4} the isotropic four-index
 * delta and the sixth pair term of A_4 read as u_i2 u_i4 delta_i1i3): the 41
 * velocities of the shells |e|^2 = 0, 1, 2, 4, 8, 9, 10, 13, 16, whose weights
 * solve eq. i2n-disc through degree 9 at the scale c_0 where the |e|^2 = 1 and
 * |e|^2 = 16 weights are equal (the largest smallest weight); zero-temperature
 * Fermi-Dirac weight only, periodic boxes with nx, ny >= 4, no obstacles or
 * body force (LBM_ERR_UNSUPPORTED otherwise), at most 512 threads per
 * workgroup (LBM_ERR_ARG otherwise).  Links reach four cells. */
typedef enum { LBM_D1V3 = 1, LBM_D2V9 = 2, LBM_D3V19 = 3, LBM_D2V41 = 4 } lbm_lattice;

/* Weight families (section "Generalized polynomials in D dimensions"):
 *   LBM_W_MB     Maxwell-Boltzmann (Gaussian) weight: J_L = Delta_L = 1, the
 *                Hermite sub-case;
 *   LBM_W_FD_T0  Fermi-Dirac at zero temperature (eq. sommerfeld at theta = 0):
 *                J_L = 1 + 2/(L + D), Delta_L^2 = (D + L)/2;
 *   LBM_W_CUSTOM J_2 and J_4 given in lbm_config, Delta_L^2 from its definition;
 *   LBM_W_FD     Fermi-Dirac at any temperature, LBM_W_BE Bose-Einstein: the
 *                weight's moments I_2N = (2 pi)^(D/2) theta^(N+D/2) g_(N+D/2)(z) with
 *                the complete integrals g_nu(z) = (1/Gamma(nu)) int_0^inf x^(nu-1) /
 *                (z^-1 e^x +- 1) dx at the fugacity z = e^(mu/theta) of lbm_config
 *                (paragraph before eq. sommerfeld); J_L depend on z only.  z > 0
 *                (Fermi-Dirac), 0 < z < 1 (Bose-Einstein); LBM_ERR_ARG otherwise;
 *   LBM_W_FD_LOCAL Fermi-Dirac at a temperature theta > 0 with the weights and
 *                equilibrium coefficients recomputed in every cell and step from
 *                the cell's chemical potential (section "The Gaussian quadrature":
 *                the weights follow the integrals I_2N and are updated every time
 *                step).  I_2N from eq. sommerfeld cut after the (theta/mu)^2 term,
 *                I_2N ~ mu^nu / Gamma(nu + 1) [1 + (pi^2/6) nu (nu - 1) (theta/mu)^2],
 *                nu = N + D/2; the cell's mu solves I_0(mu) / I_0(mu_ref) =
 *                n / rho_ref (exactly mu / mu_ref = n / rho_ref in D = 2, four
 *                Newton steps in D = 1, 3), so J_L = J_L(theta/mu) per cell.
 *                theta_over_mu of lbm_config is theta / mu_ref at rho_ref, in
 *                [0, 0.5].  The lattice e_a stays fixed, so velocities are in units
 *                of the cell's own c_0.  Periodic or bounce-back boxes without
 *                obstacles or body force (LBM_ERR_UNSUPPORTED with either, and in
 *                the batched sweep); lbm_coefficients reports the coefficients
 *                of a cell at rho_ref. */
typedef enum {
    LBM_W_MB = 0,
    LBM_W_FD_T0 = 1,
    LBM_W_CUSTOM = 2,
    LBM_W_FD = 3,
    LBM_W_BE = 4,
    LBM_W_FD_LOCAL = 5
} lbm_weight;

typedef enum { LBM_FP32_DEV = 0, LBM_FP64 = 1 } lbm_precision;
typedef enum { LBM_PERIODIC = 0, LBM_BOUNCEBACK = 1 } lbm_bc;
typedef enum { LBM_SCHEME_PUSH = 0, LBM_SCHEME_AA = 1 } lbm_scheme;

typedef struct {
    int lattice;      /* lbm_lattice; D = 1, 2, 3 */
    int nx, ny, nz;   /* box size; ny = nz = 1 for D = 1, nz = 1 for D = 2 */
    int bc[3];        /* lbm_bc per axis (both faces); bounce-back is the halfway,
                         link-wise form: walls at -1/2 and n - 1/2 */
    int weight;       /* lbm_weight */
    double J2, J4;    /* used only with LBM_W_CUSTOM */
    int order;        /* truncation order of the expansion, 2 or 3 (4 with LBM_D2V41) */
    double tau;       /* BGK relaxation time, > 1/2 */
    int precision;    /* lbm_precision */
    double rho_ref;   /* deviation reference density (1.0 if <= 0) */
    int scheme;       /* lbm_scheme: two-lattice push, or in-place AA (same results) */
    int block;        /* threads per workgroup, 0 = library default (multiple of 64, <= 1024) */
    int graph_steps;  /* > 0: replay steps in captured HIP graphs of this many steps */
    /* Porous media (section "Numerical simulations for electrons in metals":
     * flow through rigid obstacles under a constant external force).  With
     * obstacles = 1 the workspace holds a per-cell link mask and lbm_set_solid
     * marks solid cells (halfway bounce-back at every link that ends in one).
     * force is a constant body force density per cell and step, lattice units,
     * applied as the exact difference of equilibria
     * f_eq(n, u + F/n) - f_eq(n, u) after relaxation; zero means none. */
    int obstacles;    /* 0 or 1 */
    double force[3];  /* components beyond D are ignored */
    double fugacity;  /* z = e^(mu/theta) for LBM_W_FD and LBM_W_BE */
    double theta_over_mu; /* theta / mu at rho_ref for LBM_W_FD_LOCAL */
} lbm_config;

typedef struct lbm_ctx_s *lbm_ctx;

/* Coefficients of the collapsed per-class equilibrium (a0 of the hot path).
 *
 * Section "The Gaussian quadrature", the geometric-space form of the discrete
 * equilibrium, split by truncation order and collapsed per velocity class
 * (classes are |e|^2 = 0, 1, 2):
 *   f_eq,a = n w_a S_a,  S_a - 1 = eu (l1 + c3 u^2 + k4 eu^2) + q eu^2 + s u^2,
 *   eu = e_a . u0, u^2 = u0 . u0.
 * Writes, per class k = 0..ncls-1, six float64 values
 *   out[6k + 0..5] = { w_k, l1_k, q_k, s_k, c3_k, k4_k },
 * followed by { J2, J4, Delta2^2, Delta4^2 }; for LBM_D2V41 (ncls = 9) then
 * the fourth-order terms of S - 1, p4 eu^4 + r4 eu^2 u^2 + t4 u^4, as
 * { p4_k, r4_k, t4_k } per class, and last c_0 / sqrt(3 I_4 / I_2).  cap is the capacity of out in
 * doubles; *n_written receives the count.  Host only, synchronous, never
 * touches the GPU.  LBM_ERR_ARG if cap is too small or cfg is invalid. */
lbm_status lbm_coefficients(const lbm_config *cfg, double *out, int cap, int *n_written);

/* Bytes of device workspace lbm_init needs for cfg (two lattices for the
 * push scheme, one for AA, plus reduction scratch and the staging area of
 * the host lbm_moments, about 4 MB).  Host only. */
lbm_status lbm_workspace_bytes(const lbm_config *cfg, size_t *bytes);

/* Create a context and set the populations to equilibrium with the given
 * density and velocity fields (initial condition f = f_eq(n0, u0)).
 *   workspace: device pointer, >= lbm_workspace_bytes(cfg) bytes, 256-byte
 *              aligned; borrowed until lbm_free.
 *   stream:    hipStream_t the context enqueues on (NULL = null stream).
 *   n0_dev:    device float64 [nz][ny][nx] density I_0;
 *   u0_dev:    device float64 [D][nz][ny][nx] velocity u0.
 * The inputs are read by the time the stream reaches the end of this call.
 * LBM_ERR_ARG for an invalid cfg or size, LBM_ERR_HIP on a HIP failure. */
lbm_status lbm_init(const lbm_config *cfg, void *workspace, size_t bytes, void *stream,
                    const double *n0_dev, const double *u0_dev, lbm_ctx *out);

/* Advance nsteps lattice BGK steps (lattice BGK equation: stream, moments,
 * equilibrium, relaxation), fused into one kernel per step.  Asynchronous. */
lbm_status lbm_step(lbm_ctx ctx, int64_t nsteps);

/* Density n = I_0 and velocity u0 of the current populations (moment update
 * after the lattice BGK equation: I_0 = sum_a f_a, u0 = sum_a f_a e_a / I_0),
 * into caller host buffers n_host float64 [cells] and u_host float64
 * [D][cells] (layout [nz][ny][nx], x fastest).  With a body force the velocity
 * is the forced scheme's (sum_a f_a e_a + F/2) / I_0.  Computed on the device a
 * few MB of rows at a time through a staging area in the workspace and copied
 * back; synchronizes the context stream. */
lbm_status lbm_moments(lbm_ctx ctx, double *n_host, double *u_host);

/* The same moments written to caller device buffers n_dev float64 [cells] and
 * u_dev float64 [D][cells] by one kernel.  Asynchronous. */
lbm_status lbm_moments_device(lbm_ctx ctx, double *n_dev, double *u_dev);

/* Totals over the box in float64: out_host[0] = sum n, out_host[1..D] =
 * sum_cells sum_a f_a e_a (mass and momentum, solid cells left out; without
 * the half-force term), by wavefront reductions and a second
 * deterministic pass.  Synchronizes the context stream.  LBM_ERR_NUMERIC if a
 * total is not finite. */
lbm_status lbm_totals(lbm_ctx ctx, double *out_host);

/* Raw populations in storage precision and layout, with the streaming pattern
 * of the scheme resolved: the values are g = f(x, t) - w rho_ref at their
 * natural slots, f(x, t) the post-streaming populations after t steps.  bytes
 * must equal Q * cells * sizeof(storage).  Synchronizes.  Together with
 * lbm_steps_done these checkpoint a run (set_state restores bit for bit). */
lbm_status lbm_get_state(lbm_ctx ctx, void *host, size_t bytes);
lbm_status lbm_set_state(lbm_ctx ctx, const void *host, size_t bytes);
lbm_status lbm_steps_done(lbm_ctx ctx, int64_t *steps);

/* Cell count, population count and the bytes one step kernel moves by its
 * algorithm (read and write every population once: 2 Q cells sizeof(storage)),
 * for measurement.  Host only. */
lbm_status lbm_info(lbm_ctx ctx, int64_t *cells, int *Q, int64_t *bytes_per_step);

/* The velocity set in the library's population order: e_out[3 a + d] is
 * component d of e_a (zero-padded to three components).  cap is the capacity
 * of e_out in ints; *Q receives the population count.  Host only. */
lbm_status lbm_velocities(int lattice, int *e_out, int cap, int *Q);

/* Mark solid cells of a context created with obstacles = 1 from a device mask
 * of one byte per cell (nonzero = solid), [nz][ny][nx] x fastest; the mask is
 * read during the call's kernel (asynchronous) and may be reused after the
 * stream reaches it.  Solid cells take no part in the step; moments report
 * n = 0, u = 0 there and totals leave them out.  LBM_ERR_STATE without
 * obstacles or after an odd number of AA steps. */
lbm_status lbm_set_solid(lbm_ctx ctx, const unsigned char *solid_dev);

/* Release the context (host memory and any captured graphs).  Does not free
 * the workspace.  Synchronizes the stream. */
lbm_status lbm_free(lbm_ctx ctx);

const char *lbm_last_error(void);

/* ---------------------------------------------------------------------------
 * Batched closed shock tubes.
 *
 * Many independent Riemann problems (section "Numerical simulations for
 * electrons in metals": a density step at rest, advanced by the lattice BGK
 * equation of section "The Gaussian quadrature") on d2v9 boxes of nx x 4 cells
 * with halfway bounce-back walls in x and periodic y, each with its own nx,
 * tau, density pair and number of steps, advanced together.  Each tube is
 * computed cell for cell as lbm_step computes an nx x 4 box (same results, bit
 * for bit).  Internally tiles of a tube are advanced several steps at a time in
 * LDS (temporal blocking), in rounds over all tubes.
 * ------------------------------------------------------------------------- */
typedef struct {
    int nx;                  /* columns (>= 2) */
    double tau;              /* > 1/2 */
    double n_left, n_right;  /* density for x < nx/2 and beyond, velocity 0 */
    int64_t steps;           /* steps of lbm_batch_run for this tube */
} lbm_tube;

typedef struct {
    int weight;              /* lbm_weight (not LBM_W_FD_LOCAL) */
    double J2, J4;           /* LBM_W_CUSTOM only */
    int order;               /* 2 or 3 */
    int precision;           /* lbm_precision */
    double rho_ref;          /* deviation reference (1.0 if <= 0) */
    int tile_cols;           /* columns per tile, 0 = the largest that fits LDS with the halo */
    int halo;                /* steps per round = halo columns per side, 0 = 64 */
    int block;               /* threads per workgroup, 0 = 1024 */
    int use_graph;           /* capture lbm_batch_run's rounds into one HIP graph */
    double fugacity;         /* LBM_W_FD / LBM_W_BE only */
} lbm_batch_options;

typedef struct lbm_batch_s *lbm_batch;

/* Device workspace for the tube set (two population buffers plus tables). */
lbm_status lbm_batch_workspace_bytes(const lbm_tube *tubes, int ntubes, const lbm_batch_options *opt,
                                     size_t *bytes);

/* Create the batch and set every tube to its initial step (f = f_eq(n, 0)).
 * tubes: host array, read during the call.  workspace: device, 256-byte
 * aligned, borrowed until lbm_batch_free.  Synchronizes the stream once.
 * LBM_ERR_ARG for invalid tubes, options or sizes. */
lbm_status lbm_batch_init(const lbm_tube *tubes, int ntubes, const lbm_batch_options *opt, void *workspace,
                          size_t bytes, void *stream, lbm_batch *out);

/* Advance every tube by its own `steps` (one HIP graph launch when use_graph). */
lbm_status lbm_batch_run(lbm_batch b);

/* Advance the tubes with active_host[t] != 0 (all if NULL) by nsteps.
 * Synchronizes the stream before reusing its staging tables. */
lbm_status lbm_batch_advance(lbm_batch b, int64_t nsteps, const unsigned char *active_host);

/* Set the masked tubes (all if mask_host is NULL) to f = f_eq(n, u) from packed
 * device float64 fields n[cells], u[2][cells] in tube order (lbm_batch_layout),
 * x fastest within a tube.  Synchronizes. */
lbm_status lbm_batch_set_equilibrium(lbm_batch b, const double *n_dev, const double *u_dev,
                                     const unsigned char *mask_host);

/* Packed float64 moments of every tube into device buffers n[cells], u[2][cells]
 * (layout as above).  Asynchronous. */
lbm_status lbm_batch_moments(lbm_batch b, double *n_dev, double *u_dev);

/* Row-averaged float32 profiles of tubes of equal nx: prof_dev[t][0][x] = n,
 * prof_dev[t][1][x] = u0_x, device buffer of ntubes * 2 * nx floats.
 * LBM_ERR_UNSUPPORTED if the tubes differ in length.  Asynchronous. */
lbm_status lbm_batch_profiles(lbm_batch b, float *prof_dev);

/* Set the masked tubes (all if NULL) to f = f_eq(n(x), (u(x), 0)) on every row
 * from profiles laid out as lbm_batch_profiles writes them.  Synchronizes. */
lbm_status lbm_batch_set_profiles(lbm_batch b, const float *prof_dev, const unsigned char *mask_host);

/* Per tube, the number of cells whose density is not finite and positive or
 * whose momentum is not finite (the tube has broken down).  Synchronizes. */
lbm_status lbm_batch_health(lbm_batch b, int *bad_cells_host);

/* First packed cell of every tube; cell_offsets_host has ntubes + 1 entries. */
lbm_status lbm_batch_layout(lbm_batch b, int64_t *cell_offsets_host);

/* Totals for measurement: cells, lattice updates of one lbm_batch_run, rounds,
 * and the tile shape in use. */
lbm_status lbm_batch_info(lbm_batch b, int64_t *total_cells, int64_t *updates_per_run, int *rounds, int *tile_cols,
                          int *halo);

lbm_status lbm_batch_free(lbm_batch b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
