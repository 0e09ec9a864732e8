/*
 * Declarations of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY), shared by its
 * two C files: lbm_oracle.c (the lattice BGK iteration) and lbm_oracle_api.c
 * (the lbm_* call surface over it).  Nothing outside oracle/ includes this.
 */
#ifndef ORACLE_LBM_ORACLE_H
#define ORACLE_LBM_ORACLE_H

#define ORC_MAXQ 48

typedef struct {
    int D, Q;
    int e[ORC_MAXQ][3];
    double w_hat[ORC_MAXQ]; /* w_a / I_0 */
    int opp[ORC_MAXQ];
    double cvel;            /* c_0 */
    double I0, J2;          /* reference-state integral and J_2 */
    double c[5], cp[5], cb[5];
    double d4, dp4, db4;    /* isotropic-term coefficients of P_4 (after eq. H4) */
    double J4, I2;          /* for A_4 (eq. A4) */
    int order;              /* truncation order, 0..4 */
    int nx, ny, nz;
    int bc[3];              /* 0 = periodic, 1 = halfway bounce-back */
    double tau;
} orc_model;

int orc_feq(const orc_model *m, double n, const double *u0, double *feq);
int orc_init(const orc_model *m, const double *n0, const double *u0, double *f);
int orc_moments(const orc_model *m, const double *f, double *n, double *u0);
int orc_run(const orc_model *m, double *f, long steps);
int orc_run_porous(const orc_model *m, const unsigned char *solid, const double *force, double *f, long steps);

#endif
