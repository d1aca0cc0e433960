/*
 * grmhd_oracle.h -- plain FP64 CPU oracle for the GRMHD substep of
 * Zink, "HORIZON: Accelerated General Relativistic Magnetohydrodynamics"
 * (arXiv:1102.5202).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may include, link or call this code; only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
 * no source with the GPU path.
 *
 * What it computes (paper section 2, eq. 2 and the compact form eq. 3; scheme
 * choices of section 3.2): the finite-volume update of the conserved variables
 *   U = ( sqrt(-g) rho u^t,  -sqrt(-g)(T^t_t + rho u^t),  sqrt(-g) T^t_j,
 *         sqrt(-g) B^j,  Phi )
 * in a fixed static metric, with MC-limited TVD reconstruction (or, as the
 * alternative section 3.2 names, PPM) of the
 * primitives P = (rho, p, u~^x, u~^y, u~^z, B^x, B^y, B^z, Phi), HLLE face
 * fluxes, metric source terms, a bracketed Newton recovery of P from U, and
 * an SSP Runge-Kutta update.  Divergence violations are damped with a
 * GLM-type hyperbolic cleaning scalar Phi.
 *
 * Arrays are structure-of-arrays [var][z][y][x] over interior cells only,
 * x fastest.  Boundary conditions are applied by index mapping.
 */
#ifndef GRMHD_ORACLE_H
#define GRMHD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NVAR 9

enum { ORC_FLAT = 0, ORC_ISO_SCHW = 1, ORC_STORED = 2 };
enum { ORC_SOFT_SQRT = 0, ORC_SOFT_MAX = 1 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1 };
enum { ORC_RECON_MC = 0, ORC_RECON_PPM = 1 };

/* cell flags produced by the recovery + floor policy */
enum { ORC_FLAG_FAIL = 1, ORC_FLAG_ATM = 2, ORC_FLAG_PFLOOR = 4 };

typedef struct {
    int kind;       /* ORC_FLAT, ORC_ISO_SCHW or ORC_STORED (grids only) */
    int soft;       /* radius softening: ORC_SOFT_SQRT or ORC_SOFT_MAX   */
    double M;       /* mass parameter (G = c = 1)                        */
    double r_min;   /* softening radius                                  */
    /* ORC_STORED: a static, conformally flat metric with zero shift given
     * by its lapse and conformal factor psi^4 at the cell centres of the
     * grid and of 2 ghost layers on every active axis ([z][y][x], x
     * fastest, n + 4 per active axis, n otherwise).                      */
    const double *alpha_grid;
    const double *psi4_grid;
} orc_metric;

typedef struct {
    int n[3];       /* interior cells per axis; n = 1 switches an axis off */
    double lo[3];
    double hi[3];
    int bc[3];      /* ORC_BC_PERIODIC or ORC_BC_OUTFLOW                 */
} orc_grid;

typedef struct {
    orc_metric metric;
    orc_grid grid;
    double gamma;   /* ideal-gas adiabatic index                         */
    int rk_order;   /* 2 or 3 (SSP)                                      */
    double c_h;     /* cleaning speed                                    */
    double kappa;   /* cleaning damping rate                             */
    double rho_atm; /* atmosphere density                                */
    double p_atm;   /* atmosphere / floor pressure                       */
    int recon;      /* ORC_RECON_MC or ORC_RECON_PPM                     */
    int ct;         /* 0: hyperbolic cleaning; 1: flux-CT (Phi carried)  */
} orc_problem;

typedef struct {
    long long fail;    /* cells where the recovery found no physical root */
    long long atm;     /* cells reset to the atmosphere                  */
    long long pfloor;  /* cells whose pressure was raised to the floor   */
} orc_stats;

void orc_set_threads(int n);
int orc_get_threads(void);

/* Whole-grid operations (dense interior arrays, 9*N doubles each). */
int orc_prim2con(const orc_problem *pb, const double *P, double *U);
/* Recovery plus floors.  U may be modified in floored/failed cells. */
int orc_con2prim(const orc_problem *pb, double *U, const double *Pguess,
                 double *P, unsigned char *flags, orc_stats *st);
/* Right-hand side L(P) = -sum_d dF_d/dx_d + s of one substep. */
int orc_rhs(const orc_problem *pb, const double *P, double *R);
/* nsteps full SSP-RK steps in place on (U, P). */
int orc_step(const orc_problem *pb, double *U, double *P, double dt,
             int nsteps, orc_stats *st);

/* Point functions (used by the pins). */
void orc_point_geom(const orc_metric *m, double x, double y, double z,
                    double *out /* alpha, sqrtgamma, sqrtmg, g[16], gi[16], dg[48] */);
void orc_point_cons(const orc_metric *m, double gamma, double x, double y,
                    double z, const double *P, double *U);
void orc_point_flux(const orc_metric *m, double gamma, double c_h, int dir,
                    double x, double y, double z, const double *P, double *F);
void orc_point_speeds(const orc_metric *m, double gamma, int dir, double x,
                      double y, double z, const double *P, double *lm, double *lp);
void orc_point_stress(const orc_metric *m, double gamma, double x, double y,
                      double z, const double *P, double *T /* T^mu_nu, 16 */);
void orc_point_source(const orc_metric *m, double gamma, double kappa, double x,
                      double y, double z, const double *P, double *S);
int orc_point_c2p(const orc_metric *m, double gamma, double x, double y,
                  double z, const double *U, double *P);
void orc_point_face_flux(const orc_metric *m, double gamma, double c_h, int dir,
                         double x, double y, double z, const double *qL,
                         const double *qR, double *F);
double orc_mc_slope(double qm, double q0, double qp);
void orc_ppm_edges(const double *a /* cells i-2..i+2 */, double *aL, double *aR);

#ifdef __cplusplus
}
#endif
#endif
