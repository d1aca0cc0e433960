/*
 * grmhd_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Written from the paper's description of the method (arXiv:1102.5202,
 * section 2.2 and section 3.2) as plain loops over cells, in double precision,
 * with IEEE semantics (build without -ffast-math).  Every quantity is formed
 * from its textbook definition through full 4x4 metric contractions, so that
 * the code can be read against the equations directly; nothing is blocked,
 * fused or reordered.  The GPU path is a separate implementation; the two
 * share no code.
 *
 * Readings of points the paper leaves open (each is also listed in the design
 * notes of the repository):
 *  - energy variable: tau = -sqrt(-g)(T^t_t + rho u^t), the T^t_t row minus
 *    the rest-mass row (both conserved rows of eq. 2);
 *  - primitives: rho, p, the velocities u~^i = u^i + W beta^i/alpha of the
 *    footnote in section 5.2, B^i, Phi;
 *  - induction flux: sqrt(-g)(b^j u^i - b^i u^j), the sign that follows from
 *    nabla_mu *F^{mu nu} = 0 (eq. 1);
 *  - wave speeds: fast-magnetosonic isotropic estimate
 *    c^2 = cs^2 + ca^2 - cs^2 ca^2 inserted in the dispersion relation;
 *  - divergence cleaning: GLM scalar Phi with d_t Bd^j + d_i(.. + delta^ij Phi)
 *    = 0 and d_t Phi + d_i(c_h^2 Bd^i) = -kappa Phi; the (Bd^n, Phi) pair is
 *    solved exactly at each face;
 *  - source: the Christoffel contraction of eq. 2 in the equivalent form
 *    1/2 sqrt(-g) T^{kl} d_mu g_{kl};
 *  - recovery: one-dimensional bracketed Newton in the variable
 *    Wc = rho h W^2 with v^2 eliminated (the 2D_W equations reduced to one
 *    unknown);
 *  - atmosphere/floors: see c2p_cell().
 */
#include "grmhd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 1;

void orc_set_threads(int n)
{
    g_threads = n > 0 ? n : 1;
}

int orc_get_threads(void)
{
    return g_threads;
}

/* ------------------------------------------------------------------------ */
/* Geometry: a static metric with lapse alpha, shift beta^i = 0 and a
 * conformally flat spatial metric gamma_ij = psi^4 delta_ij.  ORC_ISO_SCHW is
 * the Schwarzschild metric in isotropic coordinates with the radius softened
 * near the origin, alpha = (1 - M/(2r))/(1 + M/(2r)), psi = 1 + M/(2r).      */

typedef struct {
    double alpha;
    double beta[3];
    double gam[3][3];
    double gami[3][3];
    double sqrtgamma;
    double sqrtmg;
    double g[4][4];     /* g_{mu nu}               */
    double gi[4][4];    /* g^{mu nu}               */
    double dg[4][4][4]; /* d_mu g_{kl}; mu = 0 is the time derivative */
} geom;

static double det3(const double a[3][3])
{
    return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1])
         - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
         + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
}

static void inv3(const double a[3][3], double r[3][3])
{
    double d = det3(a);
    r[0][0] = (a[1][1] * a[2][2] - a[1][2] * a[2][1]) / d;
    r[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / d;
    r[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / d;
    r[1][0] = (a[1][2] * a[2][0] - a[1][0] * a[2][2]) / d;
    r[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / d;
    r[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / d;
    r[2][0] = (a[1][0] * a[2][1] - a[1][1] * a[2][0]) / d;
    r[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) / d;
    r[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / d;
}

static void geom_build(double alpha, double psi4, const double *dalpha, const double *dpsi4, geom *G);

static void geom_at(const orc_metric *m, double x, double y, double z, geom *G)
{
    double alpha = 1.0, psi4 = 1.0;
    double dalpha[3] = {0.0, 0.0, 0.0}, dpsi4[3] = {0.0, 0.0, 0.0};
    int i;

    if (m->kind == ORC_ISO_SCHW) {
        double xs[3] = {x, y, z};
        double r = sqrt(x * x + y * y + z * z);
        double rs, drs[3];
        if (m->soft == ORC_SOFT_SQRT) {
            rs = sqrt(r * r + m->r_min * m->r_min);
            for (i = 0; i < 3; i++)
                drs[i] = xs[i] / rs;
        } else if (r > m->r_min) {
            rs = r;
            for (i = 0; i < 3; i++)
                drs[i] = xs[i] / r;
        } else {
            rs = m->r_min;
            for (i = 0; i < 3; i++)
                drs[i] = 0.0;
        }
        {
            double h = m->M / (2.0 * rs);       /* M/(2 r_s)              */
            double dh = -h / rs;                /* d h / d r_s            */
            double psi = 1.0 + h;
            double dalpha_dh = -2.0 / ((1.0 + h) * (1.0 + h));
            double dpsi4_dh = 4.0 * psi * psi * psi;
            alpha = (1.0 - h) / (1.0 + h);
            psi4 = psi * psi * psi * psi;
            for (i = 0; i < 3; i++) {
                dalpha[i] = dalpha_dh * dh * drs[i];
                dpsi4[i] = dpsi4_dh * dh * drs[i];
            }
        }
    }

    geom_build(alpha, psi4, dalpha, dpsi4, G);
}

/* The static metric with zero shift, lapse alpha and spatial metric
 * psi4 delta_ij, with the spatial derivatives of alpha and psi4. */
static void geom_build(double alpha, double psi4, const double *dalpha, const double *dpsi4, geom *G)
{
    int i, j, mu, nu;
    memset(G, 0, sizeof *G);
    G->alpha = alpha;
    for (i = 0; i < 3; i++)
        G->beta[i] = 0.0;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++)
            G->gam[i][j] = (i == j) ? psi4 : 0.0;
    inv3(G->gam, G->gami);
    G->sqrtgamma = sqrt(det3(G->gam));
    G->sqrtmg = alpha * G->sqrtgamma;

    /* 4-metric from lapse, shift and spatial metric */
    {
        double betal[3];
        double bb = 0.0;
        for (i = 0; i < 3; i++) {
            betal[i] = 0.0;
            for (j = 0; j < 3; j++)
                betal[i] += G->gam[i][j] * G->beta[j];
            bb += betal[i] * G->beta[i];
        }
        G->g[0][0] = -alpha * alpha + bb;
        for (i = 0; i < 3; i++) {
            G->g[0][i + 1] = G->g[i + 1][0] = betal[i];
            for (j = 0; j < 3; j++)
                G->g[i + 1][j + 1] = G->gam[i][j];
        }
        G->gi[0][0] = -1.0 / (alpha * alpha);
        for (i = 0; i < 3; i++) {
            G->gi[0][i + 1] = G->gi[i + 1][0] = G->beta[i] / (alpha * alpha);
            for (j = 0; j < 3; j++)
                G->gi[i + 1][j + 1] = G->gami[i][j]
                                      - G->beta[i] * G->beta[j] / (alpha * alpha);
        }
    }

    /* metric derivatives: static, so d_t g = 0; spatial from the closed form */
    for (mu = 0; mu < 4; mu++)
        for (nu = 0; nu < 4; nu++)
            G->dg[0][mu][nu] = 0.0;
    for (i = 0; i < 3; i++) {
        for (mu = 0; mu < 4; mu++)
            for (nu = 0; nu < 4; nu++)
                G->dg[i + 1][mu][nu] = 0.0;
        G->dg[i + 1][0][0] = -2.0 * alpha * dalpha[i];
        for (j = 0; j < 3; j++)
            G->dg[i + 1][j + 1][j + 1] = dpsi4[i];
    }
}

/* A stored metric (ORC_STORED): the value of a ghosted centre array at cell
 * (i, j, k) of the grid (indices down to -2 on active axes). */
static double stored_at(const orc_grid *g, const double *a, int i, int j, int k)
{
    int gx = g->n[0] > 1 ? 2 : 0, gy = g->n[1] > 1 ? 2 : 0, gz = g->n[2] > 1 ? 2 : 0;
    long long px = g->n[0] + 2 * gx, py = g->n[1] + 2 * gy;
    return a[((long long)(k + gz) * py + (j + gy)) * px + (i + gx)];
}

/* Along axis d from cell (i, j, k): the value s cells away. */
static double stored_off(const orc_grid *g, const double *a, int d, int i, int j, int k, int s)
{
    int ix[3] = {i, j, k};
    ix[d] += s;
    return stored_at(g, a, ix[0], ix[1], ix[2]);
}

/* Metric at the centre of cell (i, j, k): analytic, or for a stored metric
 * the stored values with fourth-order central differences
 * (a_{i-2} - 8 a_{i-1} + 8 a_{i+1} - a_{i+2}) / (12 dx) for the derivatives
 * (zero along an inactive axis). */
static void geom_cell(const orc_problem *pb, int i, int j, int k, geom *G)
{
    const orc_grid *g = &pb->grid;
    const orc_metric *m = &pb->metric;
    double da[3], dp[3];
    int d;
    if (m->kind != ORC_STORED) {
        /* the cell centres, evaluated as everywhere else in this file */
        geom_at(m, g->lo[0] + (i + 0.5) * ((g->hi[0] - g->lo[0]) / g->n[0]),
                g->lo[1] + (j + 0.5) * ((g->hi[1] - g->lo[1]) / g->n[1]),
                g->lo[2] + (k + 0.5) * ((g->hi[2] - g->lo[2]) / g->n[2]), G);
        return;
    }
    for (d = 0; d < 3; d++) {
        double dx = (g->hi[d] - g->lo[d]) / g->n[d];
        da[d] = dp[d] = 0.0;
        if (g->n[d] == 1)
            continue;
        da[d] = (stored_off(g, m->alpha_grid, d, i, j, k, -2) - 8.0 * stored_off(g, m->alpha_grid, d, i, j, k, -1)
                 + 8.0 * stored_off(g, m->alpha_grid, d, i, j, k, 1) - stored_off(g, m->alpha_grid, d, i, j, k, 2))
                / (12.0 * dx);
        dp[d] = (stored_off(g, m->psi4_grid, d, i, j, k, -2) - 8.0 * stored_off(g, m->psi4_grid, d, i, j, k, -1)
                 + 8.0 * stored_off(g, m->psi4_grid, d, i, j, k, 1) - stored_off(g, m->psi4_grid, d, i, j, k, 2))
                / (12.0 * dx);
    }
    geom_build(stored_at(g, m->alpha_grid, i, j, k), stored_at(g, m->psi4_grid, i, j, k), da, dp, G);
}

/* Metric at face fi[d] along d (between cells fi[d]-1 and fi[d]; position
 * pos): analytic, or for a stored metric the fourth-order interpolation
 * (-a_{f-2} + 9 a_{f-1} + 9 a_f - a_{f+1}) / 16 of the stored values. */
static void geom_face(const orc_problem *pb, int d, const int *fi, const double *pos, geom *G)
{
    const orc_grid *g = &pb->grid;
    const orc_metric *m = &pb->metric;
    static const double zero[3] = {0.0, 0.0, 0.0};
    double a, p;
    if (m->kind != ORC_STORED) {
        geom_at(m, pos[0], pos[1], pos[2], G);
        return;
    }
    a = (-stored_off(g, m->alpha_grid, d, fi[0], fi[1], fi[2], -2) + 9.0 * stored_off(g, m->alpha_grid, d, fi[0], fi[1], fi[2], -1)
         + 9.0 * stored_off(g, m->alpha_grid, d, fi[0], fi[1], fi[2], 0) - stored_off(g, m->alpha_grid, d, fi[0], fi[1], fi[2], 1))
        / 16.0;
    p = (-stored_off(g, m->psi4_grid, d, fi[0], fi[1], fi[2], -2) + 9.0 * stored_off(g, m->psi4_grid, d, fi[0], fi[1], fi[2], -1)
         + 9.0 * stored_off(g, m->psi4_grid, d, fi[0], fi[1], fi[2], 0) - stored_off(g, m->psi4_grid, d, fi[0], fi[1], fi[2], 1))
        / 16.0;
    geom_build(a, p, zero, zero, G);
}

/* ------------------------------------------------------------------------ */
/* State of the fluid + field from the primitives (Noble et al. 2006 form). */

typedef struct {
    double rho, p, ut[3], B[3], phi;
    double W;      /* Lorentz factor of the normal observer      */
    double u[4];   /* u^mu                                       */
    double ul[4];  /* u_mu                                       */
    double b[4];   /* b^mu                                       */
    double bl[4];  /* b_mu                                       */
    double b2;     /* b^mu b_mu                                  */
    double w;      /* rho h = rho + Gamma/(Gamma-1) p            */
} state;

static void state_from_prim(const geom *G, double gamma, const double *P, state *s)
{
    double uu = 0.0;
    int i, j, mu, nu;

    s->rho = P[0];
    s->p = P[1];
    for (i = 0; i < 3; i++) {
        s->ut[i] = P[2 + i];
        s->B[i] = P[5 + i];
    }
    s->phi = P[8];

    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++)
            uu += G->gam[i][j] * s->ut[i] * s->ut[j];
    s->W = sqrt(1.0 + uu);
    s->u[0] = s->W / G->alpha;
    for (i = 0; i < 3; i++)
        s->u[i + 1] = s->ut[i] - s->W * G->beta[i] / G->alpha;
    for (mu = 0; mu < 4; mu++) {
        s->ul[mu] = 0.0;
        for (nu = 0; nu < 4; nu++)
            s->ul[mu] += G->g[mu][nu] * s->u[nu];
    }
    s->b[0] = 0.0;
    for (i = 0; i < 3; i++)
        s->b[0] += s->B[i] * s->ul[i + 1];
    for (i = 0; i < 3; i++)
        s->b[i + 1] = (s->B[i] + s->b[0] * s->u[i + 1]) / s->u[0];
    for (mu = 0; mu < 4; mu++) {
        s->bl[mu] = 0.0;
        for (nu = 0; nu < 4; nu++)
            s->bl[mu] += G->g[mu][nu] * s->b[nu];
    }
    s->b2 = 0.0;
    for (mu = 0; mu < 4; mu++)
        s->b2 += s->b[mu] * s->bl[mu];
    s->w = s->rho + gamma / (gamma - 1.0) * s->p;
}

/* T^mu_nu = (w + b^2) u^mu u_nu + (p + b^2/2) delta^mu_nu - b^mu b_nu */
static void stress_mixed(const state *s, double T[4][4])
{
    int mu, nu;
    for (mu = 0; mu < 4; mu++)
        for (nu = 0; nu < 4; nu++)
            T[mu][nu] = (s->w + s->b2) * s->u[mu] * s->ul[nu]
                        + (mu == nu ? s->p + 0.5 * s->b2 : 0.0)
                        - s->b[mu] * s->bl[nu];
}

/* conserved variables w(u): algebraic (section 2.2) */
static void cons_from_state(const geom *G, const state *s, double *U)
{
    double T[4][4];
    int j;
    stress_mixed(s, T);
    U[0] = G->sqrtmg * s->rho * s->u[0];
    U[1] = -G->sqrtmg * (T[0][0] + s->rho * s->u[0]);
    for (j = 0; j < 3; j++) {
        U[2 + j] = G->sqrtmg * T[0][j + 1];
        U[5 + j] = G->sqrtmg * s->B[j];
    }
    U[8] = s->phi;
}

/* physical flux f^i of eq. 2 in direction dir (0,1,2), with the cleaning terms */
static void flux_from_state(const geom *G, const state *s, double c_h, int dir, double *F)
{
    double T[4][4];
    int i = dir + 1, j;
    stress_mixed(s, T);
    F[0] = G->sqrtmg * s->rho * s->u[i];
    F[1] = -G->sqrtmg * (T[i][0] + s->rho * s->u[i]);
    for (j = 0; j < 3; j++) {
        F[2 + j] = G->sqrtmg * T[i][j + 1];
        F[5 + j] = G->sqrtmg * (s->b[j + 1] * s->u[i] - s->b[i] * s->u[j + 1])
                   + (j == dir ? s->phi : 0.0);
    }
    F[8] = c_h * c_h * G->sqrtmg * s->B[dir];
}

/* Approximate extreme characteristic speeds dx^i/dt in direction dir. */
static void speeds_from_state(const geom *G, const state *s, double gamma, int dir,
                              double *lm, double *lp)
{
    int i = dir + 1;
    double cs2 = gamma * s->p / s->w;
    double ca2 = s->b2 / (s->w + s->b2);
    double c2 = cs2 + ca2 - cs2 * ca2;
    double ut = s->u[0], ui = s->u[i];
    double A = ut * ut - c2 * (G->gi[0][0] + ut * ut);
    double B = ut * ui - c2 * (G->gi[0][i] + ut * ui);
    double C = ui * ui - c2 * (G->gi[i][i] + ui * ui);
    double disc = B * B - A * C;
    double sq, l1, l2;
    if (disc < 0.0)
        disc = 0.0;
    sq = sqrt(disc);
    l1 = (B + sq) / A;
    l2 = (B - sq) / A;
    *lp = l1 > l2 ? l1 : l2;
    *lm = l1 > l2 ? l2 : l1;
}

/* Source s(u) of eq. 2: sqrt(-g) T^k_l Gamma^l_{mu k} = 1/2 sqrt(-g) T^{kl} d_mu g_{kl}. */
static void source_from_state(const geom *G, const state *s, double kappa, double *S)
{
    double T[4][4], Tuu[4][4], src[4];
    int mu, nu, k, l;
    stress_mixed(s, T);
    for (k = 0; k < 4; k++)
        for (l = 0; l < 4; l++) {
            Tuu[k][l] = 0.0;
            for (nu = 0; nu < 4; nu++)
                Tuu[k][l] += T[k][nu] * G->gi[nu][l];
        }
    for (mu = 0; mu < 4; mu++) {
        src[mu] = 0.0;
        for (k = 0; k < 4; k++)
            for (l = 0; l < 4; l++)
                src[mu] += Tuu[k][l] * G->dg[mu][k][l];
        src[mu] *= 0.5 * G->sqrtmg;
    }
    S[0] = 0.0;           /* rest mass: no source                       */
    S[1] = -src[0];       /* tau = -(T^t_t row) - (mass row)            */
    S[2] = src[1];
    S[3] = src[2];
    S[4] = src[3];
    S[5] = S[6] = S[7] = 0.0;
    S[8] = -kappa * s->phi;
}

/* ------------------------------------------------------------------------ */
/* Recovery of the primitives from the conserved variables (section 2.2: not
 * algebraic, solved with Newton-Raphson).  The unknown Wc = rho h W^2 is
 * solved for with v^2(Wc) eliminated through the momentum equation, and the
 * Newton steps are safeguarded by a bracket.  Inputs in the normal-observer
 * frame (Noble et al. 2006): D = rho W, Q_mu = alpha T^t_mu, Q.n, Qt^2,
 * Bc^i = alpha B^i.                                                         */

typedef struct {
    double D, Qn, Qt2, Bc2, QB, QB2, gamma;
} c2p_in;

static void c2p_v2(const c2p_in *c, double Wc, double *v2, double *dv2)
{
    double bw = c->Bc2 + Wc;
    double g = (c->Bc2 + 2.0 * Wc) / (bw * bw * Wc * Wc);
    *v2 = c->Qt2 / (bw * bw) + c->QB2 * g;
    *dv2 = -2.0 * c->Qt2 / (bw * bw * bw)
           + c->QB2 * g * (2.0 / (c->Bc2 + 2.0 * Wc) - 2.0 / bw - 2.0 / Wc);
}

/* energy residual f(Wc) and its derivative; requires v2(Wc) < 1 */
static double c2p_f(const c2p_in *c, double Wc, double *df)
{
    double v2, dv2, sq, k, p, dp;
    c2p_v2(c, Wc, &v2, &dv2);
    sq = sqrt(1.0 - v2);
    k = (c->gamma - 1.0) / c->gamma;
    p = k * (Wc * (1.0 - v2) - c->D * sq);
    dp = k * ((1.0 - v2) + (-Wc + c->D / (2.0 * sq)) * dv2);
    if (df)
        *df = -0.5 * c->Bc2 * dv2 - c->QB2 / (Wc * Wc * Wc) - 1.0 + dp;
    return -0.5 * c->Bc2 * (1.0 + v2) + c->QB2 / (2.0 * Wc * Wc) - Wc + p - c->Qn;
}

#define ORC_ATM_MARGIN 1e-10

static int isfin(double x)
{
    return isfinite(x);
}

/* returns 1 and fills P on success, 0 if no physical root was found */
static int c2p_solve(const geom *G, double gamma, const double *U, double *P)
{
    c2p_in c;
    double B[3], Bc[3], Q[3], Qu[3], Ttt, Tti[3];
    double lo, hi, v2, dv2, x, fx, dfx, W, Wc;
    int i, j, it;

    for (i = 0; i < 9; i++)
        if (!isfin(U[i]))
            return 0;
    if (!(U[0] > 0.0))
        return 0;

    for (i = 0; i < 3; i++) {
        B[i] = U[5 + i] / G->sqrtmg;
        Bc[i] = G->alpha * B[i];
        Q[i] = U[2 + i] / G->sqrtgamma;          /* alpha T^t_i          */
        Tti[i] = U[2 + i] / G->sqrtmg;
    }
    Ttt = -(U[1] + U[0]) / G->sqrtmg;
    c.D = U[0] / G->sqrtgamma;                   /* alpha rho u^t = rho W */
    c.Qn = Ttt;                                  /* Q_mu n^mu = T^t_t - beta^i T^t_i */
    for (i = 0; i < 3; i++)
        c.Qn -= G->beta[i] * Tti[i];
    c.Qt2 = 0.0;
    c.Bc2 = 0.0;
    c.QB = 0.0;
    for (i = 0; i < 3; i++) {
        Qu[i] = 0.0;
        for (j = 0; j < 3; j++) {
            Qu[i] += G->gami[i][j] * Q[j];
            c.Bc2 += G->gam[i][j] * Bc[i] * Bc[j];
        }
        c.QB += Q[i] * Bc[i];
    }
    for (i = 0; i < 3; i++)
        c.Qt2 += Qu[i] * Q[i];
    c.QB2 = c.QB * c.QB;
    c.gamma = gamma;

    /* lower end of the bracket: the smallest Wc with v^2(Wc) < 1 (v^2 falls
     * as Wc grows).  Roots below D (h W < 1) carry p < 0; they are accepted
     * and the pressure floor then applies. */
    lo = c.D;
    c2p_v2(&c, lo, &v2, &dv2);
    if (!(v2 < 1.0)) {
        double a = lo, b = 2.0 * lo;
        for (it = 0; it < 2100; it++) {
            c2p_v2(&c, b, &v2, &dv2);
            if (v2 < 1.0)
                break;
            a = b;
            b *= 2.0;
        }
        if (!(v2 < 1.0))
            return 0;
        for (it = 0; it < 200; it++) {
            double mid = 0.5 * (a + b);
            if (mid <= a || mid >= b)
                break;
            c2p_v2(&c, mid, &v2, &dv2);
            if (v2 < 1.0)
                b = mid;
            else
                a = mid;
        }
        lo = b;
    } else if (!(c2p_f(&c, lo, NULL) > 0.0)) {
        /* f decreases with Wc: a root exists only below D */
        double a = 0.5 * lo, b = lo;
        int found = 0;
        for (it = 0; it < 700; it++) {
            c2p_v2(&c, a, &v2, &dv2);
            if (!(v2 < 1.0)) {
                found = 1;
                break;
            }
            b = a;
            a *= 0.5;
        }
        if (found) {
            for (it = 0; it < 200; it++) {
                double mid = 0.5 * (a + b);
                if (mid <= a || mid >= b)
                    break;
                c2p_v2(&c, mid, &v2, &dv2);
                if (v2 < 1.0)
                    b = mid;
                else
                    a = mid;
            }
        }
        lo = b;
    }
    fx = c2p_f(&c, lo, NULL);
    if (!(fx > 0.0))
        return 0;
    /* upper end: f -> -Wc/Gamma as Wc grows */
    hi = 2.0 * lo;
    for (it = 0; it < 2100; it++) {
        if (c2p_f(&c, hi, NULL) < 0.0)
            break;
        lo = hi;
        hi *= 2.0;
    }
    if (!(c2p_f(&c, hi, NULL) < 0.0))
        return 0;

    /* safeguarded Newton inside [lo, hi] */
    x = 0.5 * (lo + hi);
    for (it = 0; it < 500; it++) {
        double xn;
        fx = c2p_f(&c, x, &dfx);
        if (fx == 0.0)
            break;
        if (fx > 0.0)
            lo = x;
        else
            hi = x;
        xn = x - fx / dfx;
        if (!(xn > lo && xn < hi))
            xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 1e-14 * x) {
            /* converged quadratically: one more Newton step reaches round-off */
            x = xn;
            fx = c2p_f(&c, x, &dfx);
            if (fx != 0.0) {
                xn = x - fx / dfx;
                if (xn > lo && xn < hi)
                    x = xn;
            }
            break;
        }
        if (hi - lo <= 4e-16 * hi) {
            x = xn;
            break;
        }
        x = xn;
    }
    Wc = x;
    c2p_v2(&c, Wc, &v2, &dv2);
    if (!(v2 >= 0.0 && v2 < 1.0) || !isfin(Wc))
        return 0;
    W = 1.0 / sqrt(1.0 - v2);
    P[0] = c.D / W;
    P[1] = (gamma - 1.0) / gamma * (Wc * (1.0 - v2) - c.D * sqrt(1.0 - v2));
    for (i = 0; i < 3; i++)
        P[2 + i] = W / (Wc + c.Bc2) * (Qu[i] + c.QB * Bc[i] / Wc);
    for (i = 0; i < 3; i++)
        P[5 + i] = B[i];
    P[8] = U[8];
    for (i = 0; i < 9; i++)
        if (!isfin(P[i]))
            return 0;
    return 1;
}

/* Recovery followed by the atmosphere / floor policy (not in the paper):
 *  failure             -> keep the guess (rho, p, u~);
 *  rho < (1 - 1e-10) rho_atm, or a failure where the guess has
 *  rho < 10 rho_atm    -> rho = rho_atm, p = p_atm, u~ = 0;
 *                         (the margin keeps cells that sit at the atmosphere
 *                          density from being reset back and forth by rounding)
 *  p < p_atm           -> p = p_atm;
 * B and Phi always come from U.  Wherever any of these fired, the matter part
 * of U (D, tau, S) is recomputed from the adjusted primitives.              */
static int c2p_cell(const geom *G, const orc_problem *pb, double *U, const double *Pg,
                    double *P)
{
    int flags = 0, i;
    if (!c2p_solve(G, pb->gamma, U, P)) {
        flags |= ORC_FLAG_FAIL;
        for (i = 0; i < 5; i++)
            P[i] = Pg[i];
        for (i = 0; i < 3; i++)
            P[5 + i] = U[5 + i] / G->sqrtmg;
        P[8] = U[8];
    }
    if (!(P[0] >= (1.0 - ORC_ATM_MARGIN) * pb->rho_atm)
        || ((flags & ORC_FLAG_FAIL) && Pg[0] < 10.0 * pb->rho_atm)) {
        flags |= ORC_FLAG_ATM;
        P[0] = pb->rho_atm;
        P[1] = pb->p_atm;
        P[2] = P[3] = P[4] = 0.0;
    }
    if (!(P[1] >= pb->p_atm)) {
        flags |= ORC_FLAG_PFLOOR;
        P[1] = pb->p_atm;
    }
    if (flags) {
        state s;
        double Un[9];
        state_from_prim(G, pb->gamma, P, &s);
        cons_from_state(G, &s, Un);
        for (i = 0; i < 5; i++)
            U[i] = Un[i];
    }
    return flags;
}

/* ------------------------------------------------------------------------ */
/* MC-limited TVD reconstruction (section 3.2): the slope of cell i is
 * minmod(2 dq-, (dq- + dq+)/2, 2 dq+); face values are q_i +- slope/2.      */

static double minmod3(double a, double b, double c)
{
    if (a > 0.0 && b > 0.0 && c > 0.0)
        return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0)
        return fmax(a, fmax(b, c));
    return 0.0;
}

double orc_mc_slope(double qm, double q0, double qp)
{
    return minmod3(2.0 * (q0 - qm), 0.5 * (qp - qm), 2.0 * (qp - q0));
}

/* PPM (the piecewise parabolic method of Colella & Woodward 1984; section 3.2
 * offers it beside MC) on cell i from the cells a[0..4] = i-2..i+2:
 * 1. the value at each of the cell's two interfaces is interpolated from the
 *    four nearest cells as the mean of its two neighbours minus one sixth of
 *    the difference of their MC-limited slopes (the fourth-order interface
 *    value of cell averages while the limiter is inactive);
 * 2. the parabola through the cell mean and these two edge values is then
 *    constrained to be monotone: at a local extremum of the cell means the
 *    reconstruction is flat (both edges = the mean); if the parabola would
 *    peak inside the cell, the edge nearer the peak is moved so that the
 *    extremum falls on the opposite edge (the edge becomes 3 a_i - 2 a_other).
 * No contact steepening and no shock flattening.                            */
void orc_ppm_edges(const double *a, double *aL, double *aR)
{
    double sm = orc_mc_slope(a[0], a[1], a[2]);   /* slope of cell i-1 */
    double s0 = orc_mc_slope(a[1], a[2], a[3]);   /* slope of cell i   */
    double sp = orc_mc_slope(a[2], a[3], a[4]);   /* slope of cell i+1 */
    double l = 0.5 * (a[1] + a[2]) - (s0 - sm) / 6.0;
    double r = 0.5 * (a[2] + a[3]) - (sp - s0) / 6.0;
    double q = a[2];
    if ((r - q) * (q - l) <= 0.0) {
        l = q;
        r = q;
    } else {
        double dlr = r - l;
        double m6 = 6.0 * (q - 0.5 * (l + r));
        if (dlr * m6 > dlr * dlr)
            l = 3.0 * q - 2.0 * r;
        else if (-dlr * dlr > dlr * m6)
            r = 3.0 * q - 2.0 * l;
    }
    *aL = l;
    *aR = r;
}

/* HLLE flux (Harten, Lax, van Leer, Einfeldt) at one face from the left and
 * right reconstructed primitives.  The normal field and Phi form a linear
 * 2x2 system that is solved exactly first; its state fixes the normal field
 * seen by both sides.                                                       */
static void face_flux(const geom *G, double gamma, double c_h, int ct, int dir, const double *qL_in,
                      const double *qR_in, double *F)
{
    double qL[9], qR[9], FL[9], FR[9], UL[9], UR[9];
    double BnL, BnR, Bs, phis, lmL, lpL, lmR, lpR, sl, sr;
    state sL, sR;
    int v;

    memcpy(qL, qL_in, sizeof qL);
    memcpy(qR, qR_in, sizeof qR);
    BnL = G->sqrtmg * qL[5 + dir];
    BnR = G->sqrtmg * qR[5 + dir];
    /* with constrained transport Phi plays no part: the normal field is the
     * mean of the two reconstructed ones (its flux is replaced later) */
    Bs = ct ? 0.5 * (BnL + BnR) : 0.5 * (BnL + BnR) - (qR[8] - qL[8]) / (2.0 * c_h);
    phis = 0.5 * (qL[8] + qR[8]) - 0.5 * c_h * (BnR - BnL);
    qL[5 + dir] = qR[5 + dir] = Bs / G->sqrtmg;

    state_from_prim(G, gamma, qL, &sL);
    state_from_prim(G, gamma, qR, &sR);
    flux_from_state(G, &sL, c_h, dir, FL);
    flux_from_state(G, &sR, c_h, dir, FR);
    cons_from_state(G, &sL, UL);
    cons_from_state(G, &sR, UR);
    speeds_from_state(G, &sL, gamma, dir, &lmL, &lpL);
    speeds_from_state(G, &sR, gamma, dir, &lmR, &lpR);
    sl = fmin(0.0, fmin(lmL, lmR));
    sr = fmax(0.0, fmax(lpL, lpR));

    for (v = 0; v < 8; v++) {
        if (v == 5 + dir)
            continue;
        if (sl == 0.0)
            F[v] = FL[v];
        else if (sr == 0.0)
            F[v] = FR[v];
        else
            F[v] = (sr * FL[v] - sl * FR[v] + sl * sr * (UR[v] - UL[v])) / (sr - sl);
    }
    F[5 + dir] = phis;
    F[8] = c_h * c_h * Bs;
}

/* ------------------------------------------------------------------------ */
/* Grid helpers */

static long long ncell(const orc_grid *g)
{
    return (long long)g->n[0] * g->n[1] * g->n[2];
}

static long long cidx(const orc_grid *g, int i, int j, int k)
{
    return ((long long)k * g->n[1] + j) * g->n[0] + i;
}

static int bc_map(int i, int n, int bc)
{
    if (i >= 0 && i < n)
        return i;
    if (bc == ORC_BC_PERIODIC)
        return ((i % n) + n) % n;
    return i < 0 ? 0 : n - 1;   /* zero-gradient outflow */
}

static double dxof(const orc_grid *g, int d)
{
    return (g->hi[d] - g->lo[d]) / g->n[d];
}

static double centre(const orc_grid *g, int d, int i)
{
    return g->lo[d] + (i + 0.5) * dxof(g, d);
}

static void load_prim(const orc_grid *g, const double *P, int i, int j, int k, double *q)
{
    long long N = ncell(g), c = cidx(g, i, j, k);
    int v;
    for (v = 0; v < 9; v++)
        q[v] = P[v * N + c];
}

/* ------------------------------------------------------------------------ */
/* Whole-grid operations */

int orc_prim2con(const orc_problem *pb, const double *P, double *U)
{
    const orc_grid *g = &pb->grid;
    long long N = ncell(g);
    int k;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (k = 0; k < g->n[2]; k++) {
        int i, j, v;
        for (j = 0; j < g->n[1]; j++)
            for (i = 0; i < g->n[0]; i++) {
                geom G;
                state s;
                double q[9], u[9];
                long long c = cidx(g, i, j, k);
                geom_cell(pb, i, j, k, &G);
                load_prim(g, P, i, j, k, q);
                state_from_prim(&G, pb->gamma, q, &s);
                cons_from_state(&G, &s, u);
                for (v = 0; v < 9; v++)
                    U[v * N + c] = u[v];
            }
    }
    return 0;
}

static int con2prim_grid(const orc_problem *pb, double *U, const double *Pg, double *P,
                         unsigned char *flags, orc_stats *st)
{
    const orc_grid *g = &pb->grid;
    long long N = ncell(g);
    long long nf = 0, na = 0, np = 0;
    int k;
#pragma omp parallel for num_threads(g_threads) schedule(static) reduction(+ : nf, na, np)
    for (k = 0; k < g->n[2]; k++) {
        int i, j, v, fl;
        for (j = 0; j < g->n[1]; j++)
            for (i = 0; i < g->n[0]; i++) {
                geom G;
                double u[9], pg[9], p[9];
                long long c = cidx(g, i, j, k);
                geom_cell(pb, i, j, k, &G);
                for (v = 0; v < 9; v++) {
                    u[v] = U[v * N + c];
                    pg[v] = Pg[v * N + c];
                }
                fl = c2p_cell(&G, pb, u, pg, p);
                for (v = 0; v < 9; v++) {
                    U[v * N + c] = u[v];
                    P[v * N + c] = p[v];
                }
                if (flags)
                    flags[c] = (unsigned char)fl;
                nf += (fl & ORC_FLAG_FAIL) != 0;
                na += (fl & ORC_FLAG_ATM) != 0;
                np += (fl & ORC_FLAG_PFLOOR) != 0;
            }
    }
    if (st) {
        st->fail += nf;
        st->atm += na;
        st->pfloor += np;
    }
    return 0;
}

int orc_con2prim(const orc_problem *pb, double *U, const double *Pguess, double *P,
                 unsigned char *flags, orc_stats *st)
{
    return con2prim_grid(pb, U, Pguess, P, flags, st);
}

/* Face index of direction dir at face/cell indices (i, j, k). */
static long long fidx(const orc_grid *g, int dir, int i, int j, int k)
{
    int nf0 = g->n[0] + (dir == 0), nf1 = g->n[1] + (dir == 1);
    return ((long long)k * nf1 + j) * nf0 + i;
}

/* Flux-CT (Toth 2000, the constrained-transport alternative to the cleaning
 * of section 3.2): for every pair (a, b) of active axes, the edge value
 *   W_ab = 1/4 [F^b(Bd^a) at the two b-faces beside the edge
 *               - F^a(Bd^b) at the two a-faces beside it]
 * (the electric field along the third axis, up to sign), from the original
 * fluxes; then F^a(Bd^b) = -1/2 (W_ab at the two edges of the a-face) and
 * F^b(Bd^a) = +1/2 (W_ab at the two edges of the b-face); the normal-field
 * and Phi fluxes vanish.  Face neighbours across a boundary map like cells.
 * The update then keeps the corner-centred divergence of Bd unchanged.   */
static int flux_ct(const orc_grid *g, double **F)
{
    int act[3], a, b;
    double *W[3][3] = {{NULL}};
    for (a = 0; a < 3; a++)
        act[a] = g->n[a] > 1;
    /* edge values from the original fluxes */
    for (a = 0; a < 3; a++)
        for (b = a + 1; b < 3; b++) {
            int e = 3 - a - b, fa, fb, ce;
            int na = g->n[a], nb = g->n[b], ne = g->n[e];
            long long NFa, NFb;
            if (!act[a] || !act[b])
                continue;
            NFa = (long long)(g->n[0] + (a == 0)) * (g->n[1] + (a == 1)) * (g->n[2] + (a == 2));
            NFb = (long long)(g->n[0] + (b == 0)) * (g->n[1] + (b == 1)) * (g->n[2] + (b == 2));
            W[a][b] = (double *)malloc(sizeof(double) * (size_t)(na + 1) * (nb + 1) * ne);
            if (!W[a][b])
                return -1;
            for (ce = 0; ce < ne; ce++)
                for (fb = 0; fb <= nb; fb++)
                    for (fa = 0; fa <= na; fa++) {
                        double s = 0.0;
                        int t;
                        for (t = 0; t < 2; t++) {
                            int ix[3], cb = bc_map(fb - 1 + t, nb, g->bc[b]), ca = bc_map(fa - 1 + t, na, g->bc[a]);
                            /* F^a(Bd^b) at a-face fa, cell cb along b */
                            ix[a] = fa;
                            ix[b] = cb;
                            ix[e] = ce;
                            s -= F[a][(5 + b) * NFa + fidx(g, a, ix[0], ix[1], ix[2])];
                            /* F^b(Bd^a) at b-face fb, cell ca along a */
                            ix[a] = ca;
                            ix[b] = fb;
                            s += F[b][(5 + a) * NFb + fidx(g, b, ix[0], ix[1], ix[2])];
                        }
                        W[a][b][((long long)ce * (nb + 1) + fb) * (na + 1) + fa] = 0.25 * s;
                    }
        }
    /* corrected fluxes */
    for (a = 0; a < 3; a++) {
        long long NFa, f;
        int i, j, k;
        if (!act[a])
            continue;
        NFa = (long long)(g->n[0] + (a == 0)) * (g->n[1] + (a == 1)) * (g->n[2] + (a == 2));
        for (k = 0; k < g->n[2] + (a == 2); k++)
            for (j = 0; j < g->n[1] + (a == 1); j++)
                for (i = 0; i < g->n[0] + (a == 0); i++) {
                    int ix[3] = {i, j, k}, b;
                    f = fidx(g, a, i, j, k);
                    F[a][(5 + a) * NFa + f] = 0.0;
                    F[a][8 * NFa + f] = 0.0;
                    for (b = 0; b < 3; b++) {
                        int lo = a < b ? a : b, hi = a < b ? b : a, e = 3 - a - b;
                        int nl = g->n[lo], nh = g->n[hi];
                        long long w0, w1;
                        double sign;
                        if (b == a || !act[b])
                            continue;
                        /* the face's two edges: the face index along a is fixed,
                         * the cell index along b gives edges b and b+1 */
                        {
                            int el[3], eh[3];
                            el[0] = ix[0];
                            el[1] = ix[1];
                            el[2] = ix[2];
                            eh[0] = ix[0];
                            eh[1] = ix[1];
                            eh[2] = ix[2];
                            eh[b] += 1;
                            w0 = ((long long)el[e] * (nh + 1) + el[hi]) * (nl + 1) + el[lo];
                            w1 = ((long long)eh[e] * (nh + 1) + eh[hi]) * (nl + 1) + eh[lo];
                        }
                        /* W is defined for (lo, hi) = (a, b) with sign +; for a > b
                         * the face is a b-face of the pair and takes +1/2 */
                        sign = a < b ? -0.5 : 0.5;
                        F[a][(5 + b) * NFa + f] = sign * (W[lo][hi][w0] + W[lo][hi][w1]);
                    }
                }
    }
    for (a = 0; a < 3; a++)
        for (b = 0; b < 3; b++)
            free(W[a][b]);
    return 0;
}

int orc_rhs(const orc_problem *pb, const double *P, double *R)
{
    const orc_grid *g = &pb->grid;
    long long N = ncell(g);
    double *Fall[3] = {NULL, NULL, NULL};
    int d;
    memset(R, 0, sizeof(double) * 9 * N);

    /* face fluxes of every active axis */
    for (d = 0; d < 3; d++) {
        int nf[3], k;
        long long NF;
        double *Fd;
        double dx = dxof(g, d);
        if (g->n[d] == 1)
            continue;
        nf[0] = g->n[0];
        nf[1] = g->n[1];
        nf[2] = g->n[2];
        nf[d] += 1;
        NF = (long long)nf[0] * nf[1] * nf[2];
        Fd = (double *)malloc(sizeof(double) * 9 * NF);
        if (!Fd) {
            for (k = 0; k < 3; k++)
                free(Fall[k]);
            return -1;
        }
        Fall[d] = Fd;

        /* face fluxes: face index f along d sits between cells f-1 and f */
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (k = 0; k < nf[2]; k++) {
            int i, j, v, s;
            for (j = 0; j < nf[1]; j++)
                for (i = 0; i < nf[0]; i++) {
                    int fi[3] = {i, j, k};
                    double q[6][9], qL[9], qR[9], F[9], pos[3];
                    geom G;
                    long long fc = ((long long)k * nf[1] + j) * nf[0] + i;
                    /* cells f-3 .. f+2 along d (boundary rule by index mapping) */
                    for (s = 0; s < 6; s++) {
                        int ci[3] = {i, j, k};
                        ci[d] = bc_map(fi[d] - 3 + s, g->n[d], g->bc[d]);
                        load_prim(g, P, ci[0], ci[1], ci[2], q[s]);
                    }
                    for (v = 0; v < 9; v++) {
                        if (pb->recon == ORC_RECON_PPM) {
                            /* left state: right edge of cell f-1; right state:
                             * left edge of cell f */
                            double a[5], e0, e1;
                            for (s = 0; s < 5; s++)
                                a[s] = q[s][v];
                            orc_ppm_edges(a, &e0, &qL[v]);
                            for (s = 0; s < 5; s++)
                                a[s] = q[s + 1][v];
                            orc_ppm_edges(a, &qR[v], &e1);
                            (void)e0;
                            (void)e1;
                        } else {
                            qL[v] = q[2][v] + 0.5 * orc_mc_slope(q[1][v], q[2][v], q[3][v]);
                            qR[v] = q[3][v] - 0.5 * orc_mc_slope(q[2][v], q[3][v], q[4][v]);
                        }
                    }
                    for (s = 0; s < 3; s++)
                        pos[s] = (s == d) ? g->lo[s] + fi[s] * dx : centre(g, s, fi[s]);
                    geom_face(pb, d, fi, pos, &G);
                    face_flux(&G, pb->gamma, pb->c_h, pb->ct, d, qL, qR, F);
                    for (v = 0; v < 9; v++)
                        Fd[v * NF + fc] = F[v];
                }
        }

    }

    if (pb->ct && flux_ct(g, Fall) != 0) {
        for (d = 0; d < 3; d++)
            free(Fall[d]);
        return -1;
    }

    /* flux differences */
    for (d = 0; d < 3; d++) {
        int nf[3], k;
        long long NF;
        const double *Fd = Fall[d];
        double dx = dxof(g, d);
        if (g->n[d] == 1)
            continue;
        nf[0] = g->n[0];
        nf[1] = g->n[1];
        nf[2] = g->n[2];
        nf[d] += 1;
        NF = (long long)nf[0] * nf[1] * nf[2];
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (k = 0; k < g->n[2]; k++) {
            int i, j, v;
            for (j = 0; j < g->n[1]; j++)
                for (i = 0; i < g->n[0]; i++) {
                    int lo_[3] = {i, j, k}, hi_[3] = {i, j, k};
                    long long c = cidx(g, i, j, k), fl, fh;
                    hi_[d] += 1;
                    fl = ((long long)lo_[2] * nf[1] + lo_[1]) * nf[0] + lo_[0];
                    fh = ((long long)hi_[2] * nf[1] + hi_[1]) * nf[0] + hi_[0];
                    for (v = 0; v < 9; v++)
                        R[v * N + c] -= (Fd[v * NF + fh] - Fd[v * NF + fl]) / dx;
                }
        }
    }
    for (d = 0; d < 3; d++)
        free(Fall[d]);

    /* cell-centred sources */
    {
        int k;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (k = 0; k < g->n[2]; k++) {
            int i, j, v;
            for (j = 0; j < g->n[1]; j++)
                for (i = 0; i < g->n[0]; i++) {
                    geom G;
                    state s;
                    double q[9], S[9];
                    long long c = cidx(g, i, j, k);
                    geom_cell(pb, i, j, k, &G);
                    load_prim(g, P, i, j, k, q);
                    state_from_prim(&G, pb->gamma, q, &s);
                    source_from_state(&G, &s, pb->kappa, S);
                    if (pb->ct)
                        S[8] = 0.0;   /* constrained transport: Phi is carried unchanged */
                    for (v = 0; v < 9; v++)
                        R[v * N + c] += S[v];
                }
        }
    }
    return 0;
}

/* SSP Runge-Kutta (Shu-Osher form): U^(s+1) = a U^n + b (U^(s) + dt L(U^(s)))
 * with a + b = 1, evaluated as U^(s) + a (U^n - U^(s)) + b dt L so that a
 * steady state (L = 0) is an exact fixed point in floating point. */
int orc_step(const orc_problem *pb, double *U, double *P, double dt, int nsteps,
             orc_stats *st)
{
    static const double rk3a[3] = {0.0, 0.75, 1.0 / 3.0};
    static const double rk3b[3] = {1.0, 0.25, 2.0 / 3.0};
    static const double rk2a[2] = {0.0, 0.5};
    static const double rk2b[2] = {1.0, 0.5};
    const double *a, *b;
    int nst, n, s;
    long long N = ncell(&pb->grid), c;
    double *Un, *R, *Pn;

    if (pb->rk_order == 3) {
        a = rk3a;
        b = rk3b;
        nst = 3;
    } else if (pb->rk_order == 2) {
        a = rk2a;
        b = rk2b;
        nst = 2;
    } else {
        return -1;
    }
    Un = (double *)malloc(sizeof(double) * 9 * N);
    R = (double *)malloc(sizeof(double) * 9 * N);
    Pn = (double *)malloc(sizeof(double) * 9 * N);
    if (!Un || !R || !Pn) {
        free(Un);
        free(R);
        free(Pn);
        return -1;
    }
    for (n = 0; n < nsteps; n++) {
        memcpy(Un, U, sizeof(double) * 9 * N);
        for (s = 0; s < nst; s++) {
            orc_rhs(pb, P, R);
            /* U holds U^(s); overwrite with U^(s+1) */
            for (c = 0; c < 9 * N; c++)
                U[c] = U[c] + a[s] * (Un[c] - U[c]) + b[s] * (dt * R[c]);
            memcpy(Pn, P, sizeof(double) * 9 * N);
            con2prim_grid(pb, U, Pn, P, NULL, st);
        }
    }
    free(Un);
    free(R);
    free(Pn);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Point functions for the pins */

void orc_point_geom(const orc_metric *m, double x, double y, double z, double *out)
{
    geom G;
    int a, b, c;
    geom_at(m, x, y, z, &G);
    out[0] = G.alpha;
    out[1] = G.sqrtgamma;
    out[2] = G.sqrtmg;
    for (a = 0; a < 4; a++)
        for (b = 0; b < 4; b++) {
            out[3 + 4 * a + b] = G.g[a][b];
            out[19 + 4 * a + b] = G.gi[a][b];
        }
    for (c = 0; c < 3; c++)
        for (a = 0; a < 4; a++)
            for (b = 0; b < 4; b++)
                out[35 + 16 * c + 4 * a + b] = G.dg[c + 1][a][b];
}

void orc_point_cons(const orc_metric *m, double gamma, double x, double y, double z,
                    const double *P, double *U)
{
    geom G;
    state s;
    geom_at(m, x, y, z, &G);
    state_from_prim(&G, gamma, P, &s);
    cons_from_state(&G, &s, U);
}

void orc_point_flux(const orc_metric *m, double gamma, double c_h, int dir, double x,
                    double y, double z, const double *P, double *F)
{
    geom G;
    state s;
    geom_at(m, x, y, z, &G);
    state_from_prim(&G, gamma, P, &s);
    flux_from_state(&G, &s, c_h, dir, F);
}

void orc_point_speeds(const orc_metric *m, double gamma, int dir, double x, double y,
                      double z, const double *P, double *lm, double *lp)
{
    geom G;
    state s;
    geom_at(m, x, y, z, &G);
    state_from_prim(&G, gamma, P, &s);
    speeds_from_state(&G, &s, gamma, dir, lm, lp);
}

void orc_point_stress(const orc_metric *m, double gamma, double x, double y, double z,
                      const double *P, double *T)
{
    geom G;
    state s;
    double t[4][4];
    int a, b;
    geom_at(m, x, y, z, &G);
    state_from_prim(&G, gamma, P, &s);
    stress_mixed(&s, t);
    for (a = 0; a < 4; a++)
        for (b = 0; b < 4; b++)
            T[4 * a + b] = t[a][b];
}

void orc_point_source(const orc_metric *m, double gamma, double kappa, double x, double y,
                      double z, const double *P, double *S)
{
    geom G;
    state s;
    geom_at(m, x, y, z, &G);
    state_from_prim(&G, gamma, P, &s);
    source_from_state(&G, &s, kappa, S);
}

int orc_point_c2p(const orc_metric *m, double gamma, double x, double y, double z,
                  const double *U, double *P)
{
    geom G;
    geom_at(m, x, y, z, &G);
    return c2p_solve(&G, gamma, U, P);
}

void orc_point_face_flux(const orc_metric *m, double gamma, double c_h, int dir, double x,
                         double y, double z, const double *qL, const double *qR, double *F)
{
    geom G;
    geom_at(m, x, y, z, &G);
    face_flux(&G, gamma, c_h, 0, dir, qL, qR, F);
}
