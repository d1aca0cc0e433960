/*
 * grmhd.h -- C ABI of the MI355X (gfx950) GRMHD substep library, libgrmhd.so.
 *
 * The library advances the equations of general-relativistic ideal MHD in a
 * fixed, given static spacetime (the Cowling setting of section 2.1 of
 * Zink, "HORIZON: Accelerated General Relativistic Magnetohydrodynamics",
 * arXiv:1102.5202) with the finite-volume method of section 2.2 and the scheme
 * choices of section 3.2: TVD reconstruction with the MC limiter, HLLE face
 * fluxes, the metric source terms of eq. 2, Newton-Raphson recovery of the
 * primitive variables, Runge-Kutta time integration, and hyperbolic
 * divergence cleaning of the constraint d_i(sqrt(-g) B^i) = 0.  Every step of
 * that update runs in hand-written HIP kernels on the device; the host only
 * enqueues launches.
 *
 * Variables (9 per cell, structure of arrays):
 *   primitives  P = (rho, p, u~x, u~y, u~z, Bx, By, Bz, Phi)
 *     u~^i = u^i + W beta^i / alpha  (the primitive velocity of the footnote
 *     in section 5.2), B^i = *F^{it} (eq. 2), Phi the cleaning scalar;
 *   conserved   U = (D, tau, Sx, Sy, Sz, Bdx, Bdy, Bdz, Phi)
 *     D = sqrt(-g) rho u^t,  tau = -sqrt(-g)(T^t_t + rho u^t),
 *     S_j = sqrt(-g) T^t_j,  Bd^j = sqrt(-g) B^j   (the conserved set of eq. 2,
 *     with the energy row written relative to the rest-mass row).
 *
 * Array layout: every P, U or R argument is a DEVICE pointer to 9*nz*ny*nx
 * doubles, index ((v*nz + k)*ny + j)*nx + i, interior cells only (no ghost
 * zones), 8-byte aligned.  Cell (i,j,k) has centre
 * lo + (i + 1/2, j + 1/2, k + 1/2) * (hi - lo)/n.  An axis with n = 1 is
 * switched off (no fluxes along it), which gives 1D and 2D problems.
 *
 * Ownership: the caller owns every buffer, the workspace and the stream.  The
 * library never allocates or frees device memory; all its scratch storage
 * lives in the caller's workspace.  Buffers must stay valid until the work
 * enqueued on the stream has completed.  One context serves one stream; a
 * context is not thread-safe.
 *
 * Errors: every call returns 0 on success or a negative grmhd_error code
 * (grmhd_strerror() describes it).  Enqueuing calls (cons, step, prim, rhs)
 * are asynchronous and never synchronise; a HIP launch error is reported by
 * the call that enqueued it.  Physical failures of the recovery (no physical
 * root, atmosphere resets, pressure floors) are not errors: they are counted
 * on the device and read with grmhd_status(), which synchronises.
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRMHD_NVAR 9

typedef enum {
    GRMHD_OK = 0,
    GRMHD_ERR_ARG = -1,        /* invalid argument (null pointer, bad size or option) */
    GRMHD_ERR_WORKSPACE = -2,  /* workspace missing or smaller than grmhd_workspace_bytes() */
    GRMHD_ERR_HIP = -3,        /* a HIP runtime call or kernel launch failed */
    GRMHD_ERR_STATE = -4,      /* call out of order (e.g. step before cons/prim) */
    GRMHD_ERR_NO_ADJOINT = -5  /* adjoint call on a context made without opts.adjoint (FP64) */
} grmhd_error;

typedef enum { GRMHD_METRIC_FLAT = 0, GRMHD_METRIC_ISO_SCHW = 1, GRMHD_METRIC_STORED = 2 } grmhd_metric_kind;
typedef enum { GRMHD_SOFT_SQRT = 0, GRMHD_SOFT_MAX = 1 } grmhd_soft_kind;
typedef enum { GRMHD_BC_PERIODIC = 0, GRMHD_BC_OUTFLOW = 1 } grmhd_bc_kind;
typedef enum { GRMHD_EOS_IDEAL = 0 } grmhd_eos_kind;
/* FP64: every step in double.  MIXED: the primitive caches, reconstruction,
 * face physics, HLLE fluxes and sources in float (the FP32 scheme of the paper,
 * section 3.2), with the metric evaluated in double and rounded once, and the
 * Runge-Kutta accumulation, the conserved variables and the primitive
 * recovery in double (the paper runs the recovery in double precision even in
 * single-precision runs, section 3.2).  User arrays are double in both. */
typedef enum { GRMHD_FP64 = 0, GRMHD_MIXED = 1 } grmhd_precision;

/* The fixed, given spacetime (section 2.1).  FLAT is Minkowski space.
 * ISO_SCHW is the Schwarzschild metric in isotropic coordinates, static and
 * without shift: alpha = (1 - M/(2 r_s))/(1 + M/(2 r_s)), gamma_ij = psi^4
 * delta_ij, psi = 1 + M/(2 r_s), with the radius softened near the origin:
 * r_s = sqrt(r^2 + r_min^2) (SQRT) or max(r, r_min) (MAX).  Requires
 * r_min > M/2 so that alpha > 0 everywhere.  STORED is any static,
 * conformally flat metric with zero shift given on the grid: its lapse and
 * psi^4 at the cell centres, set with grmhd_set_metric() (M, soft and r_min
 * are ignored). */
typedef struct {
    int kind;       /* grmhd_metric_kind */
    int soft;       /* grmhd_soft_kind   */
    double M;
    double r_min;
} grmhd_metric;

/* Cartesian uniform mesh (section 3.2).  n[d] >= 1 cells on [lo[d], hi[d]]
 * (at most 2^20 per axis and 2^38 in all); active axes (n > 1) need n >= 2
 * (n >= 3 with PPM).  bc[d] applies on both ends of axis d:
 * PERIODIC, or OUTFLOW (two zero-gradient ghost cells of the primitives). */
typedef struct {
    int n[3];
    double lo[3];
    double hi[3];
    int bc[3];
} grmhd_grid;

/* Ideal-gas equation of state p = (gamma - 1) rho eps (section 5.1). */
typedef struct {
    int kind;       /* grmhd_eos_kind (IDEAL only) */
    double gamma;   /* adiabatic index, 1 < gamma <= 2 */
    double K;       /* polytropic constant; used only to derive p_atm = K rho_atm^gamma
                       when opts.p_atm < 0 */
} grmhd_eos;

/* Primitive recovery (section 3.2 names a two-unknown and a one-unknown
 * scheme of Noble et al. 2006).  Both solve the same equations, warm-started
 * from the previous primitives, with the same acceptance test and the same
 * bracketed one-unknown fallback; they differ in the Newton iteration. */
typedef enum {
    GRMHD_RECOVERY_2D = 0,  /* Newton on (Wc = rho h W^2, v^2) */
    GRMHD_RECOVERY_1D = 1   /* Newton on Wc alone, v^2(Wc) eliminated */
} grmhd_recovery;

/* Reconstruction of the primitives at the faces (section 3.2 offers TVD with
 * the MC limiter and PPM).  PPM here is Colella & Woodward's interface
 * interpolation with MC-limited slopes and their monotonicity constraints
 * (no contact steepening, no flattening); it needs 3 cells on every active
 * axis, has no adjoint and no batched form, and 3D grids with it run the
 * face kernels of all three axes followed by the cell update (the fused
 * z-face + update kernel is MC only). */
typedef enum {
    GRMHD_RECON_MC = 0,
    GRMHD_RECON_PPM = 1
} grmhd_reconstruction;

/* Control of the divergence of the densitised field (section 3.2 names a
 * hyperbolic cleaning scheme): GLM-type cleaning with the scalar Phi, or
 * flux-CT (Toth 2000: every field flux replaced by the average of the edge
 * values -- the electric field -- built from the cleaning-free Godunov
 * fluxes of both face directions), which keeps the corner-centred
 * divergence sum_i d_i Bd^i unchanged to round-off in 3D.  With flux-CT Phi
 * is carried unchanged (no flux, no damping), the normal field at a face is
 * the mean of the two reconstructed ones, 3D grids run the face kernels of
 * all axes and the cell update (the fused kernel is cleaning only), and
 * there is no adjoint and no batched form. */
typedef enum {
    GRMHD_DIV_CLEANING = 0,
    GRMHD_DIV_FLUXCT = 1
} grmhd_divergence;

/* Scheme options and the caller's workspace. */
typedef struct {
    int rk_order;          /* 2 (SSP-RK2) or 3 (SSP-RK3, the order of section 3.2) */
    int precision;         /* grmhd_precision */
    double c_h;            /* cleaning speed, > 0 (1 if 0 is given) */
    double kappa;          /* cleaning damping rate, >= 0 */
    double rho_atm;        /* atmosphere density (absolute), > 0 */
    double p_atm;          /* atmosphere and floor pressure; < 0: K rho_atm^gamma */
    double newton_tol;     /* relative step tolerance of the recovery (1e-12 if 0) */
    int newton_maxit;      /* iteration cap of the recovery (50 if 0) */
    int recovery;          /* grmhd_recovery: the primitive recovery's Newton iteration */
    int reconstruction;    /* grmhd_reconstruction: MC (2 ghost layers) or PPM (3) */
    int divergence;        /* grmhd_divergence: hyperbolic cleaning or flux-CT */
    int timing;            /* nonzero: time every kernel launch with HIP events */
    int adjoint;           /* nonzero: reserve the workspace of the adjoint calls (FP64 only,
                              at most 2^30 cells) */
    int tape_steps;        /* with adjoint: slots of recorded steps (grmhd_step_record), 0..4096 */
    void *workspace;       /* device memory, >= grmhd_workspace_bytes(), 256-byte aligned */
    size_t workspace_bytes;
} grmhd_opts;

/* Device-side counters accumulated since the last reset. */
typedef struct {
    long long c2p_fail;     /* cells where the recovery found no physical root */
    long long atm_hits;     /* cells reset to the atmosphere */
    long long p_floor_hits; /* cells whose pressure was raised to p_atm */
    long long fallback_1d;  /* cells the 2D Newton iteration handed to the bracketed 1D solve */
    int max_newton_it;      /* most 2D Newton iterations any cell needed */
} grmhd_stats;

/* Kernel classes reported by grmhd_timing(). */
typedef enum {
    GRMHD_K_BC = 0,       /* ghost-zone fill of the primitive cache          */
    GRMHD_K_FLUX_X = 1,   /* reconstruction + face physics + HLLE, x faces   */
    GRMHD_K_FLUX_Y = 2,
    GRMHD_K_FLUX_Z = 3,
    GRMHD_K_UPDATE = 4,   /* flux divergence + sources + RK + recovery       */
    GRMHD_K_CONS = 5,     /* primitive -> conserved                          */
    GRMHD_K_PRIM = 6,     /* conserved -> primitive                          */
    GRMHD_K_RHS = 7,      /* flux divergence + sources only                  */
    GRMHD_K_ADJ_REC = 8,  /* adjoint: recovery + Runge-Kutta combination     */
    GRMHD_K_ADJ_FACE = 9, /* adjoint: face solver, one axis                  */
    GRMHD_K_ADJ_GATHER = 10, /* adjoint: reconstruction of all axes + ghost fold */
    GRMHD_K_ADJ_CELL = 11,   /* adjoint: sources + the next recovery + RK adjoint */
    GRMHD_K_CT = 12,      /* flux-CT: edge values and the corrected field fluxes */
    GRMHD_K_COUNT = 13
} grmhd_kernel;

typedef struct grmhd_ctx grmhd_ctx;

/* Bytes of device workspace a context needs for this grid and these options.
 * Returns 0 for an invalid grid or options that do not fit it (PPM on an
 * axis of fewer than 3 cells, an adjoint context of more than 2^30 cells). */
size_t grmhd_workspace_bytes(const grmhd_grid *grid, const grmhd_opts *opts);

/* Create a context (host-only; no device work, no allocation of device
 * memory).  The workspace in opts is carved into the ghosted primitive cache,
 * the stage buffer, the face-flux buffers and the counters.  *ctx is set on
 * success and must be released with grmhd_free().  The stream is the null
 * stream until grmhd_set_stream() is called. */
int grmhd_init(grmhd_ctx **ctx, const grmhd_metric *metric, const grmhd_grid *grid,
               const grmhd_eos *eos, const grmhd_opts *opts);

/* Set the HIP stream (a hipStream_t passed as void*) all later work is
 * enqueued on. */
int grmhd_set_stream(grmhd_ctx *ctx, void *stream);

/* Conserved variables from primitives, an algebraic map (section 2.2: the
 * evolution starts by converting the initial primitives).  P is read, U is
 * written (both device, layout above).  Also loads P into the context's
 * primitive cache, which seeds the next grmhd_step(). */
int grmhd_cons(grmhd_ctx *ctx, const double *P, double *U);

/* One full Runge-Kutta step of size dt (section 2.2: reconstruction, HLLE
 * fluxes, flux differences plus sources, Newton recovery, once per substep;
 * SSP-RK3 or SSP-RK2 per opts.rk_order), in place on the device array U.  The
 * primitives of U must be in the context's cache (set by grmhd_cons,
 * grmhd_prim or the previous grmhd_step).  Asynchronous; graph-capturable. */
int grmhd_step(grmhd_ctx *ctx, double *U, double dt);

/* The metric of a STORED context (section 2.1: the spacetime is given).
 * alpha and psi4 (device, double; read by work queued on the context's
 * stream, so they must stay valid until the stream reaches it) hold the lapse
 * and the conformal factor psi^4 (gamma_ij = psi^4 delta_ij, zero shift) at
 * the cell centres of the grid and of 2 ghost layers on every active axis:
 * dense [nz+2gz][ny+2gy][nx+2gx], x fastest, g = 2 on an axis with n > 1
 * and 0 otherwise; both must be positive (on a periodic axis the ghost
 * layers must repeat the opposite interior cells).  The library writes the
 * centre values, their fourth-order central differences along every active
 * axis (for the metric sources) and their fourth-order interpolation to
 * every face (for the fluxes) into buf, a caller-owned device buffer of
 * grmhd_metric_bytes(grid) bytes, 256-byte aligned, that must stay alive
 * while the context is used.  Must precede grmhd_cons, grmhd_prim,
 * grmhd_rhs and grmhd_step on a STORED context (GRMHD_ERR_STATE otherwise);
 * GRMHD_ERR_ARG on any other context, GRMHD_ERR_WORKSPACE for a buffer too
 * small or misaligned.  Asynchronous on the context's stream. */
size_t grmhd_metric_bytes(const grmhd_grid *grid);
int grmhd_set_metric(grmhd_ctx *ctx, const double *alpha, const double *psi4, void *buf, size_t buf_bytes);

/* Primitives from conserved variables by Newton-Raphson (section 2.2: the
 * inversion is not algebraic), followed by the atmosphere and floor policy.
 * U is read (never modified), P written; the context's cache, which provides
 * the Newton initial guess, is refreshed with P. */
int grmhd_prim(grmhd_ctx *ctx, const double *U, double *P);

/* Right-hand side L(P) = -sum_d (F_d(i+1/2) - F_d(i-1/2))/dx_d + s(P) of one
 * substep (compact form eq. 3) for the primitives P, written to R (device).
 * Loads P into the context's primitive cache, as grmhd_cons does. */
int grmhd_rhs(grmhd_ctx *ctx, const double *P, double *R);

/* ---- Without allocation --------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.
 * grmhd_rhs_noalloc computes what grmhd_init + grmhd_set_stream + grmhd_rhs
 * compute (the same kernels on the same inputs: R comes out bitwise the
 * same), with no context and no workspace: its scratch storage (the ghosted
 * primitive caches, the face fluxes and the counters) is a file-scope device
 * array of GRMHD_NOALLOC_SCRATCH_BYTES that every GPU the library runs on
 * holds until the process ends.  The call allocates nothing, on the device
 * or on the host.
 * Arguments as for grmhd_init (opts.workspace, timing, adjoint and
 * tape_steps are ignored; metric kind STORED, whose metric buffer the caller
 * would have to provide, is rejected with GRMHD_ERR_ARG) and grmhd_rhs (P
 * read, R written, device arrays [9][nz][ny][nx]); stream is the hipStream_t
 * (as void*) the work is enqueued on, asynchronously.  Returns
 * GRMHD_ERR_WORKSPACE when grmhd_workspace_bytes(grid, opts) exceeds
 * GRMHD_NOALLOC_SCRATCH_BYTES (64 MiB: a 3D grid of about 45^3 cells in FP64,
 * 55^3 in MIXED).  Every call on one GPU uses that GPU's one scratch array
 * and clears what must start at zero itself: calls on one stream follow each
 * other safely, calls that overlap on one GPU (other streams, other host
 * threads) race. */
#define GRMHD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int grmhd_rhs_noalloc(const grmhd_metric *metric, const grmhd_grid *grid, const grmhd_eos *eos,
                      const grmhd_opts *opts, const double *P, double *R, void *stream);

/* ---- Adjoint (reverse mode) of the discrete update, FP64 ----------------
 * The step is a map U^n -> U^(n+1) (with P^n the primitives of U^n).  The
 * adjoint calls return vector-Jacobian products of that map and of the
 * primitive/conserved conversions, for gradient-based inverse problems (the
 * source-parameter problems of section 1).  They need a context created with
 * opts.adjoint = 1 and precision FP64 (else GRMHD_ERR_NO_ADJOINT).
 * Derivatives follow the branch each limiter, min/max and upwind choice took;
 * the recovery is differentiated implicitly, dP/dU = (dU/dP)^-1 at the root;
 * floors hold their values constant and the rebuild of a floored cell's
 * conserved matter part is differentiated; a cell whose recovery failed keeps
 * its previous hydrodynamic primitives, which carry no derivative.  The
 * calls use only the adjoint part of the workspace: the forward state (the
 * primitive cache) is left as it was. */

/* Ubar <- (d U^(n+1) / d U^n)^T Ubar for one step of size dt from the state U
 * (device, read only; U's primitives are recovered first, then the step's
 * stages recomputed and reversed).  Ubar (device) is read and overwritten.
 * Recovery events of the recomputation are counted as in grmhd_step(). */
int grmhd_step_adjoint(grmhd_ctx *ctx, const double *U, double *Ubar, double dt);

/* A forward step exactly as grmhd_step (the same kernels on the same inputs:
 * U and the context's primitives come out bitwise the same) that also keeps,
 * in tape slot `slot` (0 <= slot < opts.tape_steps), what the reverse sweep
 * of this step needs: the primitives of the step's start and of every
 * stage's recovery, and the stages' floor flags.  A checkpointed reverse
 * sweep recomputes each segment once with these calls and then reverses the
 * recorded steps without recomputing them again.  The slot is overwritten;
 * its memory is part of the workspace ((rk_order + 1) ghosted FP64 primitive
 * arrays + rk_order bytes per cell per slot). */
int grmhd_step_record(grmhd_ctx *ctx, double *U, double dt, int slot);

/* Ubar <- (d U^(n+1) / d U^n)^T Ubar for the step recorded in tape slot
 * `slot` (its dt and stages as recorded; no recomputation).  Returns
 * GRMHD_ERR_STATE for a slot that was never recorded.  The result equals
 * grmhd_step_adjoint from the step's starting state up to the rounding of
 * the starting primitives (the recorded ones are those the forward step
 * used; grmhd_step_adjoint recovers them from U afresh). */
int grmhd_step_adjoint_recorded(grmhd_ctx *ctx, int slot, double *Ubar);

/* Pbar = (dU/dP)^T Ubar at the primitives P (the adjoint of grmhd_cons).
 * All device arrays; Pbar is written. */
int grmhd_cons_adjoint(grmhd_ctx *ctx, const double *P, const double *Ubar, double *Pbar);

/* Ubar = (dP/dU)^T Pbar = (dU/dP)^-T Pbar at the primitives of U, recovered
 * here (the adjoint of grmhd_prim).  All device arrays; Ubar is written. */
int grmhd_prim_adjoint(grmhd_ctx *ctx, const double *U, const double *Pbar, double *Ubar);

/* ---- Batched ensemble of independent 1D problems ------------------------
 * Many uneven 1D problems along x (flat metric, the equations and scheme of
 * the single-grid calls) advanced in ONE persistent kernel launch: one
 * workgroup per problem runs all of that problem's steps, the FP32 (mixed)
 * primitive row held in LDS when it fits.  Arrays are packed: problem b's
 * 9 x n_b values (variable-major, index 9*off_b + v*n_b + i with off_b the
 * sum of the earlier n) follow those of problem b-1; all device, double.
 * The same ownership and error rules as the single-grid calls apply. */
typedef struct {
    int nprob;             /* number of problems, 1 .. 2^20                     */
    const int *n;          /* host array: cells of each problem, 2 .. 2^24,
                              at most 2^38 over all problems                    */
    const double *lo;      /* host arrays: domain [lo, hi] of each problem      */
    const double *hi;
    const double *dt;      /* host array: time step of each problem             */
    const int *steps;      /* host array: steps each problem takes in all, >= 0 */
    int bc;                /* grmhd_bc_kind at both ends of every problem       */
} grmhd_batch_desc;

typedef struct grmhd_batch grmhd_batch;

/* Workspace bytes of a batch (opts: rk_order, precision; 0 if invalid). */
size_t grmhd_batch_workspace_bytes(const grmhd_batch_desc *desc, const grmhd_opts *opts);

/* Create a batch context (host only; the descriptor arrays are copied).
 * opts as for grmhd_init (its adjoint and timing fields are ignored). */
int grmhd_batch_init(grmhd_batch **b, const grmhd_batch_desc *desc, const grmhd_eos *eos,
                     const grmhd_opts *opts);

int grmhd_batch_set_stream(grmhd_batch *b, void *stream);

/* Conserved from primitives for every problem (packed arrays); loads the
 * primitive rows and resets every problem's step count to zero. */
int grmhd_batch_cons(grmhd_batch *b, const double *P, double *U);

/* Advance every problem by min(max_steps, steps left) steps of its own dt,
 * in place on U, in one launch.  Asynchronous. */
int grmhd_batch_evolve(grmhd_batch *b, double *U, int max_steps);

/* Primitives from conserved variables for every problem (packed). */
int grmhd_batch_prim(grmhd_batch *b, const double *U, double *P);

/* Time each launch shape (workgroup size; placement of the primitive rows)
 * on copies of the current state (U and the rows are left as they are), each
 * problem taking a share of trial_steps steps in proportion to the steps it
 * has left (the problem with the most left takes trial_steps), keep the
 * fastest for grmhd_batch_evolve, and report it in *threads and *lds (the
 * placement, as for grmhd_batch_set_shape) when not NULL.  Synchronises. */
int grmhd_batch_tune(grmhd_batch *b, const double *U, int trial_steps, int *threads, int *lds);

/* Choose the launch shape of grmhd_batch_evolve by hand: threads per
 * workgroup (256, 512 or 1024) and the placement lds of the primitive rows:
 * 0 one workgroup per problem, rows in HBM; 1 one workgroup per problem,
 * rows in LDS (refused with GRMHD_ERR_ARG when the largest row does not fit
 * in 160 KiB, or when the device refused that much LDS at grmhd_batch_init);
 * 2 (threads 256) the work (cells x steps) spread evenly over workgroups that
 * are all resident at once: a problem of more work than a workgroup's share
 * split into parts that exchange the cells beside their segments through
 * rows in HBM after each substep, smaller problems packed whole into shared
 * workgroups that run them one after another (refused where
 * grmhd_batch_init could not size the split for the device).  Rows in LDS are the initial choice wherever they are allowed.
 * grmhd_batch_evolve makes no call but its launches (one; two for the split:
 * the parts' progress counters are set from the step counts first), so it
 * can be captured in a HIP graph. */
int grmhd_batch_set_shape(grmhd_batch *b, int threads, int lds);

/* As grmhd_status, for the batch.  Returns GRMHD_ERR_STATE when a part of a
 * split launch stopped waiting for a neighbouring part (the parts were not
 * all resident at once, e.g. beside other work on the GPU); the state of the
 * problems is then not valid.  The counters are returned all the same. */
int grmhd_batch_status(grmhd_batch *b, grmhd_stats *st, int reset);

/* How busy the workgroup slots were during the last grmhd_batch_evolve
 * launch: every workgroup records its start and end on the GPU's
 * constant-rate clock, and *busy = (sum of the workgroups' durations) /
 * (S x the launch's span from the first start to the last end), with *slots
 * (may be NULL) = S = the workgroups the launch could hold resident at once
 * (its occupancy times the CUs, at most its workgroup count).  1 means every
 * slot worked until the last workgroup ended; an uneven ensemble on one
 * workgroup per problem shows the idle tail.  Synchronises the stream.
 * GRMHD_ERR_STATE before the first evolve call. */
int grmhd_batch_busy(grmhd_batch *b, double *busy, int *slots);

int grmhd_batch_free(grmhd_batch *b);

/* Copy the device counters to *st (synchronises the stream); reset them to 0
 * afterwards when reset != 0. */
int grmhd_status(grmhd_ctx *ctx, grmhd_stats *st, int reset);

/* With opts.timing set: synchronise, then report the summed duration (ms) and
 * the number of launches of each kernel class since the last reset, in arrays
 * of GRMHD_K_COUNT entries (either may be NULL). */
int grmhd_timing(grmhd_ctx *ctx, double *ms, long long *launches, int reset);

/* Release the context (host memory and HIP events only). */
int grmhd_free(grmhd_ctx *ctx);

/* For callers that check the library's compiled device arithmetic: on the
 * device arrays x, y (n doubles each), out[0..n) = x / y, out[n..2n) =
 * sqrt(x), out[2n..3n) = 1 / sqrt(x), evaluated as the kernels evaluate these
 * operations (FP64 division as a Newton-refined reciprocal times the
 * numerator; see the build flags), to be compared with correctly rounded
 * results.  out (3n doubles) is written, asynchronously on stream. */
int grmhd_device_arith(const double *x, const double *y, double *out, long long n, void *stream);

/* Static description of an error code. */
const char *grmhd_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
