/*
 * dugks3d.h -- C ABI of the three-dimensional T3S3-DUGKS sweep on MI355X
 * (gfx950): the step of dugks.h (paper section "Computational sequence of
 * the third-order DUGKS", steps (1)-(4), eq. feqIntD3rdHat2_DS) with a third
 * space axis, on a triply periodic box of uniform cells.  The paper states
 * its method for any dimension D (section "Kinetic model") and tests it in
 * two; here every step is the two-dimensional one with a third axis:
 *   - interface values (eq. interfaceEvof) from the quadratic expansion of
 *     eq. flux_DS about the upwind cell, with the three first, three second
 *     and three mixed central derivatives (the 19-point neighbourhood); a
 *     velocity parallel to a face takes the mean of the expansions about its
 *     two cells;
 *   - interface moments, equilibrium and recovery (eq. recover2f) at each
 *     face centre, the face relaxation time the mean of its two cells';
 *   - the micro-flux over the six faces (eq. microflux).
 *
 * Conventions are those of dugks.h: status codes (enum dugks_status,
 * dugks_strerror, dugks_last_error_message), precisions (enum
 * dugks_precision), memory kinds (enum dugks_mem).  Distribution arrays are
 * double [q][cell] with cell = (k ny + j) nx + i (x fastest); velocity fields
 * are double [3][cell].  The caller owns every buffer it passes.  All device
 * work is queued on the stream given at creation; functions that read into
 * host memory synchronise it.  A handle must not be used from two threads at
 * once.
 */
#ifndef DUGKS3D_H
#define DUGKS3D_H

#include "dugks.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dugks3d dugks3d_t;

/* Creation descriptor.  Pointers are host pointers, read only during
 * dugks3d_create. */
typedef struct {
    int nx, ny, nz;         /* cells per axis, each >= 3 */
    double lx, ly, lz;      /* box lengths (> 0); cells are uniform, every axis periodic */
    int nq;                 /* 19 or 27 discrete velocities (else DUGKS_ENOTSUP) */
    const double *xi;       /* [3][nq]: x, y and z components */
    const double *w;        /* [nq] equilibrium weights, Gaussian factor included:
                             * f^eq_q = w_q rho [1 + xi.u/RT + (xi.u)^2/(2RT^2) - u^2/(2RT)] */
    double RT;              /* > 0 */
    double dt;              /* > 0 */
    const double *tau;      /* [cell] per-cell relaxation time, or NULL for tau0 */
    double tau0;
    int precision;          /* dugks_precision */
    double rho0;            /* reference density of DUGKS_FP32_DELTA storage */
    double taylor_quad;     /* coefficient of the quadratic terms of eq. flux_DS:
                             * 1.0 as printed, 0.5 the Taylor polynomial; 0 selects 1.0 */
    void *stream;           /* hipStream_t, NULL = null stream */
} dugks3d_desc;

/* Build a solver.  Checks: n >= 3 per axis, lengths, dt, RT and tau > 0,
 * dt max|xi_a| <= the cell width along every axis a (CFL 1), rho0 > 0 for
 * DUGKS_FP32_DELTA,
 * dt/tau <= 12 (DUGKS_EUNSTABLE; the paper's stability bound at a = 1/3,
 * section "Time discretization"), sum w = 1, sum w xi = 0 and
 * sum w xi xi = RT I within 1e-10 (DUGKS_EMOMENT), nq in {19, 27}
 * (DUGKS_ENOTSUP).  On success *out owns four device arrays of nq x cells
 * values in the storage precision (the state, the transformed state of each
 * stage, the stage output) plus 9 doubles per cell (two sets of moments and
 * tau); the state is undefined until set_state or init_equilibrium. */
int dugks3d_create(const dugks3d_desc *d, dugks3d_t **out);

/* Release every resource of h; NULL is a no-op. */
int dugks3d_destroy(dugks3d_t *h);

/* State at t_n from the physical distribution f [q][cell]: the library keeps
 * fhat = f - (dt/4) Omega(f) (definitions under eq. feqIntD3rdHat2). */
int dugks3d_set_state(dugks3d_t *h, const double *f, int mem);

/* f = E(rho, u) in every cell; rho [cell], u [3][cell]. */
int dugks3d_init_equilibrium(dugks3d_t *h, const double *rho, const double *u, int mem);

/* Advance nsteps T3S3 steps (asynchronous on the stream): two kernels per
 * step, one per stage, each over tiles of 16 x 8 x 2 cells.  Velocity sets
 * equal to the library's D3Q19 or D3Q27 (xi = c e_q with e_q in the order of
 * cases.d3q27: q = 9 (ex+1) + 3 (ey+1) + (ez+1), D3Q19 the same order without
 * the eight corners; the standard weights) run kernels specialised at
 * compile time; any other set of 19 or 27 velocities runs kernels that read
 * the interface-expansion windows from tables.  Both give the oracle's
 * results to rounding.  There is no non-finite check (dugks_sync's flag is
 * for the two-dimensional sweep); dugks3d_moments shows a blown-up state. */
int dugks3d_step(dugks3d_t *h, int nsteps);

/* As dugks3d_step, with HIP events around every launch; synchronises and
 * returns the mean duration (ms) of the stage A and the stage C kernels
 * (either pointer may be NULL). */
int dugks3d_step_timed(dugks3d_t *h, int nsteps, double *ms_stage_a, double *ms_stage_c);

/* Cell density [cell] and velocity [3][cell] of the state (paper, section
 * "Discrete particle velocities": rho = sum f, rho u = sum xi f), taken of
 * fhat, whose moments equal those of f; NULL skips one output. */
int dugks3d_moments(dugks3d_t *h, double *rho, double *u, int mem);

/* The stored variable fhat [q][cell] in double. */
int dugks3d_get_fhat(dugks3d_t *h, double *fhat, int mem);

/* Physical distribution f = (4 tau fhat + dt E) / (4 tau + dt) [q][cell],
 * the inverse of fhat = f - (dt/4) Omega. */
int dugks3d_get_state(dugks3d_t *h, double *f, int mem);

#ifdef __cplusplus
}
#endif

#endif
