/*
 * dugks_oracle.c -- plain, slow, double-precision reference of one step of
 * the third-order discrete unified gas kinetic scheme (T3S3-DUGKS) of
 * Wu, Shu, Shi & Chen, "A third-order discrete unified gas kinetic scheme for
 * continuum and rarefied flows: low-speed isothermal case" (arXiv 1709.05458).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the HIP library is
 * checked against.  It shares no code with the library; only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it.  Nothing
 * in the product path may call it.
 *
 * Writing style: every quantity is computed the way the paper states it,
 * cell by cell and velocity by velocity, sums over q in ascending order, no
 * fusion and no algebraic re-arrangement beyond what the paper itself writes.
 *
 * Compiled twice: as `double` (liboracle.so) and, with -DORACLE_COMPLEX, as
 * `double complex` (liboracle_cs.so) so that complex-step derivatives of the
 * whole step can be taken; the step is analytic in f and tau because the
 * upwind choice depends only on the (real) particle velocity.
 *
 * Readings of the paper taken here (the paper is silent, ambiguous or
 * misprinted at these points):
 *  R1 (eq. f_tilde_1_3 / Step 2): the right-hand side 5/4*fbar^+ - 1/4*fhat
 *     already equals f + (dt/6)*Omega, i.e. the T2 post-collision variable
 *     tilde f^+ at t_n; the collision map of eq. ftp is NOT applied again.
 *     (`literal_ftilde` selects the other reading, for the pin tests.)
 *  R2 (eq. fbp_5_12): the coefficients are (24 tau - 5 dt)/(24 tau + 4 dt)
 *     and 9 dt/(24 tau + 4 dt), which map tilde f = f - (dt/6) Omega onto
 *     fbar^{+,5dt/12} = f + (5dt/24) Omega as eq. interfaceEvof requires.
 *     (`literal_fbp` selects the printed 24 tau + 10 dt form.)
 *  R3 (eq. flux_DS): the quadratic term is taken as printed, without the
 *     factor 1/2 of a Taylor polynomial (`literal_taylor`, the default of the
 *     Python wrapper); with the factor 1/2 the errors of the paper's
 *     convergence table are exceeded forty-fold at 32 cells, as printed they
 *     are matched within a factor of a few.  Both are available.
 *  R4 (eq. flux_DS, xi.n = 0): the face value is the mean of the expansions
 *     about the two adjacent cells.
 *  R5 (walls, boundary-condition section): the wall rule is applied to
 *     fbar at the wall face for the velocities leaving the wall; velocities
 *     arriving at (or parallel to) the wall are reconstructed from the
 *     interior cell; derivatives in wall-adjacent cells use the one-sided
 *     quadratic through the three nearest centres.  Bounce-back rho_w is the
 *     density of the adjacent cell at the base time of the stage.  Diffuse
 *     scattering: the sum over arriving velocities in the rho_w formula runs
 *     over the arriving interface values fbar.
 *  R6 (microflux, midpoint face rule): one quadrature point per face at its
 *     centre; cell values are point values at the cell centre.
 *  R7 (varying tau): the interface relaxation time is the mean of the two
 *     adjacent cells' values; at a wall, the interior cell's value.
 *  R8: the micro-flux carries the minus sign of L(f) = -xi . grad f.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORACLE_COMPLEX
#include <complex.h>
typedef double _Complex real;
#define OC(name) oc_cs_##name
#else
typedef double real;
#define OC(name) oc_##name
#endif

enum { BC_PERIODIC = 0, BC_BOUNCE_BACK = 1, BC_DIFFUSE = 2 };
enum { WEST = 0, EAST = 1, SOUTH = 2, NORTH = 3 };

typedef struct {
    int nx, ny, nq;
    const double *xf;   /* nx+1 face x-coordinates */
    const double *yf;   /* ny+1 face y-coordinates */
    const double *xi;   /* xi[q] = x-component, xi[nq+q] = y-component */
    const double *w;    /* equilibrium weights (Gaussian factor included) */
    const int *opp;     /* opp[q]: index of -xi_q (bounce-back only) */
    double RT;
    double dt;
    int bc[4];          /* west, east, south, north */
    double uw[4][2];    /* wall velocities */
    int literal_ftilde; /* pin-test switch, see R1 */
    int literal_fbp;    /* pin-test switch, see R2 */
    int literal_taylor; /* 1: expansion as printed (no 1/2), see R3 */
} oc_case;

#define XI(c, q) ((c)->xi[(q)])
#define ETA(c, q) ((c)->xi[(c)->nq + (q)])

/* ------------------------------------------------------------------------ */
/* Equilibrium and moments (paper eqs. for f^eq low-Mach form; rho = sum f, */
/* rho u = sum xi f in "Discrete particle velocities").                      */
/* ------------------------------------------------------------------------ */
static real equilibrium_q(const oc_case *c, int q, real rho, real ux, real uy)
{
    real eu = XI(c, q) * ux + ETA(c, q) * uy;
    real uu = ux * ux + uy * uy;
    double RT = c->RT;
    return c->w[q] * rho * (1.0 + eu / RT + eu * eu / (2.0 * RT * RT) - uu / (2.0 * RT));
}

/* moments of one cell's distribution, stride = distance between q planes */
static void moments(const oc_case *c, const real *f, long stride,
                    real *rho, real *ux, real *uy)
{
    real r = 0, mx = 0, my = 0;
    for (int q = 0; q < c->nq; q++) {
        real v = f[q * stride];
        r += v;
        mx += XI(c, q) * v;
        my += ETA(c, q) * v;
    }
    *rho = r;
    *ux = mx / r;
    *uy = my / r;
}

void OC(cell_moments)(const oc_case *c, const real *f, real *rho, real *ux, real *uy)
{
    long n = (long)c->nx * c->ny;
    for (long j = 0; j < n; j++) moments(c, f + j, n, rho + j, ux + j, uy + j);
}

void OC(equilibrium)(const oc_case *c, const real *rho, const real *ux,
                     const real *uy, real *f)
{
    long n = (long)c->nx * c->ny;
    for (int q = 0; q < c->nq; q++)
        for (long j = 0; j < n; j++)
            f[q * n + j] = equilibrium_q(c, q, rho[j], ux[j], uy[j]);
}

/* ------------------------------------------------------------------------ */
/* Geometry: cell centres (with the periodic image shift) and 3-point       */
/* derivative weights ("midpoint scheme" below eq. flux_DS).                 */
/* ------------------------------------------------------------------------ */
static double centre(const double *f, int n, int i)
{
    double L = f[n] - f[0];
    int k = i;
    double s = 0.0;
    while (k < 0) { k += n; s -= L; }
    while (k >= n) { k -= n; s += L; }
    return 0.5 * (f[k] + f[k + 1]) + s;
}

static int wrap(int i, int n)
{
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}

typedef struct {
    int off[3];      /* cell offsets of the 3 stencil points */
    double d1[3];    /* first-derivative weights at the cell centre */
    double d2[3];    /* second-derivative weights at the cell centre */
} stencil3;

/* Derivatives of the quadratic through three centres, evaluated at centre i.
 * Central (i-1, i, i+1) except next to a wall, where the three nearest
 * interior centres are used (reading R5). */
static stencil3 axis_stencil(const double *f, int n, int periodic, int i)
{
    stencil3 s;
    int o0 = -1;
    if (!periodic) {
        if (i == 0) o0 = 0;
        else if (i == n - 1) o0 = -2;
    }
    double p[3];
    double xc = centre(f, n, i);
    for (int k = 0; k < 3; k++) {
        s.off[k] = o0 + k;
        p[k] = centre(f, n, i + o0 + k) - xc;
    }
    for (int k = 0; k < 3; k++) {
        int a = (k + 1) % 3, b = (k + 2) % 3;
        double den = (p[k] - p[a]) * (p[k] - p[b]);
        s.d1[k] = -(p[a] + p[b]) / den;
        s.d2[k] = 2.0 / den;
    }
    return s;
}

/* Value at (cell (iu,ju)) + (dx,dy) of the quadratic Taylor polynomial built
 * from the 3x3 derivative stencil of plane B (eq. flux_DS with reading R3). */
static real expand(const oc_case *c, const real *B, int iu, int ju,
                   double dx, double dy)
{
    int nx = c->nx, ny = c->ny;
    int px = c->bc[WEST] == BC_PERIODIC, py = c->bc[SOUTH] == BC_PERIODIC;
    stencil3 sx = axis_stencil(c->xf, nx, px, iu);
    stencil3 sy = axis_stencil(c->yf, ny, py, ju);
    real Bx = 0, Bxx = 0, By = 0, Byy = 0, Bxy = 0;
    for (int k = 0; k < 3; k++) {
        real v = B[(long)ju * nx + wrap(iu + sx.off[k], nx)];
        Bx += sx.d1[k] * v;
        Bxx += sx.d2[k] * v;
    }
    for (int k = 0; k < 3; k++) {
        real v = B[(long)wrap(ju + sy.off[k], ny) * nx + iu];
        By += sy.d1[k] * v;
        Byy += sy.d2[k] * v;
    }
    for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++)
            Bxy += sx.d1[k] * sy.d1[l] *
                   B[(long)wrap(ju + sy.off[l], ny) * nx + wrap(iu + sx.off[k], nx)];
    real B0 = B[(long)ju * nx + iu];
    double half = c->literal_taylor ? 1.0 : 0.5;
    return B0 + dx * Bx + dy * By + half * (dx * dx * Bxx + 2.0 * dx * dy * Bxy + dy * dy * Byy);
}

/* ------------------------------------------------------------------------ */
/* Interface values fbar(x_b, t+h) = fbar^+(x_b - xi h, t) (eq.             */
/* interfaceEvof) from the plane B = fbar^+ at cell centres, plus walls.     */
/* fx: [nq][ny][nx+1] x-faces, fy: [nq][ny+1][nx] y-faces.                   */
/* rho_cell: density of the stage input in each cell (bounce-back rho_w).    */
/* ------------------------------------------------------------------------ */
static void wall_face(const oc_case *c, int side, real *fb /* stride nfaces */,
                      long stride, real rho_adj)
{
    /* outward unit normal of the fluid domain at this wall */
    double nxw = side == WEST ? -1.0 : side == EAST ? 1.0 : 0.0;
    double nyw = side == SOUTH ? -1.0 : side == NORTH ? 1.0 : 0.0;
    double ux = c->uw[side][0], uy = c->uw[side][1];
    int kind = c->bc[side];
    if (kind == BC_BOUNCE_BACK) {
        /* eq. BB: leaving velocities (xi.n < 0) from their mirrors */
        for (int q = 0; q < c->nq; q++) {
            double xn = XI(c, q) * nxw + ETA(c, q) * nyw;
            if (xn < 0.0) {
                int o = c->opp[q];
                fb[q * stride] = fb[o * stride] +
                    2.0 * rho_adj * c->w[q] * (XI(c, q) * ux + ETA(c, q) * uy) / c->RT;
            }
        }
    } else if (kind == BC_DIFFUSE) {
        /* diffuse scattering: leaving velocities are E(rho_w, u_w) with rho_w
         * from zero net mass flux through the wall */
        real num = 0;
        double den = 0.0;
        for (int q = 0; q < c->nq; q++) {
            double xn = XI(c, q) * nxw + ETA(c, q) * nyw;
            if (xn > 0.0) num += xn * fb[q * stride];
        }
        for (int q = 0; q < c->nq; q++) {
            double xn = XI(c, q) * nxw + ETA(c, q) * nyw;
            if (xn < 0.0) {
                double eu = XI(c, q) * ux + ETA(c, q) * uy;
                double uu = ux * ux + uy * uy;
                double e1 = c->w[q] * (1.0 + eu / c->RT + eu * eu / (2.0 * c->RT * c->RT) -
                                       uu / (2.0 * c->RT));
                den += -xn * e1;
            }
        }
        real rw = num / den;
        for (int q = 0; q < c->nq; q++) {
            double xn = XI(c, q) * nxw + ETA(c, q) * nyw;
            if (xn < 0.0) fb[q * stride] = equilibrium_q(c, q, rw, ux, uy);
        }
    }
}

void OC(face_values)(const oc_case *c, const real *B, const real *rho_cell,
                     double h, real *fx, real *fy)
{
    int nx = c->nx, ny = c->ny, nq = c->nq;
    long ncell = (long)nx * ny;
    long nfx = (long)ny * (nx + 1), nfy = (long)(ny + 1) * nx;
    int perx = c->bc[WEST] == BC_PERIODIC, pery = c->bc[SOUTH] == BC_PERIODIC;

    /* x-faces */
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++) {
        double yb = centre(c->yf, ny, j);
        for (int fi = 0; fi <= nx; fi++) {
            double xb = c->xf[fi];
            int wallW = (fi == 0 && !perx), wallE = (fi == nx && !perx);
            long fidx = (long)j * (nx + 1) + fi;
            if (perx && fi == nx) {   /* same face as fi = 0 */
                for (int q = 0; q < nq; q++)
                    fx[q * nfx + fidx] = fx[q * nfx + (long)j * (nx + 1)];
                continue;
            }
            for (int q = 0; q < nq; q++) {
                const real *Bq = B + q * ncell;
                double ex = XI(c, q), ey = ETA(c, q);
                double dy = -ey * h;   /* face centre and upwind centre share y */
                real v;
                if (wallW) {
                    if (ex > 0.0) continue;   /* leaving: set by the wall rule */
                    v = expand(c, Bq, 0, j, xb - ex * h - centre(c->xf, nx, 0), dy);
                } else if (wallE) {
                    if (ex < 0.0) continue;
                    v = expand(c, Bq, nx - 1, j, xb - ex * h - centre(c->xf, nx, nx - 1), dy);
                } else {
                    int iL = fi - 1, iR = fi;
                    if (ex > 0.0) {
                        v = expand(c, Bq, wrap(iL, nx), j, xb - ex * h - centre(c->xf, nx, iL), dy);
                    } else if (ex < 0.0) {
                        v = expand(c, Bq, wrap(iR, nx), j, xb - ex * h - centre(c->xf, nx, iR), dy);
                    } else {
                        real vL = expand(c, Bq, wrap(iL, nx), j, xb - centre(c->xf, nx, iL), dy);
                        real vR = expand(c, Bq, wrap(iR, nx), j, xb - centre(c->xf, nx, iR), dy);
                        v = 0.5 * (vL + vR);
                    }
                }
                fx[q * nfx + fidx] = v;
            }
            if (wallW) wall_face(c, WEST, fx + fidx, nfx, rho_cell[(long)j * nx]);
            if (wallE) wall_face(c, EAST, fx + fidx, nfx, rho_cell[(long)j * nx + nx - 1]);
        }
    }

    /* y-faces */
    #pragma omp parallel for schedule(static)
    for (int fj = 0; fj <= ny; fj++) {
        double yb = c->yf[fj];
        int wallS = (fj == 0 && !pery), wallN = (fj == ny && !pery);
        for (int i = 0; i < nx; i++) {
            double xb = centre(c->xf, nx, i);
            long fidx = (long)fj * nx + i;
            if (pery && fj == ny) continue;   /* copied from fj = 0 below */
            for (int q = 0; q < nq; q++) {
                const real *Bq = B + q * ncell;
                double ex = XI(c, q), ey = ETA(c, q);
                double dx = -ex * h;   /* face centre and upwind centre share x */
                real v;
                if (wallS) {
                    if (ey > 0.0) continue;
                    v = expand(c, Bq, i, 0, dx, yb - ey * h - centre(c->yf, ny, 0));
                } else if (wallN) {
                    if (ey < 0.0) continue;
                    v = expand(c, Bq, i, ny - 1, dx, yb - ey * h - centre(c->yf, ny, ny - 1));
                } else {
                    int jS = fj - 1, jN = fj;
                    if (ey > 0.0) {
                        v = expand(c, Bq, i, wrap(jS, ny), dx, yb - ey * h - centre(c->yf, ny, jS));
                    } else if (ey < 0.0) {
                        v = expand(c, Bq, i, wrap(jN, ny), dx, yb - ey * h - centre(c->yf, ny, jN));
                    } else {
                        real vS = expand(c, Bq, i, wrap(jS, ny), dx, yb - centre(c->yf, ny, jS));
                        real vN = expand(c, Bq, i, wrap(jN, ny), dx, yb - centre(c->yf, ny, jN));
                        v = 0.5 * (vS + vN);
                    }
                }
                fy[q * nfy + fidx] = v;
            }
            if (wallS) wall_face(c, SOUTH, fy + fidx, nfy, rho_cell[i]);
            if (wallN) wall_face(c, NORTH, fy + fidx, nfy, rho_cell[(long)(ny - 1) * nx + i]);
        }
    }
    if (pery)   /* face ny is face 0 */
        for (int q = 0; q < nq; q++)
            for (int i = 0; i < nx; i++)
                fy[q * nfy + (long)ny * nx + i] = fy[q * nfy + i];
}

/* ------------------------------------------------------------------------ */
/* Micro-flux L_j (eq. microflux, midpoint face rule, sign of R8) from the   */
/* interface values: face moments -> E_b -> f_b (eq. recover2f) -> L.        */
/* ------------------------------------------------------------------------ */
static void recover_faces(const oc_case *c, real *fb, long nf, long face,
                          real tau_b, double h)
{
    real rho, ux, uy;
    moments(c, fb + face, nf, &rho, &ux, &uy);
    for (int q = 0; q < c->nq; q++) {
        real e = equilibrium_q(c, q, rho, ux, uy);
        fb[q * nf + face] = (2.0 * tau_b * fb[q * nf + face] + h * e) / (2.0 * tau_b + h);
    }
}

int OC(flux)(const oc_case *c, const real *tau, const real *B,
             const real *rho_cell, double h, real *L)
{
    int nx = c->nx, ny = c->ny, nq = c->nq;
    long ncell = (long)nx * ny;
    long nfx = (long)ny * (nx + 1), nfy = (long)(ny + 1) * nx;
    int perx = c->bc[WEST] == BC_PERIODIC, pery = c->bc[SOUTH] == BC_PERIODIC;
    real *fx = (real *)malloc(sizeof(real) * nq * nfx);
    real *fy = (real *)malloc(sizeof(real) * nq * nfy);
    if (!fx || !fy) { free(fx); free(fy); return -1; }

    OC(face_values)(c, B, rho_cell, h, fx, fy);

    #pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int fi = 0; fi <= nx; fi++) {
            real tb;
            if (fi == 0 && !perx) tb = tau[(long)j * nx];
            else if (fi == nx && !perx) tb = tau[(long)j * nx + nx - 1];
            else tb = 0.5 * (tau[(long)j * nx + wrap(fi - 1, nx)] + tau[(long)j * nx + wrap(fi, nx)]);
            recover_faces(c, fx, nfx, (long)j * (nx + 1) + fi, tb, h);
        }
    #pragma omp parallel for schedule(static)
    for (int fj = 0; fj <= ny; fj++)
        for (int i = 0; i < nx; i++) {
            real tb;
            if (fj == 0 && !pery) tb = tau[i];
            else if (fj == ny && !pery) tb = tau[(long)(ny - 1) * nx + i];
            else tb = 0.5 * (tau[(long)wrap(fj - 1, ny) * nx + i] + tau[(long)wrap(fj, ny) * nx + i]);
            recover_faces(c, fy, nfy, (long)fj * nx + i, tb, h);
        }

    /* L_j = -(1/|V_j|) sum_faces (xi . n) |A| f_b */
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            double dx = c->xf[i + 1] - c->xf[i];
            double dy = c->yf[j + 1] - c->yf[j];
            double vol = dx * dy;
            for (int q = 0; q < nq; q++) {
                real fw = fx[q * nfx + (long)j * (nx + 1) + i];
                real fe = fx[q * nfx + (long)j * (nx + 1) + i + 1];
                real fs = fy[q * nfy + (long)j * nx + i];
                real fn = fy[q * nfy + (long)(j + 1) * nx + i];
                real flux = XI(c, q) * dy * (fe - fw) + ETA(c, q) * dx * (fn - fs);
                L[q * ncell + (long)j * nx + i] = -flux / vol;
            }
        }
    free(fx);
    free(fy);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One T3S3 step, steps (1)-(4) of "Computational sequence of the           */
/* third-order DUGKS", eq. feqIntD3rdHat2_DS.  State: fhat = f - dt/4 Omega. */
/* ------------------------------------------------------------------------ */
int OC(t3s3_step)(const oc_case *c, const real *tau, const real *fhat, real *out)
{
    int nq = c->nq;
    long n = (long)c->nx * c->ny;
    double dt = c->dt;
    size_t qs = sizeof(real) * nq * n, cs = sizeof(real) * n;
    real *E = malloc(qs), *B = malloc(qs), *Ls = malloc(qs), *G = malloc(qs);
    real *W = malloc(qs), *Bp = malloc(qs), *Lss = malloc(qs), *Ep = malloc(qs);
    real *rho = malloc(cs), *ux = malloc(cs), *uy = malloc(cs);
    real *rhop = malloc(cs), *uxp = malloc(cs), *uyp = malloc(cs);
    int rc = 0;
    if (!E || !B || !Ls || !G || !W || !Bp || !Lss || !Ep || !rho || !ux || !uy ||
        !rhop || !uxp || !uyp) { rc = -1; goto done; }

    /* moments and equilibrium at t_n (collision invariants of fhat) */
    OC(cell_moments)(c, fhat, rho, ux, uy);
    OC(equilibrium)(c, rho, ux, uy, E);

    /* Step 1: fbar^{+,dt/6}(t_n) by eq. f_bar_1_6, then L* at t* = t_n + dt/6 */
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            real t = tau[j];
            B[q * n + j] = (12.0 * t - dt) / (12.0 * t + 3.0 * dt) * fhat[q * n + j] +
                           4.0 * dt / (12.0 * t + 3.0 * dt) * E[q * n + j];
        }
    if ((rc = OC(flux)(c, tau, B, rho, dt / 6.0, Ls))) goto done;

    /* Step 2: T2 sub-step of dt/3 to t' = t_n + dt/3 (R1), then dt*Omega(t')
     * by eq. collisionterm */
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            real tt = 1.25 * B[q * n + j] - 0.25 * fhat[q * n + j];   /* eq. f_tilde_1_3 */
            if (c->literal_ftilde) {
                real t = tau[j];
                tt = (6.0 * t - dt) / (6.0 * t + dt) * tt + 2.0 * dt / (6.0 * t + dt) * E[q * n + j];
            }
            G[q * n + j] = tt + dt / 3.0 * Ls[q * n + j];           /* tilde f(t') */
        }
    OC(cell_moments)(c, G, rhop, uxp, uyp);
    OC(equilibrium)(c, rhop, uxp, uyp, Ep);
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            real t = tau[j];
            W[q * n + j] = -6.0 * dt / (6.0 * t + dt) * (G[q * n + j] - Ep[q * n + j]);
        }

    /* Step 3: fbar^{+,5dt/12}(t') by eq. fbp_5_12 (R2), then L** at
     * t** = t_n + 3dt/4 */
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            real t = tau[j];
            real a, b;
            if (c->literal_fbp) {
                a = (24.0 * t - 5.0 * dt) / (24.0 * t + 10.0 * dt);
                b = 15.0 * dt / (24.0 * t + 10.0 * dt);
            } else {
                a = (24.0 * t - 5.0 * dt) / (24.0 * t + 4.0 * dt);
                b = 9.0 * dt / (24.0 * t + 4.0 * dt);
            }
            Bp[q * n + j] = a * G[q * n + j] + b * Ep[q * n + j];
        }
    if ((rc = OC(flux)(c, tau, Bp, rhop, 5.0 * dt / 12.0, Lss))) goto done;

    /* Step 4: fhat^+ = fhat/4 + 3/4 fbar^{+,dt/6} (eq. fhp), then
     * eq. feqIntD3rdHat2_DS */
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            long k = q * n + j;
            real fhp = 0.25 * fhat[k] + 0.75 * B[k];
            out[k] = fhp + 0.75 * W[k] + dt / 7.0 * (3.0 * Ls[k] + 4.0 * Lss[k]);
        }
done:
    free(E); free(B); free(Ls); free(G); free(W); free(Bp); free(Lss); free(Ep);
    free(rho); free(ux); free(uy); free(rhop); free(uxp); free(uyp);
    return rc;
}

/* Stage-A product of one step (tilde f at t'), exposed for the tests. */
int OC(t3s3_stage_a)(const oc_case *c, const real *tau, const real *fhat, real *G)
{
    int nq = c->nq;
    long n = (long)c->nx * c->ny;
    double dt = c->dt;
    size_t qs = sizeof(real) * nq * n, cs = sizeof(real) * n;
    real *E = malloc(qs), *B = malloc(qs), *Ls = malloc(qs);
    real *rho = malloc(cs), *ux = malloc(cs), *uy = malloc(cs);
    int rc = 0;
    if (!E || !B || !Ls || !rho || !ux || !uy) { rc = -1; goto done; }
    OC(cell_moments)(c, fhat, rho, ux, uy);
    OC(equilibrium)(c, rho, ux, uy, E);
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            real t = tau[j];
            B[q * n + j] = (12.0 * t - dt) / (12.0 * t + 3.0 * dt) * fhat[q * n + j] +
                           4.0 * dt / (12.0 * t + 3.0 * dt) * E[q * n + j];
        }
    if ((rc = OC(flux)(c, tau, B, rho, dt / 6.0, Ls))) goto done;
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++)
            G[q * n + j] = 1.25 * B[q * n + j] - 0.25 * fhat[q * n + j] + dt / 3.0 * Ls[q * n + j];
done:
    free(E); free(B); free(Ls); free(rho); free(ux); free(uy);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Independent second-order integrator (Remark I, eq.                      */
/* feqIntD2nd_Explicit with the full step delta on the flux): state         */
/* tilde f = f - delta/2 Omega, reconstruction over h = delta/2.            */
/* ------------------------------------------------------------------------ */
int OC(t2_step)(const oc_case *c, const real *tau, double delta,
                const real *ft, real *out)
{
    int nq = c->nq;
    long n = (long)c->nx * c->ny;
    size_t qs = sizeof(real) * nq * n, cs = sizeof(real) * n;
    real *E = malloc(qs), *Fb = malloc(qs), *L = malloc(qs);
    real *rho = malloc(cs), *ux = malloc(cs), *uy = malloc(cs);
    int rc = 0;
    if (!E || !Fb || !L || !rho || !ux || !uy) { rc = -1; goto done; }
    OC(cell_moments)(c, ft, rho, ux, uy);
    OC(equilibrium)(c, rho, ux, uy, E);
    /* fbar^{+,h} at h = delta/2 from tilde f:  ((4 tau - delta) ft + 3 delta E) / (4 tau + 2 delta) */
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            real t = tau[j];
            Fb[q * n + j] = ((4.0 * t - delta) * ft[q * n + j] + 3.0 * delta * E[q * n + j]) /
                            (4.0 * t + 2.0 * delta);
        }
    if ((rc = OC(flux)(c, tau, Fb, rho, 0.5 * delta, L))) goto done;
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            real t = tau[j];
            real ftp = (2.0 * t - delta) / (2.0 * t + delta) * ft[q * n + j] +
                       2.0 * delta / (2.0 * t + delta) * E[q * n + j];
            out[q * n + j] = ftp + delta * L[q * n + j];
        }
done:
    free(E); free(Fb); free(L); free(rho); free(ux); free(uy);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Variable changes: fhat = f - (dt/4) Omega(f) and its inverse            */
/* (eq. feqIntD3rdHat2 definitions; eq. for fhat^+).                         */
/* ------------------------------------------------------------------------ */
int OC(f_to_fhat)(const oc_case *c, const real *tau, const real *f, real *fhat)
{
    long n = (long)c->nx * c->ny;
    real *rho = malloc(sizeof(real) * n), *ux = malloc(sizeof(real) * n),
         *uy = malloc(sizeof(real) * n);
    if (!rho || !ux || !uy) { free(rho); free(ux); free(uy); return -1; }
    OC(cell_moments)(c, f, rho, ux, uy);
    for (int q = 0; q < c->nq; q++)
        for (long j = 0; j < n; j++) {
            real e = equilibrium_q(c, q, rho[j], ux[j], uy[j]);
            fhat[q * n + j] = f[q * n + j] + c->dt / (4.0 * tau[j]) * (f[q * n + j] - e);
        }
    free(rho); free(ux); free(uy);
    return 0;
}

int OC(fhat_to_f)(const oc_case *c, const real *tau, const real *fhat, real *f)
{
    long n = (long)c->nx * c->ny;
    real *rho = malloc(sizeof(real) * n), *ux = malloc(sizeof(real) * n),
         *uy = malloc(sizeof(real) * n);
    if (!rho || !ux || !uy) { free(rho); free(ux); free(uy); return -1; }
    OC(cell_moments)(c, fhat, rho, ux, uy);
    for (int q = 0; q < c->nq; q++)
        for (long j = 0; j < n; j++) {
            real e = equilibrium_q(c, q, rho[j], ux[j], uy[j]);
            f[q * n + j] = (4.0 * tau[j] * fhat[q * n + j] + c->dt * e) / (4.0 * tau[j] + c->dt);
        }
    free(rho); free(ux); free(uy);
    return 0;
}

int OC(num_threads)(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* nsteps T3S3 steps in place on fhat */
int OC(t3s3_run)(const oc_case *c, const real *tau, real *fhat, int nsteps)
{
    long m = (long)c->nq * c->nx * c->ny;
    real *tmp = malloc(sizeof(real) * m);
    if (!tmp) return -1;
    for (int s = 0; s < nsteps; s++) {
        int rc = OC(t3s3_step)(c, tau, fhat, tmp);
        if (rc) { free(tmp); return rc; }
        memcpy(fhat, tmp, sizeof(real) * m);
    }
    free(tmp);
    return 0;
}
