/*
 * dugks_oracle3d.c -- plain, slow, double-precision reference of one T3S3
 * step in three space dimensions, on a triply periodic box of uniform cells.
 *
 * TEST INFRASTRUCTURE ONLY.  It shares no code with the HIP library (nor with
 * the two-dimensional oracle, whose arithmetic it repeats in three
 * dimensions); only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.
 *
 * The paper states its method for any dimension D (kinetic model section)
 * and tests it in two; this file takes the same steps with a third axis:
 *   - equilibrium: w_q rho [1 + xi.u/RT + (xi.u)^2/(2 RT^2) - u^2/(2 RT)];
 *   - the transforms of eqs. f_bar_1_6, f_tilde_1_3 (reading R1), fbp_5_12
 *     (reading R2), collisionterm and feqIntD3rdHat2_DS, cell by cell;
 *   - interface values (eq. interfaceEvof) from the quadratic Taylor
 *     polynomial about the upwind cell (eq. flux_DS, three dimensions):
 *       B0 + d.grad B + k (dx^2 Bxx + dy^2 Byy + dz^2 Bzz
 *                          + 2 dx dy Bxy + 2 dx dz Bxz + 2 dy dz Byz),
 *     with the 3-point central derivatives of the midpoint scheme and
 *     k = 1 as printed (reading R3) or 1/2 (`literal_taylor` = 0);
 *     a velocity parallel to the face takes the mean of the expansions about
 *     its two cells (R4);
 *   - recovery at each face (eq. recover2f) with the face moments, the
 *     relaxation time the mean of the two cells' (R7), one point per face at
 *     its centre (R6), the micro-flux with the sign of R8.
 * Sums over q run in ascending order; nothing is fused or re-arranged.
 *
 * Layout: f[q][z][y][x]; cell fields [z][y][x]; xi[q], xi[nq+q], xi[2nq+q]
 * the three velocity components.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nx, ny, nz, nq;
    double dx, dy, dz;   /* cell widths (uniform, periodic on every axis) */
    const double *xi;    /* 3 x nq velocity components */
    const double *w;     /* equilibrium weights (Gaussian factor included) */
    double RT;
    double dt;
    int literal_taylor;  /* 1: expansion as printed (R3); 0: factor 1/2 */
} o3_case;

#define XI(c, a, q) ((c)->xi[(long)(a) * (c)->nq + (q)])

static long ncells(const o3_case *c) { return (long)c->nx * c->ny * c->nz; }

static int wrap(int i, int n)
{
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}

static long cell(const o3_case *c, int i, int j, int k)
{
    return ((long)wrap(k, c->nz) * c->ny + wrap(j, c->ny)) * c->nx + wrap(i, c->nx);
}

/* ------------------------------------------------------------------------ */
/* Equilibrium and moments                                                  */
/* ------------------------------------------------------------------------ */
static double equilibrium_q(const o3_case *c, int q, double rho, const double u[3])
{
    double eu = 0.0, uu = 0.0;
    for (int a = 0; a < 3; a++) {
        eu += XI(c, a, q) * u[a];
        uu += u[a] * u[a];
    }
    return c->w[q] * rho * (1.0 + eu / c->RT + eu * eu / (2.0 * c->RT * c->RT) - uu / (2.0 * c->RT));
}

/* rho and u of one distribution; stride = distance between q planes */
static void moments(const o3_case *c, const double *f, long stride, double *rho, double u[3])
{
    double r = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < c->nq; q++) {
        double v = f[q * stride];
        r += v;
        for (int a = 0; a < 3; a++) m[a] += XI(c, a, q) * v;
    }
    *rho = r;
    for (int a = 0; a < 3; a++) u[a] = m[a] / r;
}

void o3_cell_moments(const o3_case *c, const double *f, double *rho, double *u /* [3][n] */)
{
    long n = ncells(c);
    for (long j = 0; j < n; j++) {
        double uj[3];
        moments(c, f + j, n, &rho[j], uj);
        for (int a = 0; a < 3; a++) u[a * n + j] = uj[a];
    }
}

void o3_equilibrium(const o3_case *c, const double *rho, const double *u, double *E)
{
    long n = ncells(c);
    for (int q = 0; q < c->nq; q++)
        for (long j = 0; j < n; j++) {
            double uj[3] = {u[j], u[n + j], u[2 * n + j]};
            E[q * n + j] = equilibrium_q(c, q, rho[j], uj);
        }
}

/* ------------------------------------------------------------------------ */
/* Interface values: the quadratic Taylor polynomial of plane B about cell  */
/* (i, j, k), evaluated at the centre offset d.  The derivatives are those  */
/* of the quadratic through three equispaced centres.                       */
/* ------------------------------------------------------------------------ */
static double expand(const o3_case *c, const double *B, int i, int j, int k, const double d[3])
{
    const double h[3] = {c->dx, c->dy, c->dz};
    int o[3];
    double g[3], hd[3], hx[3];   /* first, second and mixed derivatives */
    double B0 = B[cell(c, i, j, k)];
    for (int a = 0; a < 3; a++) {
        o[0] = o[1] = o[2] = 0;
        o[a] = 1;
        double p = B[cell(c, i + o[0], j + o[1], k + o[2])];
        double m = B[cell(c, i - o[0], j - o[1], k - o[2])];
        g[a] = (p - m) / (2.0 * h[a]);
        hd[a] = (p - 2.0 * B0 + m) / (h[a] * h[a]);
    }
    /* mixed: xy, xz, yz from the four edge neighbours */
    for (int p = 0; p < 3; p++) {
        int a = p == 2 ? 1 : 0, b = p == 0 ? 1 : 2;
        int ea[3] = {0, 0, 0}, eb[3] = {0, 0, 0};
        ea[a] = 1;
        eb[b] = 1;
        double s = 0.0;
        for (int sa = -1; sa <= 1; sa += 2)
            for (int sb = -1; sb <= 1; sb += 2)
                s += sa * sb *
                     B[cell(c, i + sa * ea[0] + sb * eb[0], j + sa * ea[1] + sb * eb[1], k + sa * ea[2] + sb * eb[2])];
        hx[p] = s / (4.0 * h[a] * h[b]);
    }
    double kq = c->literal_taylor ? 1.0 : 0.5;
    return B0 + d[0] * g[0] + d[1] * g[1] + d[2] * g[2] +
           kq * (d[0] * d[0] * hd[0] + d[1] * d[1] * hd[1] + d[2] * d[2] * hd[2] + 2.0 * d[0] * d[1] * hx[0] +
                 2.0 * d[0] * d[2] * hx[1] + 2.0 * d[1] * d[2] * hx[2]);
}

/* Interface value fbar(x_b, t + h) = fbar^+(x_b - xi h, t) at the low face of
 * cell (i, j, k) along axis `ax` (eq. interfaceEvof). */
static double face_value(const o3_case *c, const double *Bq, int q, int ax, int i, int j, int k, double h)
{
    const double w[3] = {c->dx, c->dy, c->dz};
    int lo[3] = {i, j, k};
    lo[ax] -= 1;   /* the cell on the low side */
    double d[3];
    for (int a = 0; a < 3; a++) d[a] = -XI(c, a, q) * h;   /* transverse: shared centres */
    double e = XI(c, ax, q);
    if (e > 0.0) {
        d[ax] = 0.5 * w[ax] - e * h;   /* from the low cell's centre */
        return expand(c, Bq, lo[0], lo[1], lo[2], d);
    }
    if (e < 0.0) {
        d[ax] = -0.5 * w[ax] - e * h;  /* from the own cell's centre */
        return expand(c, Bq, i, j, k, d);
    }
    d[ax] = 0.5 * w[ax];
    double vl = expand(c, Bq, lo[0], lo[1], lo[2], d);
    d[ax] = -0.5 * w[ax];
    double vh = expand(c, Bq, i, j, k, d);
    return 0.5 * (vl + vh);
}

/* ------------------------------------------------------------------------ */
/* Micro-flux L = -(1/|V|) sum_faces (xi . n) |A| f_b (eq. microflux, R8)   */
/* after the recovery of eq. recover2f at every face.                       */
/* fb: [3][nq][n], the low face of every cell along each axis.              */
/* ------------------------------------------------------------------------ */
int o3_face_values(const o3_case *c, const double *B, double h, double *fb)
{
    long n = ncells(c);
    int nq = c->nq;
    for (int ax = 0; ax < 3; ax++)
        for (int k = 0; k < c->nz; k++)
            for (int j = 0; j < c->ny; j++)
                for (int i = 0; i < c->nx; i++)
                    for (int q = 0; q < nq; q++)
                        fb[((long)ax * nq + q) * n + cell(c, i, j, k)] =
                            face_value(c, B + (long)q * n, q, ax, i, j, k, h);
    return 0;
}

int o3_flux(const o3_case *c, const double *tau, const double *B, double h, double *L)
{
    long n = ncells(c);
    int nq = c->nq;
    double *fb = (double *)malloc(sizeof(double) * 3 * nq * n);
    if (!fb) return -1;
    o3_face_values(c, B, h, fb);

    /* recovery: f_b = (2 tau_b fbar + h E(mom fbar)) / (2 tau_b + h) */
    for (int ax = 0; ax < 3; ax++)
        for (int k = 0; k < c->nz; k++)
            for (int j = 0; j < c->ny; j++)
                for (int i = 0; i < c->nx; i++) {
                    int lo[3] = {i, j, k};
                    lo[ax] -= 1;
                    long me = cell(c, i, j, k), ml = cell(c, lo[0], lo[1], lo[2]);
                    double tb = 0.5 * (tau[ml] + tau[me]);
                    double *f = fb + (long)ax * nq * n + me;
                    double rho, u[3];
                    moments(c, f, n, &rho, u);
                    for (int q = 0; q < nq; q++) {
                        double e = equilibrium_q(c, q, rho, u);
                        f[q * n] = (2.0 * tb * f[q * n] + h * e) / (2.0 * tb + h);
                    }
                }

    const double w[3] = {c->dx, c->dy, c->dz};
    for (int k = 0; k < c->nz; k++)
        for (int j = 0; j < c->ny; j++)
            for (int i = 0; i < c->nx; i++) {
                long me = cell(c, i, j, k);
                for (int q = 0; q < nq; q++) {
                    double s = 0.0;
                    for (int ax = 0; ax < 3; ax++) {
                        int hi[3] = {i, j, k};
                        hi[ax] += 1;
                        double flo = fb[((long)ax * nq + q) * n + me];
                        double fhi = fb[((long)ax * nq + q) * n + cell(c, hi[0], hi[1], hi[2])];
                        s += XI(c, ax, q) * (fhi - flo) / w[ax];
                    }
                    L[(long)q * n + me] = -s;
                }
            }
    free(fb);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One T3S3 step: steps (1)-(4) of the computational sequence, eq.          */
/* feqIntD3rdHat2_DS.  State: fhat = f - dt/4 Omega.                        */
/* ------------------------------------------------------------------------ */
int o3_t3s3_step(const o3_case *c, const double *tau, const double *fhat, double *out)
{
    int nq = c->nq;
    long n = ncells(c);
    double dt = c->dt;
    size_t qs = sizeof(double) * nq * n, cs = sizeof(double) * n;
    double *E = malloc(qs), *B = malloc(qs), *Ls = malloc(qs), *G = malloc(qs);
    double *W = malloc(qs), *Bp = malloc(qs), *Lss = malloc(qs), *Ep = malloc(qs);
    double *rho = malloc(cs), *u = malloc(3 * cs);
    int rc = 0;
    if (!E || !B || !Ls || !G || !W || !Bp || !Lss || !Ep || !rho || !u) { rc = -1; goto done; }

    o3_cell_moments(c, fhat, rho, u);
    o3_equilibrium(c, rho, u, E);

    /* Step 1: fbar^{+,dt/6}(t_n) (eq. f_bar_1_6), L* at t_n + dt/6 */
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            double t = tau[j];
            B[q * n + j] = (12.0 * t - dt) / (12.0 * t + 3.0 * dt) * fhat[q * n + j] +
                           4.0 * dt / (12.0 * t + 3.0 * dt) * E[q * n + j];
        }
    if ((rc = o3_flux(c, tau, B, dt / 6.0, Ls))) goto done;

    /* Step 2: T2 sub-step of dt/3 (eq. f_tilde_1_3, R1), then dt Omega(t')
     * (eq. collisionterm) */
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++)
            G[q * n + j] = 1.25 * B[q * n + j] - 0.25 * fhat[q * n + j] + dt / 3.0 * Ls[q * n + j];
    o3_cell_moments(c, G, rho, u);
    o3_equilibrium(c, rho, u, Ep);
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            double t = tau[j];
            W[q * n + j] = -6.0 * dt / (6.0 * t + dt) * (G[q * n + j] - Ep[q * n + j]);
        }

    /* Step 3: fbar^{+,5dt/12}(t') (eq. fbp_5_12, R2), L** at t_n + 3dt/4 */
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            double t = tau[j];
            Bp[q * n + j] = (24.0 * t - 5.0 * dt) / (24.0 * t + 4.0 * dt) * G[q * n + j] +
                            9.0 * dt / (24.0 * t + 4.0 * dt) * Ep[q * n + j];
        }
    if ((rc = o3_flux(c, tau, Bp, 5.0 * dt / 12.0, Lss))) goto done;

    /* Step 4: eq. fhp and eq. feqIntD3rdHat2_DS */
    for (int q = 0; q < nq; q++)
        for (long j = 0; j < n; j++) {
            long k = q * n + j;
            double fhp = 0.25 * fhat[k] + 0.75 * B[k];
            out[k] = fhp + 0.75 * W[k] + dt / 7.0 * (3.0 * Ls[k] + 4.0 * Lss[k]);
        }
done:
    free(E); free(B); free(Ls); free(G); free(W); free(Bp); free(Lss); free(Ep);
    free(rho); free(u);
    return rc;
}

int o3_run(const o3_case *c, const double *tau, double *fhat, int nsteps)
{
    long m = (long)c->nq * ncells(c);
    double *tmp = (double *)malloc(sizeof(double) * m);
    if (!tmp) return -1;
    for (int s = 0; s < nsteps; s++) {
        int rc = o3_t3s3_step(c, tau, fhat, tmp);
        if (rc) { free(tmp); return rc; }
        memcpy(fhat, tmp, sizeof(double) * m);
    }
    free(tmp);
    return 0;
}
