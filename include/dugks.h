/*
 * dugks.h -- C ABI of the MI355X (gfx950) implementation of the per-step sweep
 * of the third-order discrete unified gas kinetic scheme (T3S3-DUGKS) of
 * Wu, Shu, Shi & Chen, arXiv 1709.05458 ("A third-order discrete unified gas
 * kinetic scheme for continuum and rarefied flows: low-speed isothermal case").
 *
 * One time step (paper section "Computational sequence of the third-order
 * DUGKS", steps (1)-(4), evolution equation feqIntD3rdHat2_DS) is two sweeps
 * over every (cell, discrete velocity) pair:
 *   stage A  steps (1)-(2): fhat(t_n) -> fbar^{+,dt/6} (eq. f_bar_1_6) ->
 *            interface values at t_n + dt/6 (eqs. interfaceEvof, flux_DS) ->
 *            interface moments, equilibrium and recovery (eq. recover2f) ->
 *            micro-flux L* (eq. microflux) -> tilde f(t_n + dt/3)
 *            (eq. f_tilde_1_3 and the T2 update of Remark I with step dt/3);
 *   stage C  steps (3)-(4): tilde f(t') -> fbar^{+,5dt/12} (eq. fbp_5_12) ->
 *            interface values, moments, recovery at t_n + 3dt/4 -> L** ->
 *            fhat(t_{n+1}) = fhat^+ + 3/4 dt Omega(t') + dt/7 (3 L* + 4 L**).
 *
 * Conventions for every entry point:
 *  - Every function returns 0 (DUGKS_OK) or a negative dugks_status code; no
 *    C++ exception crosses this interface.  dugks_strerror() names a code and
 *    dugks_last_error_message() gives the detail of the last failure on the
 *    calling thread.
 *  - Distribution arrays are double, layout [q][cell] with cell = j*nx + i
 *    (x fastest); cell fields are double [cell].  `mem` says whether a pointer
 *    is host (DUGKS_MEM_HOST) or device (DUGKS_MEM_DEVICE) memory.  The caller
 *    owns every buffer it passes; the library copies what it keeps.
 *  - All device work is queued on the stream given at creation.  Functions
 *    that read results into host memory synchronise that stream.
 *  - A handle must not be used from two threads at once.
 */
#ifndef DUGKS_H
#define DUGKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dugks dugks_t;

enum dugks_status {
    DUGKS_OK = 0,
    DUGKS_EINVAL = -1,      /* invalid argument or descriptor */
    DUGKS_EUNSTABLE = -2,   /* dt/tau above 12 somewhere (paper: von Neumann bound of P_n at a = 1/3) */
    DUGKS_EMOMENT = -3,     /* weights miss sum w = 1 or sum w xi xi = RT I by more than 1e-10 */
    DUGKS_ENOMEM = -4,      /* device or host allocation failed */
    DUGKS_EDEVICE = -5,     /* a HIP runtime call failed */
    DUGKS_ENONFINITE = -6,  /* a non-finite density appeared in the state */
    DUGKS_ENOTSUP = -7      /* valid but not supported by this build */
};

enum dugks_bc {
    DUGKS_BC_PERIODIC = 0,
    DUGKS_BC_BOUNCE_BACK = 1,   /* paper eq. BB */
    DUGKS_BC_DIFFUSE = 2        /* paper's diffuse-scattering rule */
};

enum dugks_side { DUGKS_WEST = 0, DUGKS_EAST = 1, DUGKS_SOUTH = 2, DUGKS_NORTH = 3 };

enum dugks_precision {
    DUGKS_FP64 = 0,        /* state stored and swept in double */
    DUGKS_FP32_DELTA = 1   /* state stored as float g_q = f_q / w_q - rho0; moments in double */
};

enum dugks_mem { DUGKS_MEM_HOST = 0, DUGKS_MEM_DEVICE = 1 };

/* Time integrator.  T3S3: the paper's third-order two-stage step (steps
 * (1)-(4), eq. feqIntD3rdHat2_DS), state fhat = f - (dt/4) Omega.  T2S3: the
 * second-order step the paper compares against (Remark I, eq.
 * feqIntD2nd_Explicit with the full step on the flux) with the same
 * third-order interface reconstruction (eq. flux_DS): state
 * ftilde = f - (dt/2) Omega, one reconstruction per step over h = dt/2,
 *     ftilde(t+dt) = ((2 tau - dt) ftilde + 2 dt E) / (2 tau + dt) + dt L,
 * where L is the micro-flux of fbar^{+,h} = ((4 tau - dt) ftilde + 3 dt E) / (4 tau + 2 dt)
 * reconstructed at the faces and recovered (eq. recover2f). */
enum dugks_scheme { DUGKS_SCHEME_T3S3 = 0, DUGKS_SCHEME_T2S3 = 1 };

enum dugks_flags {
    DUGKS_ALLOW_MOMENT_DEFECT = 1,  /* accept weights that are not moment-exact (e.g. Newton-Cotes) */
    DUGKS_FORCE_GENERIC = 2         /* use the any-size velocity-set kernels even for D2Q9 / D2Q37 */
};

/* Creation descriptor.  Pointers are host pointers, read only during
 * dugks_create. */
typedef struct {
    int nx, ny;             /* number of cells, each >= 3 */
    const double *xf;       /* nx+1 strictly increasing face x-coordinates */
    const double *yf;       /* ny+1 strictly increasing face y-coordinates */
    int nq;                 /* number of discrete velocities, >= 1 */
    const double *xi;       /* [2][nq]: xi[q] = x-component, xi[nq+q] = y-component */
    const double *w;        /* [nq] equilibrium weights, Gaussian factor included:
                             * f^eq_q = w_q rho [1 + xi.u/RT + (xi.u)^2/(2RT^2) - u^2/(2RT)]
                             * (paper, low-Mach expansion of the Maxwellian) */
    double RT;              /* gas constant times temperature, > 0 */
    double dt;              /* time step, > 0 */
    const double *tau;      /* [ny][nx] per-cell relaxation time, or NULL for tau0 */
    double tau0;            /* uniform relaxation time when tau == NULL */
    int bc[4];              /* dugks_bc per side (west, east, south, north);
                             * periodic must be paired (west with east, south with north) */
    double u_wall[4][2];    /* wall velocity per side */
    int precision;          /* dugks_precision */
    double rho0;            /* reference density of DUGKS_FP32_DELTA storage */
    double taylor_quad;     /* coefficient of the quadratic term of the interface
                             * expansion (eq. flux_DS): 1.0 as printed, 0.5 for the
                             * Taylor polynomial; 0 selects 1.0 */
    void *stream;           /* hipStream_t for all work, NULL = null stream */
    int flags;              /* dugks_flags */
    int tile_x, tile_y;     /* sweep tile in cells; 0 = library choice */
    int scheme;             /* dugks_scheme; 0 = T3S3.  Both schemes take the
                             * dt/tau <= 12 guard; dugks_backward and batches take
                             * T3S3 only (DUGKS_ENOTSUP / DUGKS_EINVAL) */
    /* --- relaxation time from the Knudsen number (paper, "Numerical tests":
     * Kn = lambda / L with the mean free path lambda = tau sqrt(pi RT / 2)):
     * used when tau == NULL and tau0 <= 0; then tau0 = kn * l_ref / sqrt(pi RT / 2). */
    double kn;
    double l_ref;
    /* --- variants of the paper's method, run by separate kernels that follow
     * the computational sequence step by step (FP64 storage, uniform periodic
     * grids; otherwise DUGKS_ENOTSUP):
     * family_a: the member a of the time-discretization family (section "Time
     *   discretization": A = a/2, K from A = (3K-2)/(6K-3), eq. EEWithP with
     *   P_n, P', P_{n+1}); 0 selects 1/3, the paper's T3S3; other values must
     *   lie in (1/3, 1/2].  The stored state is f - P_{n+1} dt Omega.
     * reconstruction: dugks_reconstruction. */
    double family_a;
    int reconstruction;
    /* --- device memory of the handle's buffers: when dev_alloc is not NULL the
     * library takes every buffer it keeps (state, tables, workspaces) from
     * dev_alloc(bytes, alloc_ctx) and returns it with dev_free(ptr, alloc_ctx)
     * (for example a caching allocator); a NULL return fails with
     * DUGKS_ENOMEM.  Temporary staging of host arrays still uses the runtime
     * allocator. */
    void *(*dev_alloc)(size_t bytes, void *ctx);
    void (*dev_free)(void *ptr, void *ctx);
    void *alloc_ctx;
} dugks_desc;

/* Interface reconstructions (dugks_desc.reconstruction).  POINT is the
 * library's reading of eq. flux_DS: cell values as centre values, one
 * midpoint per face for eq. microflux.  CELL_AVERAGE reads the cell values
 * as cell averages (the paper's definition of f_j), reconstructs the
 * quadratic whose cell averages match them, and integrates each face with the
 * two-point Gauss rule (recovery, eq. recover2f, at each Gauss point).  S2 is
 * the original DUGKS reconstruction the paper compares with (its reference
 * for the second-order scheme): linear interpolation at the face centre minus
 * xi h times the face gradient.  With DUGKS_SCHEME_T2S3, S2 gives the paper's
 * T2S2 scheme. */
enum dugks_reconstruction {
    DUGKS_RECON_POINT = 0,
    DUGKS_RECON_CELL_AVERAGE = 1,
    DUGKS_RECON_S2 = 2
};

/* Build a solver for one grid / velocity set / relaxation field (paper:
 * finite-volume grid, discrete velocity sets, BGK relaxation time, walls).
 * Checks: nx, ny >= 3; faces increasing; periodic sides paired; dt > 0,
 * RT > 0, tau > 0; max dt/tau <= 12 (else DUGKS_EUNSTABLE); bounce-back needs
 * every velocity to have a mirror with the same weight (else EINVAL); weight
 * moments (else DUGKS_EMOMENT unless DUGKS_ALLOW_MOMENT_DEFECT).
 * Velocity sets equal to the library's D2Q9 or D2Q37 lattice (xi = c e_q in
 * its order) run the lattice kernels; any other set (e.g. Newton-Cotes
 * grids) runs the any-size kernels, which support periodic and diffuse
 * boundaries (bounce-back: DUGKS_ENOTSUP).  On success *out owns device
 * buffers of 3 * nq * nx * ny elements plus small tables (any-size kernels:
 * also per-chunk interface and cell moment sums); the state is undefined
 * until set_state or init_equilibrium. */
int dugks_create(const dugks_desc *d, dugks_t **out);

/* Release every resource of h.  h == NULL is a no-op. */
int dugks_destroy(dugks_t *h);

/* State at t_n from the physical distribution f [q][cell]; the library stores
 * fhat = f - (dt/4) Omega(f) (paper eq. feqIntD3rdHat2 definitions), or for
 * DUGKS_SCHEME_T2S3 ftilde = f - (dt/2) Omega(f). */
int dugks_set_state(dugks_t *h, const double *f, int mem);

/* f = E(rho, u) at every cell (paper: initial state is the equilibrium). */
int dugks_init_equilibrium(dugks_t *h, const double *rho, const double *ux,
                           const double *uy, int mem);

/* Advance nsteps steps of the handle's scheme (asynchronous on the stream).
 * Lattice handles (D2Q9 / D2Q37 kernels) replay each step from a HIP graph
 * captured at the second call (one graph per parity of the ping-pong state);
 * the first call, and every call while kernel timing is on, launches the
 * kernels directly.  Both give the same bits. */
int dugks_step(dugks_t *h, int nsteps);

/* Cell density and velocity [cell] of the current state: rho = sum_q f_q,
 * rho u = sum_q xi_q f_q (paper, section "Discrete particle velocities", the
 * moments of the discrete distribution), taken of fhat, whose moments equal
 * those of f because the collision conserves them (the definitions under eq.
 * feqIntD3rdHat2) when the weights are moment-exact.  Outputs are caller-owned,
 * NULL to skip one; mem == DUGKS_MEM_HOST synchronises the stream.  Errors:
 * DUGKS_EINVAL (null handle, bad mem), DUGKS_ENOMEM (host staging). */
int dugks_moments(dugks_t *h, double *rho, double *ux, double *uy, int mem);

/* Physical distribution f = (4 tau fhat + dt E) / (4 tau + dt), [q][cell],
 * the inverse of fhat = f - (dt/4) Omega (paper, definitions under eq.
 * feqIntD3rdHat2, and the fhat^+ relation that follows them; T2S3:
 * f = (2 tau ftilde + dt E) / (2 tau + dt), Remark I; family member a:
 * f = (tau fhat + P_{n+1} dt E) / (tau + P_{n+1} dt)).  f is caller-owned. */
int dugks_get_state(dugks_t *h, double *f, int mem);

/* The stored variable (fhat, or ftilde for T2S3) itself, [q][cell], in double. */
int dugks_get_fhat(dugks_t *h, double *fhat, int mem);

/* Replace the relaxation-time field ([cell], > 0, dt/tau <= 12: the paper's
 * stability bound at a = 1/3, section "Time discretization").  The BGK
 * relaxation time of Omega = -(f - f^eq)/tau (eq. BE and below); only
 * handles created with a tau field (desc.tau != NULL) take it (else
 * DUGKS_EINVAL); DUGKS_EUNSTABLE if a value breaks the bound. */
int dugks_set_tau(dugks_t *h, const double *tau, int mem);

/* Block until all queued work of h is done; reports DUGKS_ENONFINITE if a
 * stage wrote a non-finite value since the last dugks_sync.  The stage kernels
 * test one velocity of every cell they write and raise a device flag; a
 * non-finite value reaches every velocity of its cell and of its neighbours
 * through the cell and interface moments in the next stage, so it is flagged
 * at the latest one stage after it appears.  The flag is cleared by the
 * call. */
int dugks_sync(dugks_t *h);

/* Discrete adjoint (not part of the paper's method): the exact gradient of
 * the discrete map of nsteps steps (steps (1)-(4), eq. feqIntD3rdHat2_DS,
 * preceded by the f -> fhat map) for
 *     L = sum_j dL_drho_j rho_j(T) + dL_du_j . u_j(T)
 * (rho, u: moments of the state as dugks_moments returns them), with respect
 * to the physical initial state f0 ([q][cell]) and the per-cell relaxation
 * time ([cell]; for a handle with a uniform tau the per-cell sensitivity is
 * returned, whose sum is dL/dtau0).  dL_du is [2][cell] (x then y);
 * dL_drho and dL_dtau may be NULL.  All pointers are in the memory named by
 * mem; outputs are caller-owned.
 * The forward pass is run from f0 keeping the state every ckpt_every steps;
 * the reverse sweep recomputes each segment from its checkpoint, so device
 * memory grows as (nsteps/ckpt_every + ckpt_every) states plus about 14
 * double arrays of nq*nx*ny.  That workspace is allocated on the first call
 * and kept by the handle (released by dugks_destroy); a later call that needs
 * more replaces it.  The adjoint arithmetic is double for both precisions (for
 * DUGKS_FP32_DELTA it linearises around the FP32 trajectory).  No atomics:
 * results are bitwise reproducible.  The handle's state is left unchanged.
 * Any grid and walls: bounce-back (eq. BB, with the wall cell's density) and
 * diffuse walls (the diffuse-scattering rule, with its wall density) are
 * differentiated as the sweep applies them, as are the one-sided stencils
 * next to walls and the per-cell spacings of stretched grids.  The T3S3
 * scheme only (else DUGKS_ENOTSUP); batch handles: DUGKS_ENOTSUP; nsteps < 0
 * or ckpt_every < 1: DUGKS_EINVAL. */
int dugks_backward(dugks_t *h, const double *f0, int nsteps, int ckpt_every,
                   const double *dL_drho, const double *dL_du,
                   double *dL_df0, double *dL_dtau, int mem);

/* dugks_backward for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same computation and results, with its workspace carved out of a fixed
 * device array of 128 MiB (one per device, held from the first handle created
 * on it until the process ends) instead of allocated.  Every pointer is
 * device memory; the caller passes inputs and outputs.  A call whose
 * workspace (the checkpoints plus about 14 double arrays of nq*nx*ny, see
 * dugks_backward) exceeds 128 MiB returns DUGKS_EINVAL and does nothing.
 * Calls on one device share that array: calls that overlap in time on the
 * same device (other threads, other streams) race and must be serialised by
 * the caller.  The call synchronises the handle's stream before returning. */
int dugks_backward_noalloc(dugks_t *h, const double *f0, int nsteps, int ckpt_every,
                           const double *dL_drho, const double *dL_du,
                           double *dL_df0, double *dL_dtau);

/* Batch of independent instances (uneven grids, velocity sets, relaxation
 * times and walls) stepped together: every dugks_step launches one kernel
 * per tile kind for all lattice instances and one per phase for all
 * any-size instances, replayed from a HIP graph captured on the first step
 * (a step is one graph launch).  All descriptors share
 * precision and stream; instances of one lattice kind, and all any-size
 * instances, need tiles with the same cell count (any-size instances left
 * on the library's tile share one ring-tile shape).  Any-size instances take
 * velocity chunks of one common length across the batch; an instance whose
 * chunks then differ from those it takes alone sums its interface moments in
 * other groups and agrees with its single run to the rounding of those FP64
 * sums (bit for bit otherwise).  Instance handles from
 * dugks_batch_instance are owned by the batch and serve set_state,
 * init_equilibrium, moments and get_state; stepping one alone makes the
 * next batch step fail with DUGKS_EINVAL.  dugks_sync checks every instance. */
int dugks_create_batch(int n, const dugks_desc *descs, dugks_t **out);
int dugks_batch_size(dugks_t *h, int *n);
int dugks_batch_instance(dugks_t *h, int k, dugks_t **inst);

/* Kernel timing by HIP events recorded around each launch on the stream.
 * prof_begin clears the record (room for max_launches launches); after the
 * stream is synchronised, prof_query returns the mean duration in ms and the
 * count of launches of one kernel class (dugks_kernel).
 *   STAGE_A, STAGE_C: one stage of dugks_step on the lattice kernels (all of a
 *     step for T2S3: STAGE_A);
 *   AUX: one graph launch of a batch step;
 *   LQ_FACES, LQ_UPDATE: the faces and the update kernel of one stage of the
 *     any-size kernels (while profiling, those stages record these two
 *     instead of STAGE_A / STAGE_C; the two reductions are not timed);
 *   ADJ_STEP: one reverse step of dugks_backward (its five kernels: the
 *     linearisation point, two face adjoints, two cell adjoints). */
enum dugks_kernel {
    DUGKS_K_STAGE_A = 0, DUGKS_K_STAGE_C = 1, DUGKS_K_AUX = 2,
    DUGKS_K_LQ_FACES = 3, DUGKS_K_LQ_UPDATE = 4, DUGKS_K_ADJ_STEP = 5, DUGKS_K_COUNT = 6
};
int dugks_prof_begin(dugks_t *h, int max_launches);
int dugks_prof_query(dugks_t *h, int kernel, double *mean_ms, int *count);
int dugks_prof_end(dugks_t *h);

/* Description of the chosen sweep: kernel variant name and tile. */
int dugks_describe(dugks_t *h, char *buf, int len);

const char *dugks_strerror(int code);
const char *dugks_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* DUGKS_H */
