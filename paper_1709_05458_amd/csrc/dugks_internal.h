// Internal declarations shared by the C-ABI host code and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dk {

// Records msg as the calling thread's last error (dugks_last_error_message)
// and returns code.
int set_error(int code, const char *msg);

// Geometry tables for the general (walls / non-uniform) reconstruction path.
// All device pointers.  Periodic neighbours are expressed through the face
// offsets dxl/dxr, which already include the periodic image shift.
struct Geometry {
    const double *dxl, *dxr;   // [nx+1]: xf[f] - xc(f-1), xf[f] - xc(f)
    const double *dyl, *dyr;   // [ny+1]
    const int *sx_off, *sy_off;         // [n]: first cell offset of the 3-point stencil (-1, 0, -2)
    const double *sx_d1, *sx_d2;        // [nx][3] derivative weights at the cell centre
    const double *sy_d1, *sy_d2;        // [ny][3]
    const double *inv_dx, *inv_dy;      // [nx], [ny] 1 / cell width
};

// tau-dependent coefficients precomputed on the host when tau is uniform
struct UniformCoef {
    double cc[2], ce[2];        // pre-reconstruction transform of stage A / C
    double c1, e1;              // fbar^{+,dt/6} = c1 fhat + e1 E
    double kx0, ke0, aL0;       // stage A output: kx0 X + ke0 E + aL0 L
    double a_f, a_En, a_G, a_Ep;   // stage C own-cell combination
    double alpha[2], beta[2];   // interface recovery of stage A / C
};

// Stage-A coefficients of one cell: B = cc X + ce E before the reconstruction,
// output kx X + ke E + aL L.  T3S3 (state fhat): B = fbar^{+,dt/6} (eq.
// f_bar_1_6), output tilde f(t') = 5/4 B - 1/4 fhat + dt/3 L* (eq.
// f_tilde_1_3 and Step 2).  T2S3 (state ftilde, Remark I with step dt):
// B = fbar^{+,dt/2}, output ftilde^+ + dt L.
struct Stage0Coef {
    double cc, ce, kx, ke;
};
__host__ __device__ inline Stage0Coef stage0_coef(bool t2, double tau, double dt)
{
    Stage0Coef c;
    if (t2) {
        c.cc = (4.0 * tau - dt) / (4.0 * tau + 2.0 * dt);
        c.ce = 3.0 * dt / (4.0 * tau + 2.0 * dt);
        c.kx = (2.0 * tau - dt) / (2.0 * tau + dt);
        c.ke = 2.0 * dt / (2.0 * tau + dt);
    } else {
        c.cc = (12.0 * tau - dt) / (12.0 * tau + 3.0 * dt);
        c.ce = 4.0 * dt / (12.0 * tau + 3.0 * dt);
        c.kx = 1.25 * c.cc - 0.25;
        c.ke = 1.25 * c.ce;
    }
    return c;
}

// Everything a sweep kernel needs; passed by value as a kernel argument.
struct SweepParams {
    int nx, ny;
    long long ncell;
    int t2;                  // scheme T2S3 (one stage-A-shaped step, state ftilde)
    int perx, pery;          // periodic in x / y
    int uniform;             // uniform spacing in both directions
    int nq;
    double RT, dt;
    double rho0;             // FP32-delta reference density (0 for FP64 storage)
    double M0m1;             // sum w - 1
    double M1x, M1y;         // sum w xi
    double kappa;            // coefficient of the quadratic expansion term
    double clat;             // lattice scale (compile-time lattices: xi = clat * e)
    double inv_dx, inv_dy;   // uniform grids
    // relaxation time
    const double *tau;       // [cell] or nullptr
    double tau0;
    int tau_field;
    UniformCoef uc;
    double iRT;              // 1 / RT
    double state_m;          // stored state f + dt/(state_m tau) (f - E): 4 (T3S3), 2 (T2), 1/P_{n+1} (family a)
    Geometry g;
    // velocity set (device)
    const double *xi, *eta, *w;
    const double *wmom;      // [nq][3]: moment weights (w, w ex, w ey) in lattice units
    // lattices: weight of each velocity shell times 1, 2, 3 (wtab[shell][m] =
    // m w_shell), read from the kernel arguments by the fast lattice kernels
    double wtab[8][4];
    // = ncell; separate copies keep the compiler from sharing per-velocity
    // plane offsets between the load, update and store phases of a kernel
    // (dozens of long-lived scalar registers)
    long long ncell_f, ncell_o;
    const int *opp;
    // walls
    int bc[4];
    double uw[4][2];
    const double *wall_E;    // [4][nq]: storage-scaled E_q(1, u_w) of each side
    double ds_den[4];        // sum over leaving q of |xi.n| w_q P_q(u_w)
    double ds_num_off[4];    // FP32-delta: rho0 * sum over arriving q of (xi.n) w_q
    double ds_m[4][3];       // sum over leaving q of (1, xi, eta) w_q P_q(u_w)
    double ds_w[4][3];       // sum over leaving q of (1, xi, eta) w_q
    int tile_x, tile_y;
    int nxcd;                // XCDs that workgroups are dealt to round-robin
    // large velocity sets: q split into lq_nchunk chunks of lq_chunk velocities,
    // streamed through LDS lq_qs planes at a time
    int lq_chunk, lq_nchunk, lq_qs;
    // lq_update's own split of q (its work items are 256 cells x lq_uchunk velocities)
    int lq_uchunk, lq_nuchunk;
    const void *lq_rec;      // [nq] QRec<float> (FP32-delta) or QRec<double> (FP64)
    int *bad;                // set to 1 by a stage kernel that writes a non-finite value
};

// Per-stage arguments of the large-velocity-set kernels.
// Everything the any-size kernels read per velocity, packed so that a block
// copies a run of velocities into LDS with plain 32-bit loads.
template <class S>
struct QRec {
    int sg;          // bit 0: xi > 0, 1: xi < 0, 2: eta > 0, 3: eta < 0
    int gnz;         // the plane group of this velocity is complete with no zero component
    S mono[9];       // xi, eta, xi^2, xi eta, eta^2, xi^3, xi^2 eta, xi eta^2, eta^3
    S wq;            // quadrature weight (scales the equilibrium in FP64 storage)
    S we[4];         // storage-scaled E_q(1, u_w) of the W, E, S, N walls
    double wm[7];    // m, m xi, m eta, m (-xi)+, m xi+, m (-eta)+, m eta+ (m = w or 1)
};
// velocities per LDS copy of the records
constexpr int LQ_TQ = 64;

struct LQStage {
    const void *X;          // stage input (fhat or tilde f), storage units
    const void *F;          // stage C: fhat(t_n)
    void *out;              // stage output
    const double *momX;     // [cell][4] (rho, rho - rho0 or rho, rho ux, rho uy) of X
    const double *momF;     // [cell][4] of F (stage C)
    double *face_part;      // [chunk][face][4] partial interface sums
    double *face_mom;       // [face][8] interface moments and diffuse-wall density
    double *cell_part;      // [chunk][cell][4] partial cell moments of out
    double *mom_out;        // [cell][4] cell moments of out
    double h;               // characteristic step of the stage
    int stage;              // 0: stage A, 1: stage C
    void *fxv = nullptr;    // [q][(nx+1) ny] interface values of the x-faces (storage type)
    void *fyv = nullptr;    // [q][nx (ny+1)] interface values of the y-faces
};

// Per-instance buffers of one stage of the lattice kernels (batched launches).
struct StageIO {
    const void *X;      // stage input
    const void *F;      // stage C: fhat(t_n)
    void *out;          // stage output
    const void *coef;   // fast-path face weights of the stage
    double h;           // characteristic step of the stage
};

// Interface reconstructions (dugks_desc.reconstruction).
enum { RECON_POINT = 0, RECON_CELL_AVERAGE = 1, RECON_S2 = 2 };

// Arguments of the variant kernels (variant.hip): uniform periodic grids, FP64.
struct VarArgs {
    int nx, ny, nq;
    long long n;
    double dx, dy, RT;
    const double *xi, *eta, *w;
    const double *tau;   // [cell] or nullptr for tau0
    double tau0;
    int recon;
    double kappa;        // coefficient of the quadratic expansion term
    int *bad;            // non-finite flag of the handle
};

// The member a of the time-discretization family: A = a/2, K from
// A = (3K-2)/(6K-3), P_n, P', P_{n+1} and the flux weights w1, w2.
struct VarFamily {
    double dt, a, A, K, Pn, Pp, Pn1, w1, w2;
};
__host__ __device__ inline VarFamily var_family(double a, double dt)
{
    VarFamily f;
    f.dt = dt;
    f.a = a;
    f.A = 0.5 * a;
    f.K = (2.0 - 3.0 * f.A) / (3.0 - 6.0 * f.A);
    f.Pn = (1.0 - 4.0 * a + 3.0 * a * a) / (6.0 * a * (a - 1.0));
    f.Pp = -1.0 / (6.0 * a * (a - 1.0));
    f.Pn1 = (-2.0 * a + 3.0 * a * a) / (6.0 * a * (a - 1.0));
    const double den = 4.0 * (3.0 * f.K * f.K - 3.0 * f.K + 1.0);
    f.w1 = 3.0 * (2.0 * f.K - 1.0) * (2.0 * f.K - 1.0) / den;
    f.w2 = 1.0 / den;
    return f;
}

// Work arrays of a variant step (device): B, G, L* ([q][cell]), moments
// M0, M1 ([3][cell]) and the face-point values Fx, Fy ([q][point][cell]).
struct VarBuffers {
    double *B, *G, *Ls, *M0, *M1, *Fx, *Fy;
};
hipError_t variant_step(const VarArgs &a, const VarFamily &fam, bool t2, const double *X, double *Y,
                        const VarBuffers &b, hipStream_t s);

// Kernel classes for event timing.
enum KernelClass { KC_STAGE_A = 0, KC_STAGE_C = 1, KC_AUX = 2, KC_LQ_FACES = 3, KC_LQ_UPDATE = 4, KC_ADJ_STEP = 5,
                   KC_COUNT = 6 };

// Host launchers (defined in sweep.hip).  `lat`: 0 generic, 9 D2Q9, 37 D2Q37.
// `delta`: FP32-delta storage (float) else FP64 storage (double).
// parts: 1 = tiles of the fast kind, 2 = the others, 3 = all.
hipError_t launch_stage(int stage, int lat, bool delta, const SweepParams &p, double h,
                        const void *X, const void *F, void *out, const void *coef,
                        hipStream_t s, int parts = 3);
hipError_t set_stage_smem(int lat, bool delta, size_t bytes);
// Fast-kind tiles with a compile-time tile shape (sweep_fast.hip): index of
// the shape among the compiled ones, or -1.
int fast_tile_index(int tx, int ty);
hipError_t set_fast_smem(int lat, bool delta, int tx, int ty, size_t bytes);
hipError_t launch_stage_fast(int stage, int lat, bool delta, const SweepParams &p, double h, const void *X,
                             const void *F, void *out, const void *coef, hipStream_t s);
hipError_t launch_stage_fast_batched(int stage, int lat, bool delta, int tx, int ty, bool tau_field,
                                     const SweepParams *P,
                                     const StageIO *io, const int4 *work, int nwork, size_t smem,
                                     hipStream_t s);
// Many instances in one launch per tile kind: work items (instance, tile x, tile y, 0).
hipError_t launch_stage_batched(int stage, int lat, bool delta, const SweepParams *P, const StageIO *io,
                                const int4 *work_fast, int nfast, const int4 *work_gen, int ngen,
                                int nthreads, size_t smem, hipStream_t s);
// Any-size kernels over many instances: work items (instance, tile, chunk, 0) for
// the face kernel, (instance, cell block, chunk, 0) for the update and
// (instance, block, 0, 0) for the two reductions.
hipError_t launch_lq_stage_batched(bool delta, const SweepParams *P, const LQStage *A,
                                   const int4 *work_tiles, int ntiles, const int4 *work_faces, int nfaces,
                                   const int4 *work_upd, int nupd, const int4 *work_cells, int ncells,
                                   int nthreads, size_t smem, hipStream_t s);

// Large velocity sets (sweep_large.hip).  part < 0: all four kernels of the stage.
hipError_t launch_lq_stage(bool delta, const SweepParams &p, const LQStage &a, hipStream_t s, int part);
// Ring tiles of the any-size kernels: a block of tile_x x tile_y threads
// covers (tile_x - 2) x (tile_y - 2) cells.
__host__ __device__ inline int lq_ntile(const SweepParams &p)
{
    return ((p.nx + p.tile_x - 3) / (p.tile_x - 2)) * ((p.ny + p.tile_y - 3) / (p.tile_y - 2));
}
hipError_t set_lq_smem(bool delta, size_t bytes);
size_t lq_smem_bytes(const SweepParams &p, bool delta);
// resident blocks of lq_faces (faces = true) or lq_update on one CU
int lq_blocks_per_cu(bool delta, bool faces, int nthreads, size_t smem);
hipError_t launch_state_moments(const SweepParams &p, bool delta, const void *state, double *mom,
                                hipStream_t s);

// Auxiliary per-cell kernels (state conversions, moments); defined in aux.hip.
hipError_t launch_set_state(const SweepParams &p, bool delta, const double *f, void *state,
                            hipStream_t s);
hipError_t launch_get_state(const SweepParams &p, bool delta, const void *state, double *f,
                            int physical, hipStream_t s);
hipError_t launch_init_eq(const SweepParams &p, bool delta, const double *rho, const double *ux,
                          const double *uy, void *state, hipStream_t s);
hipError_t launch_moments(const SweepParams &p, bool delta, const void *state, double *rho,
                          double *ux, double *uy, int *bad, hipStream_t s);

// Discrete adjoint of one step (adjoint.hip), double: window-weight kernels on
// periodic uniform grids, general kernels on walls and stretched grids.
struct AdjArgs {
    int nx, ny, nq;
    long long n;
    double dt, RT, iRT, idx, idy;
    const double *xi, *eta, *w;
    const double *tau;       // [cell]
    const double *cA, *cC;   // [q][24] interface window weights of stage A / C
    double h1, h2;
    // walls and stretched grids (the general kernels; the periodic uniform
    // kernels use the window weights above)
    int general;
    int perx, pery;
    int bc[4];               // DUGKS_BC_* of the W, E, S, N sides
    double uw[4][2];         // wall velocities
    const int *opp;          // [q]: index of -xi_q
    double kappa;            // coefficient of the quadratic term of the expansion
    const int *sx_off, *sy_off;                    // first stencil offset per column / row
    const double *sx_d1, *sx_d2, *sy_d1, *sy_d2;   // [3 n]: 3-point derivative weights
    const double *dxl, *dxr, *dyl, *dyr;           // face offsets from the cell centres
    const double *inv_dx, *inv_dy;                 // per column / row
};
// Primal intermediates of a step from fhat and the stage A output G (storage
// format): fhat, B and moments at t_n; G, B' and moments at t'.
hipError_t adj_launch_prep(const AdjArgs &a, bool delta, double rho0, const void *fhat, const void *G,
                           double *fh_d, double *B, double *M, double *G_d, double *B2, double *M2,
                           hipStream_t s);
// lambda_in = (d out / d fhat)^T lambda_out, dtau += (d out / d tau)^T lambda_out.
// With a.general: lam_fbar [q][face] and dtau_face [face] over the natural
// face numbering, lam_rho [face] and lamBg [q][cell] as well.
hipError_t adj_launch_step(const AdjArgs &a, const double *lam_out, double *lam_in, const double *fh_d,
                           const double *B, const double *M, const double *G_d, const double *B2,
                           const double *M2, double *lam_fbar, double *dtau_face, double *lamLs,
                           double *lamB, double *lamF, double *dtau, double *lam_rho, double *lamBg,
                           hipStream_t s);
hipError_t adj_launch_seed(const AdjArgs &a, const double *fh_d, const double *dL_drho, const double *dL_du,
                           double *lam, hipStream_t s);
hipError_t adj_launch_init(const AdjArgs &a, const double *f0, const double *lam, double *dL_df0,
                           double *dtau, hipStream_t s);

}  // namespace dk
