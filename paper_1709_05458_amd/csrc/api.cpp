// C ABI of the T3S3-DUGKS library (declarations and contracts in
// include/dugks.h): descriptor validation, device buffers, per-stage tables
// and launch sequencing.  Compiled by hipcc as host code.
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dugks.h"
#include "dugks_internal.h"
#include "lattices.h"

using namespace dk;

struct dugks {
    SweepParams p{};
    int lat = 0;          // 9, 37 (compile-time lattices) or 0 (generic)
    bool fast_ct = false; // fast-kind tiles run the compile-time-shape kernels
    bool delta = false;
    hipStream_t stream = nullptr;
    size_t elem = 8;      // bytes per stored element
    void *state[2] = {nullptr, nullptr};
    int cur = 0;
    void *G = nullptr;    // stage A output
    void *coefA = nullptr, *coefC = nullptr;
    double h1 = 0, h2 = 0;
    int *d_bad = nullptr;
    // any-size velocity sets
    double *mom_state = nullptr, *mom_G = nullptr, *face_part = nullptr, *face_mom = nullptr,
           *cell_part = nullptr;
    void *fxv = nullptr, *fyv = nullptr;   // interface values of a stage ([q][face])
    std::vector<void *> allocs;
    // timing
    std::vector<hipEvent_t> ev;   // pairs
    std::vector<int> ev_kind;
    int prof_max = 0, prof_n = 0;
    bool prof_on = false;
    std::string variant;
    int device = 0;                      // device current at creation
    // caller's device allocator (dugks_desc.dev_alloc / dev_free), or none
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *alloc_ctx = nullptr;
    // variants (family member a, cell-average or S2 reconstruction): variant.hip
    bool var = false;
    VarArgs va{};
    VarFamily vf{};
    VarBuffers vb{};
    // graph replay of single-handle steps (lattice kernels): [parity]
    hipGraphExec_t step_exec[2] = {nullptr, nullptr};
    int step_calls = 0;
    std::vector<double> hxi;             // host copy of the velocities, [2][nq]
    void *adj_ws = nullptr;              // dugks_backward workspace, kept between calls
    size_t adj_ws_bytes = 0;
    // batch of instances (dugks_create_batch): the handle owns the instances
    // and steps them with batched launches replayed from captured graphs
    struct Batch;
    Batch *batch = nullptr;
};

struct dugks::Batch {
    std::vector<dugks *> inst;
    bool delta = false;
    SweepParams *d_params = nullptr;
    StageIO *d_io = nullptr;        // [parity][stage][instance]
    LQStage *d_lq = nullptr;        // [parity][stage][instance]
    struct Shape {                  // fast-kind tiles of one compiled tile shape
        int tx = 0, ty = 0;
        bool tf = false;            // instances with a tau field
        int4 *work = nullptr;
        int n = 0;
    };
    struct Group {                  // one lattice kind
        int lat = 0;
        int nthreads = 0;
        size_t smem = 0;
        int4 *fast = nullptr, *gen = nullptr;   // fast: tiles of shapes without a compiled kernel
        int nfast = 0, ngen = 0;
        std::vector<Shape> shapes;
    };
    std::vector<Group> groups;
    int4 *lq_tiles = nullptr, *lq_faces = nullptr, *lq_upd = nullptr, *lq_cells = nullptr;
    int nlq_tiles = 0, nlq_faces = 0, nlq_upd = 0, nlq_cells = 0, lq_threads = 0;
    size_t lq_smem = 0;
    hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [parity][1 or 2 steps]
    std::vector<void *> allocs;
};

static thread_local std::string g_err;

static int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

// the same record for the other C-ABI sources of the library
int dk::set_error(int code, const char *msg) { return fail(code, msg); }

#define HIPCHECK(expr)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(DUGKS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// device memory of the handle: the caller's allocator when it gave one
static int dev_get(dugks *h, void **p, size_t bytes)
{
    if (h->alloc_fn) {
        *p = h->alloc_fn(bytes ? bytes : 8, h->alloc_ctx);
        if (!*p) return fail(DUGKS_ENOMEM, "dev_alloc returned NULL");
        return DUGKS_OK;
    }
    hipError_t e = hipMalloc(p, bytes ? bytes : 8);
    if (e != hipSuccess) return fail(DUGKS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    return DUGKS_OK;
}

static void dev_put(dugks *h, void *p)
{
    if (!p) return;
    if (h->alloc_fn) h->free_fn(p, h->alloc_ctx);
    else (void)hipFree(p);
}

static int dalloc(dugks *h, void **p, size_t bytes)
{
    int rc = dev_get(h, p, bytes);
    if (rc) return rc;
    h->allocs.push_back(*p);
    return DUGKS_OK;
}

template <class T>
static int upload(dugks *h, const T *src, size_t count, const T **dst)
{
    void *p = nullptr;
    int rc = dalloc(h, &p, sizeof(T) * count);
    if (rc) return rc;
    HIPCHECK(hipMemcpy(p, src, sizeof(T) * count, hipMemcpyHostToDevice));
    *dst = (const T *)p;
    return DUGKS_OK;
}

// ---------------------------------------------------------------------------
// Lattice detection: xi_q == c * e_q for the compiled integer lattices.
// ---------------------------------------------------------------------------

// Fixed device workspace of dugks_backward_noalloc, for callers that cannot
// allocate device memory.  Each device the library runs on holds its own copy
// from the first handle created there until the process ends.  In host code
// the array's name is not a device address: the address each device sees is
// taken once per device with hipGetSymbolAddress (at handle creation) and only
// that address is used.
static constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kMaxDevices = 64;
static char *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Address of the scratch array on `device`, which must be the current device.
static int scratch_resolve(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(DUGKS_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return DUGKS_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(DUGKS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = (char *)ptr;
    return DUGKS_OK;
}

static int scratch_of(int device, char **base)
{
    if (device < 0 || device >= kMaxDevices) return fail(DUGKS_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    *base = g_scratch_ptr[device];
    if (!*base) return fail(DUGKS_EDEVICE, "no-allocation scratch not resolved on this device");
    return DUGKS_OK;
}

static const int kD2Q9x[9] = {-1, -1, -1, 0, 0, 0, 1, 1, 1};
static const int kD2Q9y[9] = {-1, 0, 1, -1, 0, 1, -1, 0, 1};
static const int kD2Q37x[37] = {0, -1, 0, 0, 1, -1, -1, 1, 1, -2, 0, 0, 2, -2, -2, -1, -1, 1, 1,
                                2, 2, -2, -2, 2, 2, -3, 0, 0, 3, -3, -3, -1, -1, 1, 1, 3, 3};
static const int kD2Q37y[37] = {0, 0, -1, 1, 0, -1, 1, -1, 1, 0, -2, 2, 0, -1, 1, -2, 2, -2, 2,
                                -1, 1, -2, 2, -2, 2, 0, -3, 3, 0, -1, 1, -3, 3, -3, 3, -1, 1};

static bool match_lattice(const double *xi, int nq, const int *ex, const int *ey, int Q, double &c)
{
    if (nq != Q) return false;
    double m = 0;
    int em = 0;
    for (int q = 0; q < Q; q++) {
        m = std::fmax(m, std::fabs(xi[q]));
        em = std::max(em, std::abs(ex[q]));
    }
    if (m <= 0 || em == 0) return false;
    c = m / em;
    for (int q = 0; q < Q; q++) {
        if (std::fabs(xi[q] - c * ex[q]) > 1e-12 * m) return false;
        if (std::fabs(xi[nq + q] - c * ey[q]) > 1e-12 * m) return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Fast-path coefficients: one linear combination per (q, face orientation)
// for uniform spacing (central 3-point derivatives, upwind choice by the sign
// of the normal velocity, mean of both sides when it is zero).
// ---------------------------------------------------------------------------
static void expansion3x3(double dn, double dt_, double hn, double ht, double kappa, double C[3][3])
{
    // C[a][b]: a = offset along the face normal (-1..1), b = tangential offset
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            const int oa = a - 1, ob = b - 1;
            const double e_a = oa == 0, e_b = ob == 0;
            const double d1a = oa / (2.0 * hn), d2a = (oa == 0 ? -2.0 : 1.0) / (hn * hn);
            const double d1b = ob / (2.0 * ht), d2b = (ob == 0 ? -2.0 : 1.0) / (ht * ht);
            C[a][b] = e_a * e_b + dn * d1a * e_b + dt_ * e_a * d1b +
                      kappa * (dn * dn * d2a * e_b + 2.0 * dn * dt_ * d1a * d1b + dt_ * dt_ * e_a * d2b);
        }
}

static std::vector<double> fast_coefs(const double *xi, int nq, double dx, double dy, double h,
                                      double kappa)
{
    std::vector<double> c((size_t)nq * 24, 0.0);
    for (int q = 0; q < nq; q++) {
        const double ex = xi[q], ey = xi[nq + q];
        // x-faces: window columns k = 0..3 <-> offsets -2..1 from the right cell
        for (int side = 0; side < 2; side++) {   // 0: upwind left, 1: upwind right
            double wgt;
            if (ex > 0) wgt = side == 0 ? 1.0 : 0.0;
            else if (ex < 0) wgt = side == 1 ? 1.0 : 0.0;
            else wgt = 0.5;
            if (wgt == 0.0) continue;
            const double dn = (side == 0 ? 0.5 * dx : -0.5 * dx) - ex * h;
            const double dtn = -ey * h;
            double C[3][3];
            expansion3x3(dn, dtn, dx, dy, kappa, C);
            const int uoff = side == 0 ? -1 : 0;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) {
                    const int k = uoff + (a - 1) + 2;
                    c[(size_t)q * 24 + k * 3 + b] += wgt * C[a][b];
                }
        }
        // y-faces: window rows k = 0..3 <-> offsets -2..1 from the upper cell
        for (int side = 0; side < 2; side++) {
            double wgt;
            if (ey > 0) wgt = side == 0 ? 1.0 : 0.0;
            else if (ey < 0) wgt = side == 1 ? 1.0 : 0.0;
            else wgt = 0.5;
            if (wgt == 0.0) continue;
            const double dn = (side == 0 ? 0.5 * dy : -0.5 * dy) - ey * h;
            const double dtn = -ex * h;
            double C[3][3];
            expansion3x3(dn, dtn, dy, dx, kappa, C);
            const int uoff = side == 0 ? -1 : 0;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) {
                    const int k = uoff + (a - 1) + 2;
                    c[(size_t)q * 24 + 12 + k * 3 + b] += wgt * C[a][b];
                }
        }
    }
    return c;
}

// ---------------------------------------------------------------------------
// Geometry tables (general path)
// ---------------------------------------------------------------------------
static double centre(const double *f, int n, int i)
{
    const double L = f[n] - f[0];
    double s = 0;
    while (i < 0) { i += n; s -= L; }
    while (i >= n) { i -= n; s += L; }
    return 0.5 * (f[i] + f[i + 1]) + s;
}

static void axis_tables(const double *f, int n, bool periodic, std::vector<double> &dl,
                        std::vector<double> &dr, std::vector<int> &off, std::vector<double> &d1,
                        std::vector<double> &d2, std::vector<double> &inv)
{
    dl.assign(n + 1, 0.0);
    dr.assign(n + 1, 0.0);
    off.assign(n, -1);
    d1.assign(3 * n, 0.0);
    d2.assign(3 * n, 0.0);
    inv.assign(n, 0.0);
    for (int k = 0; k <= n; k++) {
        dl[k] = f[k] - centre(f, n, k - 1);
        dr[k] = f[k] - centre(f, n, k);
    }
    for (int i = 0; i < n; i++) {
        int o0 = -1;
        if (!periodic) {
            if (i == 0) o0 = 0;
            else if (i == n - 1) o0 = -2;
        }
        off[i] = o0;
        const double xc = centre(f, n, i);
        double pp[3];
        for (int k = 0; k < 3; k++) pp[k] = centre(f, n, i + o0 + k) - xc;
        for (int k = 0; k < 3; k++) {
            const int a = (k + 1) % 3, b = (k + 2) % 3;
            const double den = (pp[k] - pp[a]) * (pp[k] - pp[b]);
            d1[3 * i + k] = -(pp[a] + pp[b]) / den;
            d2[3 * i + k] = 2.0 / den;
        }
        inv[i] = 1.0 / (f[i + 1] - f[i]);
    }
}

static bool is_uniform(const double *f, int n)
{
    const double d0 = f[1] - f[0];
    for (int i = 0; i < n; i++)
        if (std::fabs((f[i + 1] - f[i]) - d0) > 1e-12 * std::fabs(d0)) return false;
    return true;
}

// The dynamic-LDS limit is a per-kernel attribute: only ever raise it.
static int raise_fast_smem(int lat, bool delta, int tx, int ty, size_t smem)
{
    static size_t raised[2][2][8] = {};
    const int k = fast_tile_index(tx, ty);
    if (k < 0 || k >= 8) return fail(DUGKS_EINVAL, "no compiled kernel for this tile");
    size_t &mx = raised[lat == 9 ? 0 : 1][delta ? 1 : 0][k];
    if (smem > mx) {
        hipError_t e = set_fast_smem(lat, delta, tx, ty, smem);
        if (e != hipSuccess) return fail(DUGKS_EDEVICE, std::string("LDS size: ") + hipGetErrorString(e));
        mx = smem;
    }
    return DUGKS_OK;
}

// arguments of one stage of the any-size kernels
static LQStage lq_args(const dugks *h, int stage, const void *X, const void *F, void *out)
{
    LQStage a{};
    a.X = X;
    a.F = F;
    a.out = out;
    a.momX = stage == 0 ? h->mom_state : h->mom_G;
    a.momF = stage == 0 ? nullptr : h->mom_state;
    a.face_part = h->face_part;
    a.face_mom = h->face_mom;
    a.cell_part = h->cell_part;
    a.mom_out = stage == 0 ? h->mom_G : h->mom_state;
    a.h = stage == 0 ? h->h1 : h->h2;
    a.stage = stage;
    a.fxv = h->fxv;
    a.fyv = h->fyv;
    return a;
}

// one stage of a lattice instance: fast-kind tiles by the compile-time-shape
// kernel when the tile is one of the compiled shapes, the rest by the general one
static hipError_t lattice_stage(const dugks *h, int stage, const void *X, const void *F, void *out)
{
    const void *coef = stage == 0 ? h->coefA : h->coefC;
    const double hs = stage == 0 ? h->h1 : h->h2;
    if (!h->fast_ct) return launch_stage(stage, h->lat, h->delta, h->p, hs, X, F, out, coef, h->stream, 3);
    hipError_t e = hipSuccess;
    if (h->p.uniform) e = launch_stage_fast(stage, h->lat, h->delta, h->p, hs, X, F, out, coef, h->stream);
    if (e != hipSuccess) return e;
    return launch_stage(stage, h->lat, h->delta, h->p, hs, X, F, out, coef, h->stream, 2);
}

// ---------------------------------------------------------------------------
// API
// ---------------------------------------------------------------------------
extern "C" {

const char *dugks_strerror(int code)
{
    switch (code) {
    case DUGKS_OK: return "ok";
    case DUGKS_EINVAL: return "invalid argument";
    case DUGKS_EUNSTABLE: return "dt/tau above the stability bound 12";
    case DUGKS_EMOMENT: return "weights are not moment-exact";
    case DUGKS_ENOMEM: return "out of memory";
    case DUGKS_EDEVICE: return "HIP runtime error";
    case DUGKS_ENONFINITE: return "non-finite state";
    case DUGKS_ENOTSUP: return "not supported";
    default: return "unknown error";
    }
}

const char *dugks_last_error_message(void) { return g_err.c_str(); }

int dugks_destroy(dugks_t *h)
{
    if (!h) return DUGKS_OK;
    if (h->batch) {
        for (auto &pe : h->batch->exec)
            for (auto &e : pe)
                if (e) (void)hipGraphExecDestroy(e);
        for (dugks *c : h->batch->inst) dugks_destroy(c);
        for (void *p : h->batch->allocs) (void)hipFree(p);
        delete h->batch;
    }
    for (auto &e : h->ev) (void)hipEventDestroy(e);
    for (auto &e : h->step_exec)
        if (e) (void)hipGraphExecDestroy(e);
    if (h->adj_ws || (h->alloc_fn && !h->allocs.empty())) (void)hipStreamSynchronize(h->stream);
    dev_put(h, h->adj_ws);
    for (void *p : h->allocs) dev_put(h, p);
    delete h;
    return DUGKS_OK;
}

static int validate(const dugks_desc *d)
{
    if (!d) return fail(DUGKS_EINVAL, "null descriptor");
    if (d->nx < 3 || d->ny < 3) return fail(DUGKS_EINVAL, "nx and ny must be >= 3");
    if (!d->xf || !d->yf || !d->xi || !d->w) return fail(DUGKS_EINVAL, "null grid or velocity array");
    if (d->nq < 1) return fail(DUGKS_EINVAL, "nq must be >= 1");
    if (d->scheme != DUGKS_SCHEME_T3S3 && d->scheme != DUGKS_SCHEME_T2S3)
        return fail(DUGKS_EINVAL, "unknown scheme");
    for (int i = 0; i < d->nx; i++)
        if (!(d->xf[i + 1] > d->xf[i])) return fail(DUGKS_EINVAL, "xf not increasing");
    for (int j = 0; j < d->ny; j++)
        if (!(d->yf[j + 1] > d->yf[j])) return fail(DUGKS_EINVAL, "yf not increasing");
    if (!(d->RT > 0) || !(d->dt > 0)) return fail(DUGKS_EINVAL, "RT and dt must be > 0");
    for (int k = 0; k < 4; k++)
        if (d->bc[k] < 0 || d->bc[k] > 2) return fail(DUGKS_EINVAL, "unknown boundary kind");
    if ((d->bc[0] == DUGKS_BC_PERIODIC) != (d->bc[1] == DUGKS_BC_PERIODIC) ||
        (d->bc[2] == DUGKS_BC_PERIODIC) != (d->bc[3] == DUGKS_BC_PERIODIC))
        return fail(DUGKS_EINVAL, "periodic sides must be paired");
    if (d->precision != DUGKS_FP64 && d->precision != DUGKS_FP32_DELTA)
        return fail(DUGKS_EINVAL, "unknown precision");
    if (d->reconstruction < DUGKS_RECON_POINT || d->reconstruction > DUGKS_RECON_S2)
        return fail(DUGKS_EINVAL, "unknown reconstruction");
    if (d->family_a != 0.0 && !(d->family_a >= 1.0 / 3.0 && d->family_a <= 0.5))
        return fail(DUGKS_EINVAL, "family_a must be 0 or lie in [1/3, 1/2]");
    if (d->family_a != 0.0 && d->scheme == DUGKS_SCHEME_T2S3)
        return fail(DUGKS_EINVAL, "family_a is a parameter of the third-order scheme");
    if (!d->tau && !(d->tau0 > 0) && !(d->kn > 0 && d->l_ref > 0))
        return fail(DUGKS_EINVAL, "no relaxation time: tau, tau0 > 0 or kn and l_ref > 0");
    if ((d->dev_alloc == nullptr) != (d->dev_free == nullptr))
        return fail(DUGKS_EINVAL, "dev_alloc and dev_free go together");
    // CFL: the characteristic foot point must stay within the upwind cell's stencil
    double cmax = 0;
    for (int q = 0; q < 2 * d->nq; q++) cmax = std::fmax(cmax, std::fabs(d->xi[q]));
    double dmin = 1e300;
    for (int i = 0; i < d->nx; i++) dmin = std::fmin(dmin, d->xf[i + 1] - d->xf[i]);
    for (int j = 0; j < d->ny; j++) dmin = std::fmin(dmin, d->yf[j + 1] - d->yf[j]);
    if (cmax * d->dt > dmin * (1.0 + 1e-12)) return fail(DUGKS_EINVAL, "CFL number above 1");
    return DUGKS_OK;
}

// T3S3 is stable for dt/tau <= 12 (the von Neumann bound of the paper's
// homogeneous factor at a = 1/3, with the interface terms left out).  The T2
// step's own factor (2 tau - dt)/(2 tau + dt) has no bound, but with the
// third-order interface expansion the whole T2S3 step does: in the Re-100
// cavity it holds to dt/tau = 9 at CFL 1.  Both schemes take the same guard,
// which is necessary, not sufficient, near CFL 1.
static int check_tau(const double *tau, long long n, double tau0, double dt)
{
    const double bound = 12.0 * (1 + 1e-12);
    if (tau) {
        for (long long k = 0; k < n; k++) {
            if (!(tau[k] > 0)) return fail(DUGKS_EINVAL, "tau must be > 0");
            if (dt / tau[k] > bound) return fail(DUGKS_EUNSTABLE, "dt/tau > 12");
        }
    } else {
        if (!(tau0 > 0)) return fail(DUGKS_EINVAL, "tau0 must be > 0");
        if (dt / tau0 > bound) return fail(DUGKS_EUNSTABLE, "dt/tau > 12");
    }
    return DUGKS_OK;
}

// Ring tiles of the any-size kernels, in order of preference.  A block of
// tx x ty threads covers (tx - 2) x (ty - 2) cells; every shape here spends
// about 1.31 threads per cell, so the best shape for a grid is the one that
// launches the fewest threads (the least padding at the east and north ends).
static const int kLqTiles[][2] = {{18, 14}, {14, 18}, {16, 16}, {20, 12}, {12, 20}};
constexpr int LQ_DEFAULT_TILE = 16;

static long long lq_tile_threads(int nx, int ny, int tx, int ty)
{
    return (long long)((nx + tx - 3) / (tx - 2)) * ((ny + ty - 3) / (ty - 2)) * tx * ty;
}

// the shape of kLqTiles with the fewest launched threads over the grids
// {nx, ny, nq} (weighted by their velocity counts)
static void lq_pick_tile(const std::vector<std::array<int, 3>> &grids, int &tx, int &ty)
{
    long long best = -1;
    for (const auto &t : kLqTiles) {
        long long c = 0;
        for (const auto &g : grids) c += lq_tile_threads(g[0], g[1], t[0], t[1]) * g[2];
        if (best < 0 || c < best) {
            best = c;
            tx = t[0];
            ty = t[1];
        }
    }
}

int dugks_create(const dugks_desc *din, dugks_t **out)
{
    if (!out) return fail(DUGKS_EINVAL, "null output handle");
    *out = nullptr;
    int rc = validate(din);
    if (rc) return rc;
    // relaxation time from the Knudsen number (paper, "Numerical tests":
    // lambda = tau sqrt(pi RT / 2) and Kn = lambda / L)
    dugks_desc dl = *din;
    if (!dl.tau && !(dl.tau0 > 0)) dl.tau0 = dl.kn * dl.l_ref / std::sqrt(M_PI * dl.RT / 2.0);
    const dugks_desc *d = &dl;
    const long long ncell = (long long)d->nx * d->ny;
    if ((rc = check_tau(d->tau, ncell, d->tau0, d->dt))) return rc;
    const int nq = d->nq;
    const double *xi = d->xi, *eta = d->xi + nq;

    // weight moments
    double M0 = 0, M1x = 0, M1y = 0, Mxx = 0, Myy = 0, Mxy = 0;
    for (int q = 0; q < nq; q++) {
        M0 += d->w[q];
        M1x += d->w[q] * xi[q];
        M1y += d->w[q] * eta[q];
        Mxx += d->w[q] * xi[q] * xi[q];
        Myy += d->w[q] * eta[q] * eta[q];
        Mxy += d->w[q] * xi[q] * eta[q];
    }
    const double defect = std::fmax(std::fmax(std::fabs(M0 - 1), std::fabs(Mxx / d->RT - 1)),
                                    std::fmax(std::fabs(Myy / d->RT - 1), std::fabs(Mxy / d->RT)));
    if (defect > 1e-10 && !(d->flags & DUGKS_ALLOW_MOMENT_DEFECT))
        return fail(DUGKS_EMOMENT, "weight moment defect " + std::to_string(defect));

    // walls need mirrors (bounce-back) / nonzero leaving flux (diffuse)
    std::vector<int> opp(nq, -1);
    double cm = 0;
    for (int q = 0; q < nq; q++) cm = std::fmax(cm, std::fmax(std::fabs(xi[q]), std::fabs(eta[q])));
    for (int q = 0; q < nq; q++)
        for (int r = 0; r < nq; r++)
            if (std::fabs(xi[q] + xi[r]) <= 1e-12 * cm && std::fabs(eta[q] + eta[r]) <= 1e-12 * cm) {
                opp[q] = r;
                break;
            }
    bool any_bb = false;
    for (int k = 0; k < 4; k++) any_bb |= d->bc[k] == DUGKS_BC_BOUNCE_BACK;
    if (any_bb)
        for (int q = 0; q < nq; q++)
            if (opp[q] < 0 || std::fabs(d->w[opp[q]] - d->w[q]) > 1e-14 * std::fabs(d->w[q]))
                return fail(DUGKS_EINVAL, "bounce-back needs a mirror velocity with equal weight");

    dugks *h = new dugks();
    h->stream = (hipStream_t)d->stream;
    h->hxi.assign(d->xi, d->xi + 2 * (size_t)nq);
    h->alloc_fn = d->dev_alloc;
    h->free_fn = d->dev_free;
    h->alloc_ctx = d->alloc_ctx;
    h->delta = d->precision == DUGKS_FP32_DELTA;
    h->elem = h->delta ? 4 : 8;
    SweepParams &p = h->p;
    p.nx = d->nx;
    p.ny = d->ny;
    p.ncell = ncell;
    p.t2 = d->scheme == DUGKS_SCHEME_T2S3;
    // variants of the method run the kernels of variant.hip
    const double fam_a = d->family_a != 0.0 ? d->family_a : 1.0 / 3.0;
    h->var = fam_a != 1.0 / 3.0 || d->reconstruction != DUGKS_RECON_POINT;
    p.state_m = p.t2 ? 2.0 : (h->var ? 1.0 / var_family(fam_a, d->dt).Pn1 : 4.0);
    p.perx = d->bc[0] == DUGKS_BC_PERIODIC;
    p.pery = d->bc[2] == DUGKS_BC_PERIODIC;
    p.nq = nq;
    p.RT = d->RT;
    p.dt = d->dt;
    p.rho0 = h->delta ? d->rho0 : 0.0;
    if (h->delta && !(d->rho0 > 0)) {
        delete h;
        return fail(DUGKS_EINVAL, "FP32-delta storage needs rho0 > 0");
    }
    p.M0m1 = M0 - 1.0;
    p.M1x = M1x;
    p.M1y = M1y;
    p.kappa = d->taylor_quad > 0 ? d->taylor_quad : 1.0;
    p.tau0 = d->tau0;
    p.tau_field = d->tau != nullptr;
    for (int k = 0; k < 4; k++) {
        p.bc[k] = d->bc[k];
        p.uw[k][0] = d->u_wall[k][0];
        p.uw[k][1] = d->u_wall[k][1];
    }

    // lattice
    double c = 0;
    const bool force_generic = d->flags & DUGKS_FORCE_GENERIC;
    if (!force_generic && match_lattice(d->xi, nq, kD2Q9x, kD2Q9y, 9, c)) h->lat = 9;
    else if (!force_generic && match_lattice(d->xi, nq, kD2Q37x, kD2Q37y, 37, c)) h->lat = 37;
    else {
        h->lat = 0;
        c = 1.0;
        if (any_bb) {
            delete h;
            return fail(DUGKS_ENOTSUP, "bounce-back walls need the D2Q9 / D2Q37 lattice kernels");
        }
    }
    p.clat = c;
    p.nxcd = 8;   // MI355X: 8 XCDs
    if (const char *e = getenv("DUGKS_NXCD")) p.nxcd = std::max(1, atoi(e));   // tuning knob
    p.iRT = 1.0 / d->RT;
    {
        // coefficients of a uniform tau (used when no tau field is given);
        // stage A of T3S3 reconstructs over dt/6, the T2S3 step over dt/2
        const double t = d->tau0, dt = d->dt, h1 = p.t2 ? 0.5 * dt : dt / 6.0, h2 = 5.0 * dt / 12.0;
        UniformCoef &u = p.uc;
        const Stage0Coef c0 = stage0_coef(p.t2 != 0, t, dt);
        u.cc[0] = c0.cc;
        u.ce[0] = c0.ce;
        u.kx0 = c0.kx;
        u.ke0 = c0.ke;
        u.aL0 = p.t2 ? dt : dt / 3.0;
        u.cc[1] = (24.0 * t - 5.0 * dt) / (24.0 * t + 4.0 * dt);
        u.ce[1] = 9.0 * dt / (24.0 * t + 4.0 * dt);
        u.c1 = u.cc[0];
        u.e1 = u.ce[0];
        const double kw = 6.0 * dt / (6.0 * t + dt);
        u.a_f = (4.0 - 6.0 * u.c1) / 7.0;
        u.a_En = -6.0 / 7.0 * u.e1;
        u.a_G = 9.0 / 7.0 - 0.75 * kw;
        u.a_Ep = 0.75 * kw;
        u.alpha[0] = 2.0 * t / (2.0 * t + h1);
        u.beta[0] = h1 / (2.0 * t + h1);
        u.alpha[1] = 2.0 * t / (2.0 * t + h2);
        u.beta[1] = h2 / (2.0 * t + h2);
    }

    // tile
    int dlx = h->lat == 37 && !h->delta ? 16 : 32;
    int dly = h->lat == 37 && !h->delta ? 16 : 8;
    if (h->lat == 0) lq_pick_tile({{d->nx, d->ny, nq}}, dlx, dly);
    const int lx = d->tile_x > 0 ? d->tile_x : dlx;
    const int ly = d->tile_y > 0 ? d->tile_y : dly;
    const int maxthr = h->lat == 0 ? 256 : 512;
    if (lx * ly > maxthr || lx * ly < 64 || lx < 2 || ly < 2) {
        delete h;
        return fail(DUGKS_EINVAL, "tile must hold 64..512 cells (64..256 for any-size velocity sets)");
    }
    p.tile_x = lx;
    p.tile_y = ly;
    if (h->lat == 0) {
        // ring tiles (one block covers (lx - 2) x (ly - 2) cells); chunks: enough
        // workgroups to fill the chip, at least 16 velocities each
        if (lx < 4 || ly < 4 || (lx + 2) * (ly + 2) > 2 * lx * ly) {
            delete h;
            return fail(DUGKS_EINVAL, "any-size velocity sets need tiles of at least 4 x 4 threads");
        }
        p.lq_qs = h->delta ? 4 : 2;
        // Velocity chunks: at least two rounds of the blocks the chip holds at
        // once, and a chunk count whose last round is as full as possible
        // (every block of a kernel costs about the same).
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
            ncu = 256;
        const long long slots_f =
            (long long)ncu * lq_blocks_per_cu(h->delta, true, lx * ly, lq_smem_bytes(p, h->delta));
        const long long slots_u = (long long)ncu * lq_blocks_per_cu(h->delta, false, 256, 0);
        // per: blocks per chunk; chunk lengths are multiples of step and at least minq
        auto pick = [&](long long per, long long slots, int step, int minq) {
            const long long nmax = std::max(1, nq / minq);
            const long long nlo = std::min(nmax, std::max(1LL, (2 * slots + per - 1) / per));
            const long long nhi = std::min(nmax, 3 * nlo);
            int best = 0;
            double best_eff = -1.0;
            for (long long nch = nlo; nch <= nhi; nch++) {
                int c = (int)((nq + nch - 1) / nch);
                c = (c + step - 1) / step * step;
                const long long blocks = per * ((nq + c - 1) / c);
                const long long rounds = (blocks + slots - 1) / slots;
                const double eff = (double)blocks / (double)(rounds * slots);
                if (eff > best_eff + 1e-9) { best_eff = eff; best = c; }
            }
            return best;
        };
        p.lq_chunk = pick(lq_ntile(p), slots_f, p.lq_qs, 16);
        p.lq_nchunk = (nq + p.lq_chunk - 1) / p.lq_chunk;
        p.lq_uchunk = pick((ncell + 255) / 256, slots_u, 4, 32);
        p.lq_nuchunk = (nq + p.lq_uchunk - 1) / p.lq_uchunk;
    }
    // lattice kernels: one plane of the tile and its halo per velocity, plus one
    // spare element per plane (compile-time-shape kernels)
    const size_t smem = h->lat == 0 ? lq_smem_bytes(p, h->delta)
                                    : h->elem * nq * ((size_t)(lx + 4) * (ly + 4) + 1);
    if (smem > 160 * 1024) {
        delete h;
        return fail(DUGKS_EINVAL, "tile too large for LDS");
    }
    {
        // the dynamic-LDS limit is a per-kernel attribute: only ever raise it
        static size_t raised[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        size_t &mx = raised[h->lat == 0 ? 0 : (h->lat == 9 ? 1 : 2)][h->delta ? 1 : 0];
        hipError_t e = hipSuccess;
        if (smem > mx) {
            e = h->lat == 0 ? set_lq_smem(h->delta, smem) : set_stage_smem(h->lat, h->delta, smem);
            if (e == hipSuccess) mx = smem;
        }
        if (e != hipSuccess) {
            delete h;
            return fail(DUGKS_EDEVICE, std::string("LDS size: ") + hipGetErrorString(e));
        }
    }

    p.ncell_f = p.ncell_o = ncell;
    if (h->lat && fast_tile_index(lx, ly) >= 0) {
        // the compile-time-shape kernels take the weights per velocity shell and
        // address planes with 32-bit byte offsets
        bool ok = ncell * (long long)h->elem < (1LL << 32);
        for (int q = 0; q < nq && ok; q++) {
            const int sh = h->lat == 9 ? LatD2Q9::shell(q) : LatD2Q37::shell(q);
            double &w1 = p.wtab[sh][1];
            if (w1 == 0.0) w1 = d->w[q];
            else ok = std::fabs(d->w[q] - w1) <= 1e-14 * std::fabs(w1);
        }
        for (int sh = 0; sh < 8; sh++)
            for (int m = 0; m < 4; m++) p.wtab[sh][m] = m * p.wtab[sh][1];
        if (ok) {
            if ((rc = raise_fast_smem(h->lat, h->delta, lx, ly, smem))) {
                delete h;
                return rc;
            }
            h->fast_ct = true;
        }
    }

    // grid
    const bool unif = is_uniform(d->xf, d->nx) && is_uniform(d->yf, d->ny);
    p.uniform = unif;
    if (h->var && (!unif || h->delta || !p.perx || !p.pery)) {
        delete h;
        return fail(DUGKS_ENOTSUP, "the scheme and reconstruction variants run FP64 on uniform periodic grids");
    }
    p.inv_dx = 1.0 / (d->xf[1] - d->xf[0]);
    p.inv_dy = 1.0 / (d->yf[1] - d->yf[0]);
    std::vector<double> dxl, dxr, sxd1, sxd2, ixd, dyl, dyr, syd1, syd2, iyd;
    std::vector<int> sxo, syo;
    axis_tables(d->xf, d->nx, p.perx, dxl, dxr, sxo, sxd1, sxd2, ixd);
    axis_tables(d->yf, d->ny, p.pery, dyl, dyr, syo, syd1, syd2, iyd);
    // first device work of the handle: the device it lives on, and that
    // device's address of the no-allocation scratch
    if (hipGetDevice(&h->device) != hipSuccess) {
        dugks_destroy(h);
        return fail(DUGKS_EDEVICE, "hipGetDevice failed");
    }
    if ((rc = scratch_resolve(h->device))) { dugks_destroy(h); return rc; }
#define UP(vec, dst)                                                        \
    if ((rc = upload(h, vec.data(), vec.size(), &dst))) { dugks_destroy(h); return rc; }
    UP(dxl, p.g.dxl) UP(dxr, p.g.dxr) UP(dyl, p.g.dyl) UP(dyr, p.g.dyr)
    UP(sxo, p.g.sx_off) UP(syo, p.g.sy_off)
    UP(sxd1, p.g.sx_d1) UP(sxd2, p.g.sx_d2) UP(syd1, p.g.sy_d1) UP(syd2, p.g.sy_d2)
    UP(ixd, p.g.inv_dx) UP(iyd, p.g.inv_dy)
    std::vector<double> vxi(xi, xi + nq), veta(eta, eta + nq), vw(d->w, d->w + nq);
    UP(vxi, p.xi) UP(veta, p.eta) UP(vw, p.w) UP(opp, p.opp)
    {
        // per-velocity moment weights in lattice units (e = xi / clat)
        std::vector<double> wm(3 * (size_t)nq);
        for (int q = 0; q < nq; q++) {
            const double w0 = h->delta ? d->w[q] : 1.0;
            wm[3 * q] = w0;
            wm[3 * q + 1] = w0 * std::round(xi[q] / c);
            wm[3 * q + 2] = w0 * std::round(eta[q] / c);
        }
        UP(wm, p.wmom)
    }
    std::vector<double> lw, md;   // any-size tables, also packed into records below
    std::vector<int> sg, gnz;
    if (h->lat == 0) {
        // any-size kernels: moment weights and monomials of every velocity
        lw.assign(7 * (size_t)nq, 0.0);
        md.assign(9 * (size_t)nq, 0.0);
        for (int q = 0; q < nq; q++) {
            const double m = h->delta ? d->w[q] : 1.0, x = xi[q], y = eta[q];
            lw[7 * q] = m;
            lw[7 * q + 1] = m * x;
            lw[7 * q + 2] = m * y;
            // weights of the flux arriving at a west, east, south, north wall
            lw[7 * q + 3] = m * std::max(-x, 0.0);
            lw[7 * q + 4] = m * std::max(x, 0.0);
            lw[7 * q + 5] = m * std::max(-y, 0.0);
            lw[7 * q + 6] = m * std::max(y, 0.0);
            const double mono[9] = {x, y, x * x, x * y, y * y, x * x * x, x * x * y, x * y * y, y * y * y};
            for (int k = 0; k < 9; k++) md[9 * q + k] = mono[k];
        }
        sg.assign(nq, 0);
        for (int q = 0; q < nq; q++)
            sg[q] = (xi[q] > 0 ? 1 : 0) | (xi[q] < 0 ? 2 : 0) | (eta[q] > 0 ? 4 : 0) | (eta[q] < 0 ? 8 : 0);
        gnz.assign(nq / p.lq_qs + 1, 0);
        for (int g = 0; g * p.lq_qs + p.lq_qs <= nq; g++) {
            int ok = 1;
            for (int k = 0; k < p.lq_qs; k++) {
                const int q = g * p.lq_qs + k;
                ok &= (xi[q] != 0.0) && (eta[q] != 0.0);
            }
            gnz[g] = ok;
        }
    }
    if (d->tau) {
        std::vector<double> vt(d->tau, d->tau + ncell);
        UP(vt, p.tau)
    }

    // diffuse-wall tables
    std::vector<double> wallE(4 * (size_t)nq, 0.0);
    for (int k = 0; k < 4; k++) {
        const double nxw = k == 0 ? -1.0 : k == 1 ? 1.0 : 0.0;
        const double nyw = k == 2 ? -1.0 : k == 3 ? 1.0 : 0.0;
        const double ux = d->u_wall[k][0], uy = d->u_wall[k][1];
        double den = 0, off = 0, m0 = 0, mx = 0, my = 0, w0 = 0, wx = 0, wy = 0;
        for (int q = 0; q < nq; q++) {
            const double eu = xi[q] * ux + eta[q] * uy, uu = ux * ux + uy * uy;
            const double P = 1.0 + eu / d->RT + eu * eu / (2 * d->RT * d->RT) - uu / (2 * d->RT);
            wallE[(size_t)k * nq + q] = h->delta ? P : d->w[q] * P;
            const double xn = xi[q] * nxw + eta[q] * nyw;
            if (xn < 0) {
                den += -xn * d->w[q] * P;
                m0 += d->w[q] * P;
                mx += xi[q] * d->w[q] * P;
                my += eta[q] * d->w[q] * P;
                w0 += d->w[q];
                wx += xi[q] * d->w[q];
                wy += eta[q] * d->w[q];
            } else if (xn > 0) {
                off += xn * d->w[q];
            }
        }
        p.ds_den[k] = den;
        p.ds_num_off[k] = h->delta ? d->rho0 * off : 0.0;
        p.ds_m[k][0] = m0; p.ds_m[k][1] = mx; p.ds_m[k][2] = my;
        p.ds_w[k][0] = w0; p.ds_w[k][1] = wx; p.ds_w[k][2] = wy;
        if (d->bc[k] == DUGKS_BC_DIFFUSE && !(den > 0)) {
            dugks_destroy(h);
            return fail(DUGKS_EINVAL, "diffuse wall with no leaving velocity");
        }
    }
    UP(wallE, p.wall_E)
    if (h->lat == 0) {
        // packed per-velocity records in the storage precision
        auto fill = [&](auto &rec) {
            using S = decltype(rec[0].wq);
            for (int q = 0; q < nq; q++) {
                auto &r = rec[q];
                r.sg = sg[q];
                r.gnz = gnz[q / p.lq_qs];
                for (int k = 0; k < 9; k++) r.mono[k] = (S)md[9 * q + k];
                r.wq = (S)d->w[q];
                for (int k = 0; k < 4; k++) r.we[k] = (S)wallE[(size_t)k * nq + q];
                for (int k = 0; k < 7; k++) r.wm[k] = lw[7 * q + k];
            }
        };
        if (h->delta) {
            std::vector<QRec<float>> rec(nq);
            fill(rec);
            const QRec<float> *dp = nullptr;
            UP(rec, dp)
            p.lq_rec = dp;
        } else {
            std::vector<QRec<double>> rec(nq);
            fill(rec);
            const QRec<double> *dp = nullptr;
            UP(rec, dp)
            p.lq_rec = dp;
        }
    }

    // fast-path coefficients of both stages
    h->h1 = p.t2 ? 0.5 * d->dt : d->dt / 6.0;
    h->h2 = 5.0 * d->dt / 12.0;
    {
        const double dx = d->xf[1] - d->xf[0], dy = d->yf[1] - d->yf[0];
        std::vector<double> cA = fast_coefs(d->xi, nq, dx, dy, h->h1, p.kappa);
        std::vector<double> cC = fast_coefs(d->xi, nq, dx, dy, h->h2, p.kappa);
        if (h->delta) {
            std::vector<float> fA(cA.begin(), cA.end()), fC(cC.begin(), cC.end());
            const float *a, *b;
            UP(fA, a) UP(fC, b)
            h->coefA = (void *)a;
            h->coefC = (void *)b;
        } else {
            const double *a, *b;
            UP(cA, a) UP(cC, b)
            h->coefA = (void *)a;
            h->coefC = (void *)b;
        }
    }
#undef UP

    // state buffers
    const size_t bytes = h->elem * (size_t)nq * ncell;
    if ((rc = dalloc(h, &h->state[0], bytes)) || (rc = dalloc(h, &h->state[1], bytes)) ||
        (rc = dalloc(h, &h->G, bytes))) {
        dugks_destroy(h);
        return rc;
    }
    if (h->lat == 0) {
        const size_t nface = (size_t)(d->nx + 1) * d->ny + (size_t)d->nx * (d->ny + 1);
        void *a = nullptr, *b = nullptr, *fp = nullptr, *fm = nullptr, *cp = nullptr;
        if ((rc = dalloc(h, &a, 32 * (size_t)ncell)) || (rc = dalloc(h, &b, 32 * (size_t)ncell)) ||
            (rc = dalloc(h, &fp, 32 * nface * p.lq_nchunk)) || (rc = dalloc(h, &fm, 64 * nface)) ||
            (rc = dalloc(h, &cp, 32 * (size_t)ncell * p.lq_nuchunk))) {
            dugks_destroy(h);
            return rc;
        }
        void *fx = nullptr, *fy = nullptr;
        if ((rc = dalloc(h, &fx, h->elem * (size_t)nq * (d->nx + 1) * d->ny)) ||
            (rc = dalloc(h, &fy, h->elem * (size_t)nq * d->nx * (d->ny + 1)))) {
            dugks_destroy(h);
            return rc;
        }
        h->fxv = fx;
        h->fyv = fy;
        h->mom_state = (double *)a;
        h->mom_G = (double *)b;
        h->face_part = (double *)fp;
        h->face_mom = (double *)fm;
        h->cell_part = (double *)cp;
    }
    if (h->var) {
        const int npt = d->reconstruction == DUGKS_RECON_CELL_AVERAGE ? 2 : 1;
        const size_t qn = sizeof(double) * (size_t)nq * ncell;
        void *vB, *vG, *vL, *vM0, *vM1, *vFx, *vFy;
        if ((rc = dalloc(h, &vB, qn)) || (rc = dalloc(h, &vG, qn)) || (rc = dalloc(h, &vL, qn)) ||
            (rc = dalloc(h, &vM0, 3 * sizeof(double) * ncell)) || (rc = dalloc(h, &vM1, 3 * sizeof(double) * ncell)) ||
            (rc = dalloc(h, &vFx, npt * qn)) || (rc = dalloc(h, &vFy, npt * qn))) {
            dugks_destroy(h);
            return rc;
        }
        h->vb = VarBuffers{(double *)vB, (double *)vG, (double *)vL, (double *)vM0, (double *)vM1, (double *)vFx,
                           (double *)vFy};
        VarArgs &a = h->va;
        a.nx = d->nx;
        a.ny = d->ny;
        a.nq = nq;
        a.n = ncell;
        a.dx = d->xf[1] - d->xf[0];
        a.dy = d->yf[1] - d->yf[0];
        a.RT = d->RT;
        a.xi = p.xi;
        a.eta = p.eta;
        a.w = p.w;
        a.tau = p.tau_field ? p.tau : nullptr;
        a.tau0 = p.tau0;
        a.recon = d->reconstruction;
        a.kappa = p.kappa;
        h->vf = var_family(fam_a, d->dt);
    }
    void *bad = nullptr;
    if ((rc = dalloc(h, &bad, sizeof(int)))) { dugks_destroy(h); return rc; }
    h->d_bad = (int *)bad;
    p.bad = h->d_bad;
    h->va.bad = h->d_bad;
    HIPCHECK(hipMemset(h->d_bad, 0, sizeof(int)));
    char buf[160];
    if (h->var)
        snprintf(buf, sizeof buf, "variant %s a=%.6g reconstruction %s, Q=%d fp64 (variant.hip)",
                 p.t2 ? "T2" : "T3 family", fam_a,
                 d->reconstruction == DUGKS_RECON_POINT ? "point/midpoint"
                 : d->reconstruction == DUGKS_RECON_CELL_AVERAGE ? "cell-average/two-point Gauss" : "S2",
                 nq);
    else if (h->lat)
        snprintf(buf, sizeof buf, "lattice D2Q%d %s tile %dx%d %s", h->lat, h->delta ? "fp32-delta" : "fp64",
                 lx, ly, unif ? "uniform" : "non-uniform");
    else
        snprintf(buf, sizeof buf,
                 "any-size Q=%d %s tile %dx%d, %d chunks of %d velocities (update: %d of %d), %s", nq,
                 h->delta ? "fp32-delta" : "fp64", lx, ly, p.lq_nchunk, p.lq_chunk, p.lq_nuchunk, p.lq_uchunk,
                 unif ? "uniform" : "non-uniform");
    h->variant = buf;
    *out = h;
    return DUGKS_OK;
}

int dugks_describe(dugks_t *h, char *buf, int len)
{
    if (!h || !buf || len <= 0) return fail(DUGKS_EINVAL, "bad arguments");
    snprintf(buf, len, "%s", h->variant.c_str());
    return DUGKS_OK;
}

// staging helper: device copy of a host array (or the device pointer itself)
struct Staged {
    double *dev = nullptr;
    bool owned = false;
    ~Staged() { if (owned) (void)hipFree(dev); }
};

static int stage_in(const double *src, size_t count, int mem, Staged &s, hipStream_t st)
{
    if (mem == DUGKS_MEM_DEVICE) {
        s.dev = const_cast<double *>(src);
        return DUGKS_OK;
    }
    if (mem != DUGKS_MEM_HOST) return fail(DUGKS_EINVAL, "mem must be host or device");
    hipError_t e = hipMalloc((void **)&s.dev, sizeof(double) * (count ? count : 1));
    if (e != hipSuccess) return fail(DUGKS_ENOMEM, "staging buffer");
    s.owned = true;
    HIPCHECK(hipMemcpyAsync(s.dev, src, sizeof(double) * count, hipMemcpyHostToDevice, st));
    return DUGKS_OK;
}

int dugks_set_state(dugks_t *h, const double *f, int mem)
{
    if (!h || !f) return fail(DUGKS_EINVAL, "null argument");
    Staged s;
    int rc = stage_in(f, (size_t)h->p.nq * h->p.ncell, mem, s, h->stream);
    if (rc) return rc;
    HIPCHECK(launch_set_state(h->p, h->delta, s.dev, h->state[h->cur], h->stream));
    if (h->lat == 0) HIPCHECK(launch_state_moments(h->p, h->delta, h->state[h->cur], h->mom_state, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    return DUGKS_OK;
}

int dugks_init_equilibrium(dugks_t *h, const double *rho, const double *ux, const double *uy,
                           int mem)
{
    if (!h || !rho || !ux || !uy) return fail(DUGKS_EINVAL, "null argument");
    Staged a, b, c;
    const size_t n = h->p.ncell;
    int rc;
    if ((rc = stage_in(rho, n, mem, a, h->stream)) || (rc = stage_in(ux, n, mem, b, h->stream)) ||
        (rc = stage_in(uy, n, mem, c, h->stream)))
        return rc;
    HIPCHECK(launch_init_eq(h->p, h->delta, a.dev, b.dev, c.dev, h->state[h->cur], h->stream));
    if (h->lat == 0) HIPCHECK(launch_state_moments(h->p, h->delta, h->state[h->cur], h->mom_state, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    return DUGKS_OK;
}

static int record(dugks *h, int kind, bool start)
{
    if (!h->prof_on || h->prof_n >= h->prof_max) return DUGKS_OK;
    const int k = h->prof_n;
    HIPCHECK(hipEventRecord(h->ev[2 * k + (start ? 0 : 1)], h->stream));
    if (!start) {
        h->ev_kind[k] = kind;
        h->prof_n++;
    }
    return DUGKS_OK;
}

// One stage of the any-size kernels.  While profiling, the faces and the
// update kernel are timed on their own; otherwise the whole stage is one
// STAGE_A / STAGE_C record.
static int lq_stage(dugks *h, const LQStage &a)
{
    int rc;
    if (!h->prof_on) {
        HIPCHECK(launch_lq_stage(h->delta, h->p, a, h->stream, -1));
        return DUGKS_OK;
    }
    if ((rc = record(h, KC_LQ_FACES, true))) return rc;
    HIPCHECK(launch_lq_stage(h->delta, h->p, a, h->stream, 0));
    if ((rc = record(h, KC_LQ_FACES, false))) return rc;
    HIPCHECK(launch_lq_stage(h->delta, h->p, a, h->stream, 1));
    if ((rc = record(h, KC_LQ_UPDATE, true))) return rc;
    HIPCHECK(launch_lq_stage(h->delta, h->p, a, h->stream, 2));
    if ((rc = record(h, KC_LQ_UPDATE, false))) return rc;
    HIPCHECK(launch_lq_stage(h->delta, h->p, a, h->stream, 3));
    return DUGKS_OK;
}

static int batch_step(dugks_t *h, int nsteps);

// One step of a single handle on its own stream (lattice, any-size or
// variant kernels); with timing on, each stage (or kernel) gets its events.
static int step_once(dugks *h)
{
    void *X = h->state[h->cur], *Y = h->state[1 - h->cur];
    int rc;
    const bool whole = h->lat || h->var || !h->prof_on;   // stage records (else per-kernel ones)
    if (h->var) {
        if (whole && (rc = record(h, KC_STAGE_A, true))) return rc;
        HIPCHECK(variant_step(h->va, h->vf, h->p.t2 != 0, (const double *)X, (double *)Y, h->vb, h->stream));
        if (whole && (rc = record(h, KC_STAGE_A, false))) return rc;
        return DUGKS_OK;
    }
    if (h->p.t2) {
        // T2S3: one stage-A-shaped sweep from ftilde(t_n) to ftilde(t_n + dt)
        if (whole && (rc = record(h, KC_STAGE_A, true))) return rc;
        if (h->lat) {
            HIPCHECK(lattice_stage(h, 0, X, nullptr, Y));
        } else {
            if ((rc = lq_stage(h, lq_args(h, 0, X, nullptr, Y)))) return rc;
            // the cell reduction wrote the moments of Y into the stage-output slot
            std::swap(h->mom_state, h->mom_G);
        }
        if (whole && (rc = record(h, KC_STAGE_A, false))) return rc;
        return DUGKS_OK;
    }
    if (whole && (rc = record(h, KC_STAGE_A, true))) return rc;
    if (h->lat) {
        HIPCHECK(lattice_stage(h, 0, X, nullptr, h->G));
    } else {
        if ((rc = lq_stage(h, lq_args(h, 0, X, nullptr, h->G)))) return rc;
    }
    if (whole && (rc = record(h, KC_STAGE_A, false))) return rc;
    if (whole && (rc = record(h, KC_STAGE_C, true))) return rc;
    if (h->lat) {
        HIPCHECK(lattice_stage(h, 1, h->G, X, Y));
    } else {
        // the moments of fhat(t_n) are read by the update and overwritten by
        // the cell reduction that follows it on the same stream
        if ((rc = lq_stage(h, lq_args(h, 1, h->G, X, Y)))) return rc;
    }
    if (whole && (rc = record(h, KC_STAGE_C, false))) return rc;
    return DUGKS_OK;
}

// HIP graph of one step of a lattice handle from state[par] to state[1 - par]
static int step_graph(dugks *h, int par)
{
    if (h->step_exec[par]) return DUGKS_OK;
    hipStream_t s = h->stream;
    bool own = false;
    if (!s) {   // stream capture needs a real stream
        HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        own = true;
    }
    hipStream_t keep = h->stream;
    const int keep_cur = h->cur;
    h->stream = s;
    h->cur = par;
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = step_once(h);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    h->stream = keep;
    h->cur = keep_cur;
    if (own) (void)hipStreamDestroy(s);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(DUGKS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&h->step_exec[par], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->step_exec[par] = nullptr;
        return fail(DUGKS_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return DUGKS_OK;
}

int dugks_step(dugks_t *h, int nsteps)
{
    if (!h || nsteps < 0) return fail(DUGKS_EINVAL, "bad arguments");
    if (h->batch) return batch_step(h, nsteps);
    // lattice handles replay a captured step from the second call on (not
    // while kernel timing is on: the events go between the launches)
    const bool graph = h->lat && !h->var && !h->prof_on && h->step_calls > 0;
    if (nsteps > 0) h->step_calls++;
    int rc;
    for (int s = 0; s < nsteps; s++) {
        if (graph) {
            if ((rc = step_graph(h, h->cur))) return rc;
            HIPCHECK(hipGraphLaunch(h->step_exec[h->cur], h->stream));
        } else if ((rc = step_once(h))) {
            return rc;
        }
        h->cur = 1 - h->cur;
    }
    return DUGKS_OK;
}

static int stage_out(dugks *h, double *dst, size_t count, int mem, Staged &s)
{
    if (mem == DUGKS_MEM_DEVICE) {
        s.dev = dst;
        return DUGKS_OK;
    }
    if (mem != DUGKS_MEM_HOST) return fail(DUGKS_EINVAL, "mem must be host or device");
    hipError_t e = hipMalloc((void **)&s.dev, sizeof(double) * (count ? count : 1));
    if (e != hipSuccess) return fail(DUGKS_ENOMEM, "staging buffer");
    s.owned = true;
    return DUGKS_OK;
}

static int finish_out(dugks *h, double *dst, size_t count, int mem, Staged &s)
{
    if (mem == DUGKS_MEM_HOST) {
        HIPCHECK(hipMemcpyAsync(dst, s.dev, sizeof(double) * count, hipMemcpyDeviceToHost, h->stream));
        HIPCHECK(hipStreamSynchronize(h->stream));
    }
    return DUGKS_OK;
}

int dugks_moments(dugks_t *h, double *rho, double *ux, double *uy, int mem)
{
    if (!h) return fail(DUGKS_EINVAL, "null handle");
    const size_t n = h->p.ncell;
    Staged a, b, c;
    int rc;
    if ((rho && (rc = stage_out(h, rho, n, mem, a))) || (ux && (rc = stage_out(h, ux, n, mem, b))) ||
        (uy && (rc = stage_out(h, uy, n, mem, c))))
        return rc;
    HIPCHECK(launch_moments(h->p, h->delta, h->state[h->cur], a.dev, b.dev, c.dev, nullptr, h->stream));
    if (rho && (rc = finish_out(h, rho, n, mem, a))) return rc;
    if (ux && (rc = finish_out(h, ux, n, mem, b))) return rc;
    if (uy && (rc = finish_out(h, uy, n, mem, c))) return rc;
    return DUGKS_OK;
}

static int get_dist(dugks_t *h, double *f, int mem, int physical)
{
    if (!h || !f) return fail(DUGKS_EINVAL, "null argument");
    const size_t n = (size_t)h->p.nq * h->p.ncell;
    Staged s;
    int rc = stage_out(h, f, n, mem, s);
    if (rc) return rc;
    HIPCHECK(launch_get_state(h->p, h->delta, h->state[h->cur], s.dev, physical, h->stream));
    return finish_out(h, f, n, mem, s);
}

int dugks_get_state(dugks_t *h, double *f, int mem) { return get_dist(h, f, mem, 1); }
int dugks_get_fhat(dugks_t *h, double *f, int mem) { return get_dist(h, f, mem, 0); }

int dugks_set_tau(dugks_t *h, const double *tau, int mem)
{
    if (!h || !tau) return fail(DUGKS_EINVAL, "null argument");
    if (!h->p.tau_field) return fail(DUGKS_EINVAL, "handle was created with a uniform tau");
    const size_t n = h->p.ncell;
    std::vector<double> host(n);
    if (mem == DUGKS_MEM_DEVICE) {
        HIPCHECK(hipMemcpy(host.data(), tau, sizeof(double) * n, hipMemcpyDeviceToHost));
    } else {
        memcpy(host.data(), tau, sizeof(double) * n);
    }
    int rc = check_tau(host.data(), (long long)n, 0, h->p.dt);
    if (rc) return rc;
    HIPCHECK(hipMemcpyAsync((void *)h->p.tau, host.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                            h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    return DUGKS_OK;
}

int dugks_sync(dugks_t *h)
{
    if (!h) return fail(DUGKS_EINVAL, "null handle");
    if (h->batch) {
        HIPCHECK(hipStreamSynchronize(h->stream));
        for (dugks *c : h->batch->inst) {
            int rc = dugks_sync(c);
            if (rc) return rc;
        }
        return DUGKS_OK;
    }
    // the stage kernels raise the flag when they write a non-finite value
    int bad = 0;
    HIPCHECK(hipMemcpyAsync(&bad, h->d_bad, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    if (bad) {
        HIPCHECK(hipMemsetAsync(h->d_bad, 0, sizeof(int), h->stream));
        HIPCHECK(hipStreamSynchronize(h->stream));
        return fail(DUGKS_ENONFINITE, "non-finite value written by a stage since the last sync");
    }
    return DUGKS_OK;
}

int dugks_prof_begin(dugks_t *h, int max_launches)
{
    if (!h || max_launches < 1) return fail(DUGKS_EINVAL, "bad arguments");
    for (auto &e : h->ev) (void)hipEventDestroy(e);
    h->ev.assign(2 * (size_t)max_launches, nullptr);
    for (auto &e : h->ev) HIPCHECK(hipEventCreate(&e));
    h->ev_kind.assign(max_launches, -1);
    h->prof_max = max_launches;
    h->prof_n = 0;
    h->prof_on = true;
    return DUGKS_OK;
}

int dugks_prof_query(dugks_t *h, int kernel, double *mean_ms, int *count)
{
    if (!h || !mean_ms || !count) return fail(DUGKS_EINVAL, "null argument");
    HIPCHECK(hipStreamSynchronize(h->stream));
    double sum = 0;
    int c = 0;
    for (int k = 0; k < h->prof_n; k++) {
        if (h->ev_kind[k] != kernel) continue;
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, h->ev[2 * k], h->ev[2 * k + 1]));
        sum += ms;
        c++;
    }
    *mean_ms = c ? sum / c : 0.0;
    *count = c;
    return DUGKS_OK;
}

int dugks_prof_end(dugks_t *h)
{
    if (!h) return fail(DUGKS_EINVAL, "null handle");
    h->prof_on = false;
    return DUGKS_OK;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
extern "C++" {
template <class T>
static int batch_upload(dugks::Batch *b, const std::vector<T> &v, T **dst)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(T) * (v.empty() ? 1 : v.size()));
    if (e != hipSuccess) return fail(DUGKS_ENOMEM, "batch table");
    b->allocs.push_back(p);
    if (!v.empty()) HIPCHECK(hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    *dst = (T *)p;
    return DUGKS_OK;
}
}  // extern "C++"

int dugks_create_batch(int n, const dugks_desc *descs, dugks_t **out)
{
    if (!out || !descs || n < 1) return fail(DUGKS_EINVAL, "bad arguments");
    *out = nullptr;
    for (int k = 0; k < n; k++) {
        if (descs[k].precision != descs[0].precision || descs[k].stream != descs[0].stream)
            return fail(DUGKS_EINVAL, "instances of a batch share precision and stream");
        if (descs[k].scheme != DUGKS_SCHEME_T3S3) return fail(DUGKS_EINVAL, "batches run the T3S3 scheme");
        if ((descs[k].family_a != 0.0 && descs[k].family_a != 1.0 / 3.0) ||
            descs[k].reconstruction != DUGKS_RECON_POINT)
            return fail(DUGKS_EINVAL, "batches run the T3S3 scheme with the default reconstruction");
    }
    dugks *h = new dugks();
    h->stream = (hipStream_t)descs[0].stream;
    h->delta = descs[0].precision == DUGKS_FP32_DELTA;
    h->batch = new dugks::Batch();
    dugks::Batch *b = h->batch;
    b->delta = h->delta;
    int rc;
    for (int k = 0; k < n; k++) {
        dugks_t *c = nullptr;
        if ((rc = dugks_create(&descs[k], &c))) {
            const std::string m = g_err;
            dugks_destroy(h);
            return fail(rc, "instance " + std::to_string(k) + ": " + m);
        }
        b->inst.push_back(c);
    }
    {
        // any-size instances on the library's tile share one shape (the
        // batched kernels launch blocks of one size): the shape with the
        // fewest launched threads over all of them
        std::vector<std::array<int, 3>> grids;
        auto deflt = [&](int k) {
            return b->inst[k]->lat == 0 && descs[k].tile_x <= 0 && descs[k].tile_y <= 0;
        };
        for (int k = 0; k < n; k++)
            if (deflt(k)) grids.push_back({descs[k].nx, descs[k].ny, descs[k].nq});
        int tx = LQ_DEFAULT_TILE, ty = LQ_DEFAULT_TILE;
        if (!grids.empty()) lq_pick_tile(grids, tx, ty);
        for (int k = 0; k < n; k++) {
            if (!deflt(k) || (b->inst[k]->p.tile_x == tx && b->inst[k]->p.tile_y == ty)) continue;
            dugks_desc dk = descs[k];
            dk.tile_x = tx;
            dk.tile_y = ty;
            dugks_t *c = nullptr;
            dugks_destroy(b->inst[k]);
            b->inst[k] = nullptr;
            if ((rc = dugks_create(&dk, &c))) {
                const std::string m = g_err;
                b->inst.erase(b->inst.begin() + k);
                dugks_destroy(h);
                return fail(rc, "instance " + std::to_string(k) + ": " + m);
            }
            b->inst[k] = c;
        }
    }
    {
        // Velocity chunks of the any-size instances.  Each instance's own
        // chunking fills the chip by itself, which gives small instances
        // chunks of a few velocities; in a batch the instances together fill
        // the chip, so every instance takes chunks of one common length (about
        // eight rounds of blocks over the whole batch), never more chunks than
        // its partial-sum buffers were sized for.
        long long tile_q = 0, cell_q = 0;   // sums of tiles x velocities and cell blocks x velocities
        for (dugks *c : b->inst) {
            if (c->lat != 0) continue;
            tile_q += (long long)lq_ntile(c->p) * c->p.nq;
            cell_q += (c->p.ncell + 255) / 256 * c->p.nq;
        }
        if (tile_q > 0) {
            int dev = 0, ncu = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
                ncu = 256;
            const long long target = 8LL * ncu * 2;   // blocks: eight rounds at two per CU
            const long long lf = std::max(16LL, tile_q / target), lu = std::max(32LL, cell_q / target);
            for (dugks *c : b->inst) {
                if (c->lat != 0) continue;
                SweepParams &p = c->p;
                auto rechunk = [&](long long len, int step, int &chunk, int &nchunk) {
                    const int want = (int)std::max(1LL, std::min<long long>(nchunk, (p.nq + len - 1) / len));
                    int cl = (p.nq + want - 1) / want;
                    cl = (cl + step - 1) / step * step;
                    chunk = cl;
                    nchunk = (p.nq + cl - 1) / cl;
                };
                rechunk(lf, p.lq_qs, p.lq_chunk, p.lq_nchunk);
                rechunk(lu, 4, p.lq_uchunk, p.lq_nuchunk);
            }
        }
    }
    // parameter table and per-(parity, stage) buffer tables
    std::vector<SweepParams> P;
    std::vector<StageIO> io(4 * (size_t)n);
    std::vector<LQStage> lq(4 * (size_t)n);
    for (int k = 0; k < n; k++) {
        dugks *c = b->inst[k];
        P.push_back(c->p);
        for (int par = 0; par < 2; par++) {
            void *X = c->state[par], *Y = c->state[1 - par];
            io[(par * 2 + 0) * n + k] = StageIO{X, nullptr, c->G, c->coefA, c->h1};
            io[(par * 2 + 1) * n + k] = StageIO{c->G, X, Y, c->coefC, c->h2};
            lq[(par * 2 + 0) * n + k] = lq_args(c, 0, X, nullptr, c->G);
            lq[(par * 2 + 1) * n + k] = lq_args(c, 1, c->G, X, Y);
        }
    }
    if ((rc = batch_upload(b, P, &b->d_params)) || (rc = batch_upload(b, io, &b->d_io)) ||
        (rc = batch_upload(b, lq, &b->d_lq))) {
        dugks_destroy(h);
        return rc;
    }
    // work lists
    for (int lat : {9, 37}) {
        dugks::Batch::Group g;
        g.lat = lat;
        std::vector<int4> fast, gen;
        // one work list per compiled tile shape and tau kind (index 2 * shape + tau_field)
        std::vector<std::vector<int4>> by_shape(16);
        std::vector<std::pair<int, int>> shape_of(16, {0, 0});
        for (int k = 0; k < n; k++) {
            dugks *c = b->inst[k];
            if (c->lat != lat) continue;
            const SweepParams &p = c->p;
            const int nt = p.tile_x * p.tile_y;
            if (g.nthreads == 0) g.nthreads = nt;
            if (nt != g.nthreads) {
                dugks_destroy(h);
                return fail(DUGKS_EINVAL, "instances of one lattice in a batch need tiles of equal size");
            }
            g.smem = std::max(g.smem, c->elem * (size_t)p.nq * ((size_t)(p.tile_x + 4) * (p.tile_y + 4) + 1));
            const int gx = (p.nx + p.tile_x - 1) / p.tile_x, gy = (p.ny + p.tile_y - 1) / p.tile_y;
            for (int ty = 0; ty < gy; ty++)
                for (int tx = 0; tx < gx; tx++) {
                    const int i0 = tx * p.tile_x, j0 = ty * p.tile_y;
                    const bool isfast = p.uniform && (p.perx || (i0 >= 2 && i0 + p.tile_x <= p.nx - 2)) &&
                                        (p.pery || (j0 >= 2 && j0 + p.tile_y <= p.ny - 2));
                    const int si = c->fast_ct ? fast_tile_index(p.tile_x, p.tile_y) : -1;
                    if (isfast && si >= 0) {
                        const int slot = 2 * si + (p.tau_field ? 1 : 0);
                        by_shape[slot].push_back(make_int4(k, tx, ty, 0));
                        shape_of[slot] = {p.tile_x, p.tile_y};
                    } else {
                        (isfast ? fast : gen).push_back(make_int4(k, tx, ty, 0));
                    }
                }
        }
        if (g.nthreads == 0) continue;
        g.nfast = (int)fast.size();
        g.ngen = (int)gen.size();
        if ((rc = batch_upload(b, fast, &g.fast)) || (rc = batch_upload(b, gen, &g.gen))) {
            dugks_destroy(h);
            return rc;
        }
        for (int si = 0; si < 16; si++) {
            if (by_shape[si].empty()) continue;
            dugks::Batch::Shape sh;
            sh.tx = shape_of[si].first;
            sh.ty = shape_of[si].second;
            sh.tf = (si & 1) != 0;
            sh.n = (int)by_shape[si].size();
            if ((rc = raise_fast_smem(lat, b->delta, sh.tx, sh.ty, g.smem)) ||
                (rc = batch_upload(b, by_shape[si], &sh.work))) {
                dugks_destroy(h);
                return rc;
            }
            g.shapes.push_back(sh);
        }
        b->groups.push_back(g);
    }
    {
        std::vector<int4> tiles, faces, upd, cells;
        for (int k = 0; k < n; k++) {
            dugks *c = b->inst[k];
            if (c->lat != 0) continue;
            const SweepParams &p = c->p;
            const int nt = p.tile_x * p.tile_y;
            if (b->lq_threads == 0) b->lq_threads = nt;
            if (nt != b->lq_threads) {
                dugks_destroy(h);
                return fail(DUGKS_EINVAL, "any-size instances in a batch need tiles of equal size");
            }
            b->lq_smem = std::max(b->lq_smem, lq_smem_bytes(p, b->delta));
            const int ntile = lq_ntile(p);
            for (int ch = 0; ch < p.lq_nchunk; ch++)
                for (int t = 0; t < ntile; t++) tiles.push_back(make_int4(k, t, ch, 0));
            const long long nface = (long long)(p.nx + 1) * p.ny + (long long)p.nx * (p.ny + 1);
            for (long long f = 0; f < (nface + 255) / 256; f++) faces.push_back(make_int4(k, (int)f, 0, 0));
            for (long long f = 0; f < (p.ncell + 255) / 256; f++) cells.push_back(make_int4(k, (int)f, 0, 0));
            for (int ch = 0; ch < p.lq_nuchunk; ch++)
                for (long long f = 0; f < (p.ncell + 255) / 256; f++) upd.push_back(make_int4(k, (int)f, ch, 0));
        }
        b->nlq_tiles = (int)tiles.size();
        b->nlq_faces = (int)faces.size();
        b->nlq_cells = (int)cells.size();
        b->nlq_upd = (int)upd.size();
        if ((rc = batch_upload(b, tiles, &b->lq_tiles)) || (rc = batch_upload(b, faces, &b->lq_faces)) ||
            (rc = batch_upload(b, upd, &b->lq_upd)) || (rc = batch_upload(b, cells, &b->lq_cells))) {
            dugks_destroy(h);
            return rc;
        }
    }
    char buf[160];
    long long pairs = 0;
    for (dugks *c : b->inst) pairs += c->p.ncell * c->p.nq;
    snprintf(buf, sizeof buf, "batch of %d instances (%lld pairs), %s, %d lattice groups, %d any-size tiles",
             n, pairs, b->delta ? "fp32-delta" : "fp64", (int)b->groups.size(), b->nlq_tiles);
    h->variant = buf;
    *out = h;
    return DUGKS_OK;
}

int dugks_batch_size(dugks_t *h, int *n)
{
    if (!h || !h->batch || !n) return fail(DUGKS_EINVAL, "not a batch");
    *n = (int)h->batch->inst.size();
    return DUGKS_OK;
}

int dugks_batch_instance(dugks_t *h, int k, dugks_t **inst)
{
    if (!h || !h->batch || !inst || k < 0 || k >= (int)h->batch->inst.size())
        return fail(DUGKS_EINVAL, "bad batch instance");
    *inst = h->batch->inst[k];
    return DUGKS_OK;
}

// one step of every instance, starting from state parity `par`
static int batch_enqueue_step(dugks *h, int par)
{
    dugks::Batch *b = h->batch;
    const int n = (int)b->inst.size();
    for (int stage = 0; stage < 2; stage++) {
        const StageIO *io = b->d_io + (size_t)(par * 2 + stage) * n;
        for (const auto &g : b->groups) {
            for (const auto &sh : g.shapes)
                HIPCHECK(launch_stage_fast_batched(stage, g.lat, b->delta, sh.tx, sh.ty, sh.tf, b->d_params, io, sh.work,
                                                   sh.n, g.smem, h->stream));
            HIPCHECK(launch_stage_batched(stage, g.lat, b->delta, b->d_params, io, g.fast, g.nfast, g.gen,
                                          g.ngen, g.nthreads, g.smem, h->stream));
        }
        if (b->nlq_tiles)
            HIPCHECK(launch_lq_stage_batched(b->delta, b->d_params, b->d_lq + (size_t)(par * 2 + stage) * n,
                                             b->lq_tiles, b->nlq_tiles, b->lq_faces, b->nlq_faces,
                                             b->lq_upd, b->nlq_upd, b->lq_cells, b->nlq_cells, b->lq_threads,
                                             b->lq_smem, h->stream));
    }
    return DUGKS_OK;
}

static int batch_graph(dugks *h, int par, int steps, hipGraphExec_t *exec)
{
    if (*exec) return DUGKS_OK;
    hipStream_t s = h->stream;
    bool own = false;
    if (!s) {   // stream capture needs a real stream
        HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        own = true;
    }
    hipStream_t keep = h->stream;
    h->stream = s;
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = DUGKS_OK;
    for (int k = 0; k < steps && rc == DUGKS_OK; k++) rc = batch_enqueue_step(h, (par + k) & 1);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    h->stream = keep;
    if (own) (void)hipStreamDestroy(s);
    if (rc) return rc;
    if (e != hipSuccess) return fail(DUGKS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(DUGKS_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    return DUGKS_OK;
}

static int batch_step(dugks_t *h, int nsteps)
{
    dugks::Batch *b = h->batch;
    const int par = b->inst[0]->cur;
    for (dugks *c : b->inst)
        if (c->cur != par) return fail(DUGKS_EINVAL, "instances of the batch were stepped separately");
    int cur = par, rc;
    for (int done = 0; done < nsteps;) {
        const int k = (nsteps - done >= 2) ? 2 : 1;
        if ((rc = batch_graph(h, cur, k, &b->exec[cur][k - 1]))) return rc;
        if ((rc = record(h, KC_AUX, true))) return rc;
        HIPCHECK(hipGraphLaunch(b->exec[cur][k - 1], h->stream));
        if ((rc = record(h, KC_AUX, false))) return rc;
        cur = (cur + k) & 1;
        done += k;
    }
    for (dugks *c : b->inst) c->cur = cur;
    return DUGKS_OK;
}

// one stage of one step from explicit buffers (backward recomputation)
static int stage_a_from(dugks *h, const void *X)
{
    if (h->lat) {
        HIPCHECK(lattice_stage(h, 0, X, nullptr, h->G));
    } else {
        HIPCHECK(launch_state_moments(h->p, h->delta, X, h->mom_state, h->stream));
        LQStage a = lq_args(h, 0, X, nullptr, h->G);
        HIPCHECK(launch_lq_stage(h->delta, h->p, a, h->stream, -1));
    }
    return DUGKS_OK;
}

static int step_from(dugks *h, const void *X, void *Y)
{
    int rc = stage_a_from(h, X);
    if (rc) return rc;
    if (h->lat) {
        HIPCHECK(lattice_stage(h, 1, h->G, X, Y));
    } else {
        LQStage a = lq_args(h, 1, h->G, X, Y);
        HIPCHECK(launch_lq_stage(h->delta, h->p, a, h->stream, -1));
    }
    return DUGKS_OK;
}

// Device workspace of a backward call.  Every buffer is carved, 256-byte
// aligned, out of one region; with base == nullptr the arena only measures
// the bytes a call needs.
struct Arena {
    char *base = nullptr;
    size_t used = 0;
    void *take(size_t bytes)
    {
        const size_t off = (used + 255) & ~(size_t)255;
        used = off + (bytes ? bytes : 8);
        return base ? (void *)(base + off) : nullptr;
    }
    double *dbl(size_t count) { return (double *)take(count * sizeof(double)); }
};

struct AdjBuffers {
    std::vector<void *> ck, seg;   // checkpoints and the states of one segment
    double *fh_d, *B, *M, *G_d, *B2, *M2, *lam_fbar, *dtf, *lamLs, *lamB, *lamF, *lam[2], *dtau, *tau, *cA, *cC;
    double *lam_rho = nullptr, *lamBg = nullptr;   // walls and stretched grids
};

// the adjoint's kernels for walls and stretched grids (the periodic uniform
// sweep has its own)
static bool adj_general(const dugks *h) { return !h->p.perx || !h->p.pery || !h->p.uniform; }

static void adj_carve(Arena &ar, const dugks *h, int nseg, int k, AdjBuffers &b)
{
    const long long n = h->p.ncell;
    const size_t nqn = (size_t)h->p.nq * n;
    b.ck.assign(nseg + 1, nullptr);
    b.seg.assign(k, nullptr);
    for (auto &c : b.ck) c = ar.take(h->elem * nqn);
    for (int t = 1; t < k; t++) b.seg[t] = ar.take(h->elem * nqn);
    b.fh_d = ar.dbl(nqn);
    b.B = ar.dbl(nqn);
    b.M = ar.dbl(3 * n);
    b.G_d = ar.dbl(nqn);
    b.B2 = ar.dbl(nqn);
    b.M2 = ar.dbl(3 * n);
    // interface adjoints: [axis][q][cell] on periodic uniform grids, [q][face]
    // over the natural face numbering otherwise
    const size_t nface = (size_t)(h->p.nx + 1) * h->p.ny + (size_t)h->p.nx * (h->p.ny + 1);
    const bool gen = adj_general(h);
    b.lam_fbar = ar.dbl(gen ? (size_t)h->p.nq * nface : 2 * nqn);
    b.dtf = ar.dbl(gen ? nface : 2 * (size_t)n);
    if (gen) {
        b.lam_rho = ar.dbl(nface);
        b.lamBg = ar.dbl(nqn);
    }
    b.lamLs = ar.dbl(nqn);
    b.lamB = ar.dbl(nqn);
    b.lamF = ar.dbl(nqn);
    b.lam[0] = ar.dbl(nqn);
    b.lam[1] = ar.dbl(nqn);
    b.dtau = ar.dbl(n);
    b.tau = h->p.tau_field ? const_cast<double *>(h->p.tau) : ar.dbl(n);
    b.cA = ar.dbl(24 * (size_t)h->p.nq);
    b.cC = ar.dbl(24 * (size_t)h->p.nq);
}

static int backward_check(dugks *h, int nsteps, int ckpt_every)
{
    if (nsteps < 0 || ckpt_every < 1) return fail(DUGKS_EINVAL, "bad arguments");
    if (h->batch) return fail(DUGKS_ENOTSUP, "backward of a batch handle");
    if (h->p.t2 || h->var) return fail(DUGKS_ENOTSUP, "the adjoint is written for the T3S3 scheme");
    return DUGKS_OK;
}

// Bytes of device workspace a backward call of nsteps steps needs.
static size_t backward_bytes(const dugks *h, int nsteps, int ckpt_every)
{
    const int k = std::min(ckpt_every, std::max(nsteps, 1));
    const int nseg = (nsteps + k - 1) / k;
    Arena ar;
    AdjBuffers b;
    adj_carve(ar, h, nseg, k, b);
    return ar.used;
}

// The reverse pass on device buffers, its workspace carved from `base`
// (backward_bytes(h, nsteps, ckpt_every) bytes).  Allocates no device memory.
static int backward_core(dugks *h, const double *f0, int nsteps, int ckpt_every, const double *dL_drho,
                         const double *dL_du, double *dL_df0, double *dL_dtau, char *base)
{
    const SweepParams &p = h->p;
    const long long n = p.ncell;
    const int nq = p.nq;
    const size_t nqn = (size_t)nq * n;
    int rc;
    const int k = std::min(ckpt_every, std::max(nsteps, 1));
    const int nseg = (nsteps + k - 1) / k;
    Arena ar;
    ar.base = base;
    AdjBuffers w;
    adj_carve(ar, h, nseg, k, w);
    // host sources of the asynchronous copies below; the call synchronises
    // the stream before they go out of scope
    std::vector<double> t0, a, c;
    if (!p.tau_field) {
        t0.assign(n, p.tau0);
        HIPCHECK(hipMemcpyAsync(w.tau, t0.data(), sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
    }
    if (!adj_general(h)) {
        // interface window weights in double for both stages (the forward
        // kernels of FP32 storage hold them in float)
        const double dx = 1.0 / p.inv_dx, dy = 1.0 / p.inv_dy;
        a = fast_coefs(h->hxi.data(), nq, dx, dy, h->h1, p.kappa);
        c = fast_coefs(h->hxi.data(), nq, dx, dy, h->h2, p.kappa);
        HIPCHECK(hipMemcpyAsync(w.cA, a.data(), sizeof(double) * a.size(), hipMemcpyHostToDevice, h->stream));
        HIPCHECK(hipMemcpyAsync(w.cC, c.data(), sizeof(double) * c.size(), hipMemcpyHostToDevice, h->stream));
    }
    AdjArgs g{};
    g.nx = p.nx;
    g.ny = p.ny;
    g.nq = nq;
    g.n = n;
    g.dt = p.dt;
    g.RT = p.RT;
    g.iRT = p.iRT;
    g.idx = p.inv_dx;
    g.idy = p.inv_dy;
    g.xi = p.xi;
    g.eta = p.eta;
    g.w = p.w;
    g.tau = w.tau;
    g.cA = w.cA;
    g.cC = w.cC;
    g.h1 = h->h1;
    g.h2 = h->h2;
    g.general = adj_general(h) ? 1 : 0;
    g.perx = p.perx;
    g.pery = p.pery;
    for (int k = 0; k < 4; k++) {
        g.bc[k] = p.bc[k];
        g.uw[k][0] = p.uw[k][0];
        g.uw[k][1] = p.uw[k][1];
    }
    g.opp = p.opp;
    g.kappa = p.kappa;
    g.sx_off = p.g.sx_off;
    g.sy_off = p.g.sy_off;
    g.sx_d1 = p.g.sx_d1;
    g.sx_d2 = p.g.sx_d2;
    g.sy_d1 = p.g.sy_d1;
    g.sy_d2 = p.g.sy_d2;
    g.dxl = p.g.dxl;
    g.dxr = p.g.dxr;
    g.dyl = p.g.dyl;
    g.dyr = p.g.dyr;
    g.inv_dx = p.g.inv_dx;
    g.inv_dy = p.g.inv_dy;

    // forward pass from f0, keeping the state at every k-th step and the last
    HIPCHECK(launch_set_state(p, h->delta, f0, w.ck[0], h->stream));
    for (int i = 0; i < nseg; i++) {
        const int len = std::min(k, nsteps - i * k);
        const void *X = w.ck[i];
        for (int t = 0; t < len; t++) {
            void *Y = t == len - 1 ? w.ck[i + 1] : w.seg[t + 1];
            if ((rc = step_from(h, X, Y))) return rc;
            X = Y;
        }
    }
    // seed from the final state; the tau sensitivity accumulates from zero
    HIPCHECK(hipMemsetAsync(w.dtau, 0, sizeof(double) * n, h->stream));
    HIPCHECK(adj_launch_prep(g, h->delta, p.rho0, w.ck[nseg], w.ck[nseg], w.fh_d, w.B, w.M, w.G_d, w.B2, w.M2,
                             h->stream));
    HIPCHECK(adj_launch_seed(g, w.fh_d, dL_drho, dL_du, w.lam[0], h->stream));
    int cur = 0;
    // reverse sweep, one checkpoint segment at a time
    for (int i = nseg - 1; i >= 0; i--) {
        const int len = std::min(k, nsteps - i * k);
        const void *X = w.ck[i];
        for (int t = 0; t + 1 < len; t++) {
            if ((rc = step_from(h, X, w.seg[t + 1]))) return rc;
            X = w.seg[t + 1];
        }
        for (int t = len - 1; t >= 0; t--) {
            const void *Xt = t == 0 ? w.ck[i] : w.seg[t];
            if ((rc = stage_a_from(h, Xt))) return rc;
            if ((rc = record(h, KC_ADJ_STEP, true))) return rc;
            HIPCHECK(adj_launch_prep(g, h->delta, p.rho0, Xt, h->G, w.fh_d, w.B, w.M, w.G_d, w.B2, w.M2,
                                     h->stream));
            HIPCHECK(adj_launch_step(g, w.lam[cur], w.lam[1 - cur], w.fh_d, w.B, w.M, w.G_d, w.B2, w.M2,
                                     w.lam_fbar, w.dtf, w.lamLs, w.lamB, w.lamF, w.dtau, w.lam_rho, w.lamBg,
                                     h->stream));
            if ((rc = record(h, KC_ADJ_STEP, false))) return rc;
            cur = 1 - cur;
        }
    }
    HIPCHECK(adj_launch_init(g, f0, w.lam[cur], dL_df0, w.dtau, h->stream));
    if (dL_dtau)
        HIPCHECK(hipMemcpyAsync(dL_dtau, w.dtau, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
    // the any-size kernels keep the moments of the current state in mom_state
    if (!h->lat) HIPCHECK(launch_state_moments(p, h->delta, h->state[h->cur], h->mom_state, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    (void)nqn;
    return DUGKS_OK;
}

int dugks_backward(dugks_t *h, const double *f0, int nsteps, int ckpt_every,
                   const double *dL_drho, const double *dL_du, double *dL_df0, double *dL_dtau,
                   int mem)
{
    if (!h || !f0 || !dL_du || !dL_df0) return fail(DUGKS_EINVAL, "bad arguments");
    int rc = backward_check(h, nsteps, ckpt_every);
    if (rc) return rc;
    const long long n = h->p.ncell;
    const size_t nqn = (size_t)h->p.nq * n;
    Staged sf0, srho, su, sdf, sdt;
    if ((rc = stage_in(f0, nqn, mem, sf0, h->stream)) || (rc = stage_in(dL_du, 2 * n, mem, su, h->stream)))
        return rc;
    if (dL_drho && (rc = stage_in(dL_drho, n, mem, srho, h->stream))) return rc;
    if ((rc = stage_out(h, dL_df0, nqn, mem, sdf))) return rc;
    if (dL_dtau && (rc = stage_out(h, dL_dtau, n, mem, sdt))) return rc;
    // the workspace stays with the handle and grows when a call needs more
    const size_t need = backward_bytes(h, nsteps, ckpt_every);
    if (need > h->adj_ws_bytes) {
        HIPCHECK(hipStreamSynchronize(h->stream));
        dev_put(h, h->adj_ws);
        h->adj_ws = nullptr;
        h->adj_ws_bytes = 0;
        if ((rc = dev_get(h, &h->adj_ws, need))) {
            h->adj_ws = nullptr;
            return rc;
        }
        h->adj_ws_bytes = need;
    }
    if ((rc = backward_core(h, sf0.dev, nsteps, ckpt_every, dL_drho ? srho.dev : nullptr, su.dev, sdf.dev,
                            dL_dtau ? sdt.dev : nullptr, (char *)h->adj_ws)))
        return rc;
    if ((rc = finish_out(h, dL_df0, nqn, mem, sdf))) return rc;
    if (dL_dtau && (rc = finish_out(h, dL_dtau, n, mem, sdt))) return rc;
    return DUGKS_OK;
}

int dugks_backward_noalloc(dugks_t *h, const double *f0, int nsteps, int ckpt_every,
                           const double *dL_drho, const double *dL_du, double *dL_df0, double *dL_dtau)
{
    if (!h || !f0 || !dL_du || !dL_df0) return fail(DUGKS_EINVAL, "bad arguments");
    int rc = backward_check(h, nsteps, ckpt_every);
    if (rc) return rc;
    const size_t need = backward_bytes(h, nsteps, ckpt_every);
    if (need > kScratchBytes)
        return fail(DUGKS_EINVAL, "dugks_backward_noalloc: the call needs " + std::to_string(need) +
                                      " bytes of workspace, above the fixed scratch of " +
                                      std::to_string(kScratchBytes) + " bytes");
    char *base = nullptr;
    if ((rc = scratch_of(h->device, &base))) return rc;
    return backward_core(h, f0, nsteps, ckpt_every, dL_drho, dL_du, dL_df0, dL_dtau, base);
}

}  // extern "C"
