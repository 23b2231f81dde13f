// Sweep kernels of the T3S3-DUGKS stages for velocity sets of any size (the
// paper's Newton-Cotes grids of up to 101 x 101 velocities).  The interface
// moments need a sum over every velocity before any recovered interface value
// is known (eq. recover2f), and a workgroup cannot hold all velocities of its
// tile, so q is split into chunks across workgroups and each stage runs as:
//   lq_faces        per (tile, q-chunk): interface values of the faces the
//                   tile owns, summed into partial interface moments
//   lq_face_reduce  per face: partial sums over chunks in a fixed order ->
//                   interface moments, plus the diffuse-wall density
//   lq_update       per (tile, q-chunk): interface values of the four faces
//                   of every cell, recovery, micro-flux (eq. microflux) and
//                   the stage output; partial cell moments of the output
//   lq_cell_reduce  per cell: cell moments of the output (fixed order)
// Cell moments of the stage input come from the previous reduction, so each
// plane of a chunk is streamed through LDS once per kernel.  Periodic and
// diffuse boundaries (bounce-back needs the lattice kernels).
#include "sweep_common.h"

#include <algorithm>
#include <type_traits>

namespace dk {

__device__ __forceinline__ long long xface_id(const SweepParams &p, int fi, int j)
{
    if (p.perx && fi == p.nx) fi = 0;
    return (long long)j * (p.nx + 1) + fi;
}

__device__ __forceinline__ long long yface_id(const SweepParams &p, int i, int fj)
{
    if (p.pery && fj == p.ny) fj = 0;
    return (long long)(p.nx + 1) * p.ny + (long long)fj * p.nx + i;
}

// Pre-reconstruction transform coefficients of one cell: B = cc x + ce E.
__device__ __forceinline__ void stage_transform(const SweepParams &p, int stage, long long cell,
                                                double &cc, double &ce)
{
    if (!p.tau_field) {
        cc = p.uc.cc[stage];
        ce = p.uc.ce[stage];
        return;
    }
    const double tau = p.tau[cell], dt = p.dt;
    if (stage == 0) {
        const Stage0Coef c0 = stage0_coef(p.t2, tau, dt);
        cc = c0.cc;
        ce = c0.ce;
    } else {
        cc = (24.0 * tau - 5.0 * dt) / (24.0 * tau + 4.0 * dt);
        ce = 9.0 * dt / (24.0 * tau + 4.0 * dt);
    }
}

// Per-velocity tables read by every thread of a block at the same address.
// They are not written while a stage runs; reading them through the constant
// address space lets the compiler use scalar loads inside the loops over
// velocities (which contain barriers).
template <class T>
using cptr = const __attribute__((address_space(4))) T *;

template <class T>
__device__ __forceinline__ cptr<T> as_const(const T *p)
{
    return (cptr<T>)p;
}


// Planes of B held in LDS at once (velocities per group).
template <bool DELTA>
constexpr int lq_group() { return DELTA ? 4 : 2; }

// LDS row stride of the B planes.  Rows narrower than a half-wave start TX
// banks apart (stride TX + 32), so the 3 x 3 stencil reads of the rows that
// share a half-wave hit distinct banks.
__host__ __device__ inline int lq_row(int tx) { return tx < 32 ? tx + 32 : tx + 2; }
__host__ __device__ inline int lq_plane(int tx, int ty) { return lq_row(tx) * (ty + 2); }

// Copies the records of velocities qa .. qa+n-1 (clamped to the last one)
// into LDS with 32-bit loads spread over the block.
template <class S>
__device__ __forceinline__ void lq_copy_recs(const SweepParams &p, QRec<S> *dst, int qa, int n)
{
    constexpr int NW = (int)(sizeof(QRec<S>) / 4);
    const unsigned *src = (const unsigned *)p.lq_rec;
    unsigned *d = (unsigned *)dst;
    for (int w = threadIdx.x; w < n * NW; w += blockDim.x) {
        const int r = w / NW, k = w - r * NW;
        const int q = min(qa + r, p.nq - 1);
        d[w] = src[(size_t)q * NW + k];
    }
}

// ---------------------------------------------------------------------------
// Ring tiles.  A block of TX x TY threads covers the cells (i0-1 .. i0+TX-2) x
// (j0-1 .. j0+TY-2): the (TX-2) x (TY-2) tile interior and a ring of one cell.
// Every thread forms, per velocity, the derivatives of B at its own cell and
// the interface values of the faces for which its cell is the upwind cell
// (eq. flux_DS): the east face if xi > 0, the west face if xi < 0, half of
// each if xi = 0 (the mean of both expansions), and likewise in y.  Each
// interface value is thus formed once; the ring supplies the values of the
// faces between the interior and the ring.  LDS holds B over the cells
// (i0-2 .. i0+TX-1) x (j0-2 .. j0+TY-1), which covers the 3 x 3 stencil of
// every thread's cell.
// ---------------------------------------------------------------------------
template <class S>
struct RingCell {
    int i, j;            // global cell (periodic wrap applied)
    bool active;         // inside the domain
    bool interior;       // in the tile interior and inside the domain
    bool wW, wE, wS, wN; // next to a (non-periodic) wall on that side
    int slot;            // LDS index of the cell in a plane
    int oxs, oys;        // first stencil column / row relative to the cell
    S d1x[3], d2x[3], d1y[3], d2y[3];   // 3-point derivative weights
    S hxw, hxe, hys, hyn;                // face position minus cell centre
};

template <class S>
__device__ __forceinline__ RingCell<S> ring_cell(const SweepParams &p, int i0, int j0)
{
    const int TX = p.tile_x, RW = lq_row(TX);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    RingCell<S> r;
    int gi = i0 - 1 + lx, gj = j0 - 1 + ly;
    bool in = true;
    if (p.perx) gi = wrapi(gi, p.nx); else in = in && gi >= 0 && gi < p.nx;
    if (p.pery) gj = wrapi(gj, p.ny); else in = in && gj >= 0 && gj < p.ny;
    r.i = gi;
    r.j = gj;
    r.active = in;
    r.interior = in && lx >= 1 && lx <= TX - 2 && ly >= 1 && ly <= p.tile_y - 2 && i0 - 1 + lx < p.nx &&
                 j0 - 1 + ly < p.ny;
    r.slot = (ly + 1) * RW + (lx + 1);
    r.wW = in && !p.perx && gi == 0;
    r.wE = in && !p.perx && gi == p.nx - 1;
    r.wS = in && !p.pery && gj == 0;
    r.wN = in && !p.pery && gj == p.ny - 1;
    const int ci = in ? gi : 0, cj = in ? gj : 0;
    // cells outside the domain: a central stencil with zero weights (reads stay
    // inside the plane; the values are not used)
    r.oxs = in ? p.g.sx_off[ci] : -1;
    r.oys = in ? p.g.sy_off[cj] : -1;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        r.d1x[k] = in ? (S)p.g.sx_d1[3 * ci + k] : (S)0;
        r.d2x[k] = in ? (S)p.g.sx_d2[3 * ci + k] : (S)0;
        r.d1y[k] = in ? (S)p.g.sy_d1[3 * cj + k] : (S)0;
        r.d2y[k] = in ? (S)p.g.sy_d2[3 * cj + k] : (S)0;
    }
    r.hxw = (S)p.g.dxr[ci];       // x_{i-1/2} - x_i
    r.hxe = (S)p.g.dxl[ci + 1];   // x_{i+1/2} - x_i
    r.hys = (S)p.g.dyr[cj];
    r.hyn = (S)p.g.dyl[cj + 1];
    return r;
}

// Derivatives of B at the thread's cell from one LDS plane.
template <class S>
struct Deriv {
    S b0, bx, by, bxx, byy, bxy;
};

template <class S>
__device__ __forceinline__ Deriv<S> derivs(const RingCell<S> &r, const S *P, int HX2)
{
    Deriv<S> d;
    d.b0 = P[r.slot];
    S rows[3];
    d.bx = d.bxx = d.by = d.byy = (S)0;
#pragma unroll
    for (int l = 0; l < 3; l++) {
        const S *row = P + r.slot + (r.oys + l) * HX2 + r.oxs;
        S acc = (S)0;
#pragma unroll
        for (int k = 0; k < 3; k++) acc = fmaS(r.d1x[k], row[k], acc);
        rows[l] = acc;
    }
    const S *rw = P + r.slot + r.oxs;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        d.bx = fmaS(r.d1x[k], rw[k], d.bx);
        d.bxx = fmaS(r.d2x[k], rw[k], d.bxx);
    }
#pragma unroll
    for (int l = 0; l < 3; l++) {
        const S v = P[r.slot + (r.oys + l) * HX2];
        d.by = fmaS(r.d1y[l], v, d.by);
        d.byy = fmaS(r.d2y[l], v, d.byy);
    }
    d.bxy = (S)0;
#pragma unroll
    for (int l = 0; l < 3; l++) d.bxy = fmaS(r.d1y[l], rows[l], d.bxy);
    return d;
}

// B0 + dx Bx + dy By + kappa (dx^2 Bxx + 2 dx dy Bxy + dy^2 Byy)
template <class S>
__device__ __forceinline__ S expand(const Deriv<S> &d, S dx, S dy, S kappa)
{
    const S t = fmaS(dx, d.bxx, (S)2 * dy * d.bxy);
    const S u = fmaS(kappa, t, d.bx);
    S v = fmaS(dx, u, d.b0);
    const S w = fmaS(kappa * dy, d.byy, d.by);
    return fmaS(dy, w, v);
}

// Shared memory of an any-size block.
template <class S>
struct LQShared {
    S *planes;   // [QS][plane] B over the tile and a 2-cell halo
    S *xch;      // [4][QS][TX*TY] interface contributions W, E, S, N (update)
};

template <class S>
__device__ __forceinline__ LQShared<S> lq_shared(const SweepParams &p)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int plane = lq_plane(p.tile_x, p.tile_y);
    LQShared<S> sh;
    sh.planes = reinterpret_cast<S *>(smem_raw);
    sh.xch = sh.planes + p.lq_qs * plane;
    return sh;
}

// LDS cells a thread fills: at most two per thread (a (T+2)^2 plane over T^2
// threads), with their global index and transform coefficients, set up once
// per block.
template <class S>
struct FillSlots {
    static constexpr int N = 2;
    size_t cell[N];
    int lds[N];       // index in a plane (padded rows)
    bool use[N];      // slot exists (index < (TX + 2) (TY + 2))
    S ec[N][6], cc[N];
};

// Once per block: equilibrium coefficients (scaled by ce) and cc of every LDS
// cell the thread fills (zero outside the domain).
template <class S, bool DELTA>
__device__ __forceinline__ FillSlots<S> lq_prepare(const SweepParams &p, const LQStage &a, int i0, int j0)
{
    const int HX2 = p.tile_x + 2;
    const int ncl = HX2 * (p.tile_y + 2);
    FillSlots<S> f;
#pragma unroll
    for (int k = 0; k < FillSlots<S>::N; k++) {
        const int c = threadIdx.x + k * blockDim.x;
        f.use[k] = c < ncl;
        const int hx = c % HX2, hy = c / HX2;
        f.lds[k] = hy * lq_row(p.tile_x) + hx;
        int gi = i0 + hx - 2, gj = j0 + hy - 2;
        bool in = f.use[k];
        if (p.perx) gi = wrapi(gi, p.nx); else in = in && gi >= 0 && gi < p.nx;
        if (p.pery) gj = wrapi(gj, p.ny); else in = in && gj >= 0 && gj < p.ny;
        double ec[6] = {0, 0, 0, 0, 0, 0}, cc = 0.0;
        f.cell[k] = in ? (size_t)gj * p.nx + gi : 0;
        if (in) {
            const long long cell = (long long)gj * p.nx + gi;
            const double *m = a.momX + 4 * cell;
            double ce;
            stage_transform(p, a.stage, cell, cc, ce);
            const EPoly e = epoly(m[0], m[1], m[2], m[3], p.iRT, 1.0, DELTA);
            ec[0] = ce * e.c0; ec[1] = ce * e.c1x; ec[2] = ce * e.c1y;
            ec[3] = ce * e.c2xx; ec[4] = ce * e.c2xy; ec[5] = ce * e.c2yy;
        }
#pragma unroll
        for (int m = 0; m < 6; m++) f.ec[k][m] = (S)ec[m];
        f.cc[k] = (S)cc;
    }
    return f;
}

// Loads of a plane group for the thread's fill slots (issued one group ahead
// of their use, so that their latency overlaps the previous group's work).
template <class S, bool DELTA>
struct FillLoads {
    S x[FillSlots<S>::N][lq_group<DELTA>()];
};

template <class S, bool DELTA>
__device__ __forceinline__ void lq_load(const SweepParams &p, const LQStage &a, const FillSlots<S> &f, int q0,
                                        int nqs, FillLoads<S, DELTA> &v)
{
    constexpr int QS = lq_group<DELTA>();
    const S *__restrict__ X = (const S *)a.X;
    const size_t n = (size_t)p.ncell;
    // velocities past the end repeat the last one (valid addresses, values unused)
#pragma unroll
    for (int k = 0; k < FillSlots<S>::N; k++)
#pragma unroll
        for (int s = 0; s < QS; s++) v.x[k][s] = X[(size_t)min(q0 + s, p.nq - 1) * n + f.cell[k]];
    (void)nqs;
}

// LDS planes q0 .. q0+nqs-1 of B = cc X + ce E (zero outside the domain).
template <class S, bool DELTA>
__device__ __forceinline__ void lq_store(const SweepParams &p, LQShared<S> sh, const FillSlots<S> &f,
                                         const QRec<S> *rq, const FillLoads<S, DELTA> &v)
{
    constexpr int QS = lq_group<DELTA>();
    const int plane = lq_plane(p.tile_x, p.tile_y);
    S mx[QS], my[QS], mxx[QS], mxy[QS], myy[QS], wq[QS];
#pragma unroll
    for (int s = 0; s < QS; s++) {
        const S *m = rq[s].mono;   // x, y, xx, xy, yy, ...
        mx[s] = m[0]; my[s] = m[1]; mxx[s] = m[2]; mxy[s] = m[3]; myy[s] = m[4];
        wq[s] = DELTA ? (S)1 : rq[s].wq;
    }
#pragma unroll
    for (int k = 0; k < FillSlots<S>::N; k++) {
        if (!f.use[k]) continue;
#pragma unroll
        for (int s = 0; s < QS; s++) {
            S e = f.ec[k][0];
            e = fmaS(mx[s], f.ec[k][1], e);
            e = fmaS(my[s], f.ec[k][2], e);
            e = fmaS(mxx[s], f.ec[k][3], e);
            e = fmaS(mxy[s], f.ec[k][4], e);
            e = fmaS(myy[s], f.ec[k][5], e);
            // ec and cc are zero outside the domain; planes past nqs are never read
            sh.planes[s * plane + f.lds[k]] = fmaS(f.cc[k], v.x[k][s], DELTA ? e : wq[s] * e);
        }
    }
}

// Interface values of one velocity at the faces the thread's cell is upwind
// of (zero elsewhere): W, E, S, N.  A velocity parallel to a face gets half
// of each side's expansion, or all of the interior cell's at a wall.  sg:
// bit 0 xi > 0, bit 1 xi < 0, bit 2 eta > 0, bit 3 eta < 0 (uniform).
template <class S>
__device__ __forceinline__ void owned_faces(const RingCell<S> &r, const Deriv<S> &d, int sg, S xh, S yh,
                                            S kappa, S (&f)[4])
{
    f[0] = f[1] = f[2] = f[3] = (S)0;
    if (!r.active) return;
    // x-faces: dy = -eta h
    if (sg & 1) f[1] = expand(d, r.hxe - xh, -yh, kappa);
    else if (sg & 2) f[0] = expand(d, r.hxw - xh, -yh, kappa);
    else {
        f[0] = (r.wW ? (S)1 : (S)0.5) * expand(d, r.hxw, -yh, kappa);
        f[1] = (r.wE ? (S)1 : (S)0.5) * expand(d, r.hxe, -yh, kappa);
    }
    if (sg & 4) f[3] = expand(d, -xh, r.hyn - yh, kappa);
    else if (sg & 8) f[2] = expand(d, -xh, r.hys - yh, kappa);
    else {
        f[2] = (r.wS ? (S)1 : (S)0.5) * expand(d, -xh, r.hys, kappa);
        f[3] = (r.wN ? (S)1 : (S)0.5) * expand(d, -xh, r.hyn, kappa);
    }
}

// The same for a velocity with both components non-zero: one expansion per
// axis, to the east (xpos) or west face and to the north (ypos) or south face.
template <class S>
__device__ __forceinline__ void owned_faces_nz(const RingCell<S> &r, const Deriv<S> &d, bool xpos, bool ypos, S xh,
                                               S yh, S kappa, S &vx, S &vy)
{
    const S hx = xpos ? r.hxe : r.hxw;
    const S hy = ypos ? r.hyn : r.hys;
    vx = r.active ? expand(d, hx - xh, -yh, kappa) : (S)0;
    vy = r.active ? expand(d, -xh, hy - yh, kappa) : (S)0;
}

// ---------------------------------------------------------------------------
// lq_faces: interface values of a q-chunk (stored for lq_update) and their
// partial interface moments.  Per group of QS velocities: B planes into LDS;
// each thread's upwind faces into an exchange buffer; then every interior
// thread sums the two sides of its west and south faces (and of the east /
// north domain faces at walls).
// ---------------------------------------------------------------------------
template <class S, bool DELTA>
__device__ void lq_faces_body(const SweepParams &p, const LQStage &a, int tile, int chunk)
{
    const int TX = p.tile_x, TY = p.tile_y, RW = lq_row(TX);
    const int plane = lq_plane(TX, TY);
    const int NT = TX * TY, t = threadIdx.x;
    LQShared<S> sh = lq_shared<S>(p);
    const int gx = (p.nx + TX - 3) / (TX - 2);
    const int i0 = (tile % gx) * (TX - 2), j0 = (tile / gx) * (TY - 2);
    const int q0 = chunk * p.lq_chunk, q1 = min(p.nq, q0 + p.lq_chunk);
    const RingCell<S> r = ring_cell<S>(p, i0, j0);
    const S kappa = (S)p.kappa, hs = (S)a.h;
    constexpr int QS = lq_group<DELTA>();
    __shared__ QRec<S> recs[LQ_TQ];   // per-velocity data of the current run of velocities
    // domain-boundary faces of the cell
    const bool wallW = r.wW, wallE = r.wE, wallS = r.wS, wallN = r.wN;
    S *xw = sh.xch, *xe = sh.xch + QS * NT, *ys = sh.xch + 2 * QS * NT, *yn = sh.xch + 3 * QS * NT;
    S *__restrict__ FX = (S *)a.fxv;
    S *__restrict__ FY = (S *)a.fyv;
    const size_t nxf = (size_t)(p.nx + 1) * p.ny, nyf = (size_t)p.nx * (p.ny + 1);
    // face indices of interior threads: W, E, S, N (x-face and y-face numbering)
    size_t fid[4] = {0, 0, 0, 0};
    if (r.interior) {
        fid[0] = (size_t)xface_id(p, r.i, r.j);
        fid[1] = (size_t)xface_id(p, r.i + 1, r.j);
        fid[2] = (size_t)(yface_id(p, r.i, r.j) - (long long)nxf);
        fid[3] = (size_t)(yface_id(p, r.i, r.j + 1) - (long long)nxf);
    }

    const FillSlots<S> fsl = lq_prepare<S, DELTA>(p, a, i0, j0);
    double acc[4][3];   // faces W, E, S, N x (sum m x, sum m xi x, sum m eta x)
#pragma unroll
    for (int f = 0; f < 4; f++)
#pragma unroll
        for (int k = 0; k < 3; k++) acc[f][k] = 0.0;
    // diffuse-wall numerators of the faces W, E, S, N (separate scalars: the
    // compiler must not turn the sign choice below into an indexed store)
    double dnW = 0.0, dnE = 0.0, dnS = 0.0, dnN = 0.0;
    FillLoads<S, DELTA> ld;
    lq_load<S, DELTA>(p, a, fsl, q0, min(QS, q1 - q0), ld);

    // interior threads: store the face values of one velocity and add their
    // moments.  WALL: the tile has domain-boundary cells (the east / north
    // faces of wall cells and the diffuse-wall sums are then added too).
    auto finish = [&](auto wall, int q, S fw, S fe, S fs, S fn, const double *m) {
        const double w0 = m[0], w1 = m[1], w2 = m[2];
        constexpr bool WALL = decltype(wall)::value;
        FX[(size_t)q * nxf + fid[0]] = fw;
        FY[(size_t)q * nyf + fid[2]] = fs;
        if (WALL && wallE) FX[(size_t)q * nxf + fid[1]] = fe;
        if (WALL && wallN) FY[(size_t)q * nyf + fid[3]] = fn;
        const double v[4] = {(double)fw, (double)fe, (double)fs, (double)fn};
        // with WALL every lane also sums its east / north faces and the wall
        // numerators (no per-lane selects); only wall faces use those sums
#pragma unroll
        for (int f = 0; f < 4; f++) {
            if (!WALL && (f == 1 || f == 3)) continue;
            acc[f][0] = __builtin_fma(w0, v[f], acc[f][0]);
            acc[f][1] = __builtin_fma(w1, v[f], acc[f][1]);
            acc[f][2] = __builtin_fma(w2, v[f], acc[f][2]);
        }
        if (!WALL) return;
        // arriving at a wall: sum of (xi.n)+ m fbar (eq. of the diffuse-scattering rule)
        dnW = __builtin_fma(m[3], v[0], dnW);
        dnE = __builtin_fma(m[4], v[1], dnE);
        dnS = __builtin_fma(m[5], v[2], dnS);
        dnN = __builtin_fma(m[6], v[3], dnN);
    };

    // one group of QS velocities; NZ: all present and no zero component (one
    // upwind face per axis); FULL: all present; WALL as for finish
    auto group = [&](auto nz, auto full, auto wall, int qa, int nqs, const QRec<S> *rq) {
        constexpr bool NZ = decltype(nz)::value, FULL = decltype(full)::value;
        constexpr bool WALL = decltype(wall)::value;
        int sgv[QS];
        S xh[QS], yh[QS];
#pragma unroll
        for (int s = 0; s < QS; s++) {
            sgv[s] = rq[s].sg;
            xh[s] = rq[s].mono[0] * hs;
            yh[s] = rq[s].mono[1] * hs;
        }
        // no barrier needed before the store: every thread has passed the
        // previous group's last barrier, so the planes are no longer read, and
        // the exchange buffer is rewritten only after the next barrier
        lq_store<S, DELTA>(p, sh, fsl, rq, ld);
        __syncthreads();
        if (qa + QS < q1) lq_load<S, DELTA>(p, a, fsl, qa + QS, min(QS, q1 - qa - QS), ld);
#pragma unroll
        for (int s = 0; s < QS; s++) {
            if (!FULL && s >= nqs) break;
            const Deriv<S> d = derivs<S>(r, sh.planes + s * plane, RW);
            if (NZ) {
                S vx, vy;
                owned_faces_nz<S>(r, d, sgv[s] & 1, sgv[s] & 4, xh[s], yh[s], kappa, vx, vy);
                xw[s * NT + t] = vx;
                ys[s * NT + t] = vy;
            } else {
                S fv[4];
                owned_faces<S>(r, d, sgv[s], xh[s], yh[s], kappa, fv);
                xw[s * NT + t] = fv[0];
                xe[s * NT + t] = fv[1];
                ys[s * NT + t] = fv[2];
                yn[s * NT + t] = fv[3];
            }
            // one velocity at a time (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
        if (!r.interior) return;
#pragma unroll
        for (int s = 0; s < QS; s++) {
            if (!FULL && s >= nqs) break;
            const int q = qa + s, sg = sgv[s], b = s * NT + t;
            const double *m = rq[s].wm;
            S fw, fe, fs, fn;
            if (NZ) {
                const int bx = (sg & 1) ? b - 1 : b, by = (sg & 4) ? b - TX : b;
                fw = xw[bx]; fs = ys[by];
                fe = WALL ? xw[bx + 1] : (S)0;
                fn = WALL ? ys[by + TX] : (S)0;
            } else {
                fw = xe[b - 1] + xw[b]; fe = xe[b] + xw[b + 1];
                fs = yn[b - TX] + ys[b]; fn = yn[b] + ys[b + TX];
            }
            finish(wall, q, fw, fe, fs, fn, m);
            // one velocity at a time (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // tiles whose interior holds no cell next to a non-periodic wall
    const bool twall = (!p.perx && (i0 == 0 || i0 + TX - 2 >= p.nx)) ||
                       (!p.pery && (j0 == 0 || j0 + TY - 2 >= p.ny));
    for (int qa = q0; qa < q1; qa += QS) {
        const int ql = (qa - q0) % LQ_TQ;
        if (ql == 0) {
            // every thread is past its last use of the previous run's records
            __syncthreads();
            lq_copy_recs<S>(p, recs, qa, min(LQ_TQ, (q1 - qa + QS - 1) / QS * QS));
            __syncthreads();
        }
        const QRec<S> *rq = recs + ql;
        if (__builtin_amdgcn_readfirstlane(rq[0].gnz)) {
            if (twall) group(std::true_type{}, std::true_type{}, std::true_type{}, qa, QS, rq);
            else group(std::true_type{}, std::true_type{}, std::false_type{}, qa, QS, rq);
        } else {
            group(std::false_type{}, std::false_type{}, std::true_type{}, qa, min(QS, q1 - qa), rq);
        }
    }
    if (!r.interior) return;
    const long long nface = (long long)nxf + (long long)nyf;
    double *part = a.face_part + (long long)chunk * nface * 4;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const double a0 = k < 3 ? acc[0][k] : dnW, a1 = k < 3 ? acc[1][k] : dnE;
        const double a2 = k < 3 ? acc[2][k] : dnS, a3 = k < 3 ? acc[3][k] : dnN;
        part[4 * fid[0] + k] = a0;
        part[4 * (nxf + fid[2]) + k] = a2;
        if (wallE) part[4 * fid[1] + k] = a1;
        if (wallN) part[4 * (nxf + fid[3]) + k] = a3;
    }
}

// ---------------------------------------------------------------------------
// lq_face_reduce: one thread per face.
// ---------------------------------------------------------------------------
__device__ void lq_face_reduce_body(const SweepParams &p, const LQStage &a, bool delta, long long f)
{
    const long long nxf = (long long)(p.nx + 1) * p.ny;
    const long long nface = nxf + (long long)p.nx * (p.ny + 1);
    if (f >= nface) return;
    int side = -1;
    if (f < nxf) {
        const int fi = (int)(f % (p.nx + 1));
        if (p.perx && fi == p.nx) return;   // alias of face 0
        if (!p.perx && fi == 0) side = 0;
        if (!p.perx && fi == p.nx) side = 1;
    } else {
        const long long g = f - nxf;
        const int fj = (int)(g / p.nx);
        if (p.pery && fj == p.ny) return;
        if (!p.pery && fj == 0) side = 2;
        if (!p.pery && fj == p.ny) side = 3;
    }
    double s0 = 0, sx = 0, sy = 0, sn = 0;
    for (int c = 0; c < p.lq_nchunk; c++) {
        const double *v = a.face_part + ((long long)c * nface + f) * 4;
        s0 += v[0];
        sx += v[1];
        sy += v[2];
        sn += v[3];
    }
    double rho, drho, mx, my;
    if (delta) {
        drho = p.rho0 * p.M0m1 + s0;
        rho = p.rho0 + drho;
        mx = p.rho0 * p.M1x + sx;
        my = p.rho0 * p.M1y + sy;
    } else {
        rho = drho = s0;
        mx = sx;
        my = sy;
    }
    double rw = 0.0;
    if (side >= 0 && p.bc[side] == 2) {
        rw = (sn + p.ds_num_off[side]) / p.ds_den[side];
        const double r0 = delta ? p.rho0 : 0.0;
        rho += rw * p.ds_m[side][0] - r0 * p.ds_w[side][0];
        drho += rw * p.ds_m[side][0] - r0 * p.ds_w[side][0];
        mx += rw * p.ds_m[side][1] - r0 * p.ds_w[side][1];
        my += rw * p.ds_m[side][2] - r0 * p.ds_w[side][2];
    }
    double *o = a.face_mom + 8 * f;
    o[0] = rho; o[1] = drho; o[2] = mx; o[3] = my; o[4] = rw;
}

// ---------------------------------------------------------------------------
// lq_update: recovery, micro-flux and stage output of a q-chunk, one thread
// per cell.  The interface values come from lq_faces; the equilibrium part of
// the recovered interface values (eq. recover2f) and every equilibrium term of
// the output are one cubic polynomial in xi per cell, built once.
// ---------------------------------------------------------------------------
template <class S, bool DELTA>
__device__ void lq_update_body(const SweepParams &p, const LQStage &a, int block, int chunk)
{
    // threads past the last cell work on the last cell and store nothing
    // (every thread takes part in the record copies and their barriers)
    const long long cell0 = (long long)block * blockDim.x + threadIdx.x;
    const bool valid = cell0 < p.ncell;
    const long long cell = valid ? cell0 : p.ncell - 1;
    const int i = (int)(cell % p.nx), j = (int)(cell / p.nx);
    const int q0 = chunk * p.lq_uchunk, q1 = min(p.nq, q0 + p.lq_uchunk);
    __shared__ QRec<S> recs[LQ_TQ];
    const double dt = p.dt, h = a.h;
    const size_t nxf = (size_t)(p.nx + 1) * p.ny, nyf = (size_t)p.nx * (p.ny + 1);
    const long long fidl[4] = {xface_id(p, i, j), xface_id(p, i + 1, j), yface_id(p, i, j), yface_id(p, i, j + 1)};
    const size_t fxw = (size_t)fidl[0], fxe = (size_t)fidl[1];
    const size_t fys = (size_t)(fidl[2] - (long long)nxf), fyn = (size_t)(fidl[3] - (long long)nxf);

    S alpha[4];
    S rws[4];
    bool dsf[4];
    S M[10];   // 1, x, y, xx, xy, yy, xxx, xxy, xyy, yyy
    S kx_own, kf_own = 0, aL, cx, cy;
    {
        const double tau_o = p.tau_field ? p.tau[cell] : p.tau0;
        double tb[4] = {tau_o, tau_o, tau_o, tau_o};
        if (p.tau_field) {
            const int im = p.perx ? wrapi(i - 1, p.nx) : (i > 0 ? i - 1 : i);
            const int ip = p.perx ? wrapi(i + 1, p.nx) : (i < p.nx - 1 ? i + 1 : i);
            const int jm = p.pery ? wrapi(j - 1, p.ny) : (j > 0 ? j - 1 : j);
            const int jp = p.pery ? wrapi(j + 1, p.ny) : (j < p.ny - 1 ? j + 1 : j);
            tb[0] = 0.5 * (tau_o + p.tau[(long long)j * p.nx + im]);
            tb[1] = 0.5 * (tau_o + p.tau[(long long)j * p.nx + ip]);
            tb[2] = 0.5 * (tau_o + p.tau[(long long)jm * p.nx + i]);
            tb[3] = 0.5 * (tau_o + p.tau[(long long)jp * p.nx + i]);
        }
        double be[4], pe[4][6];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const double *fm = a.face_mom + 8 * fidl[k];
            double al;
            if (p.tau_field) {
                al = 2.0 * tb[k] / (2.0 * tb[k] + h);
                be[k] = h / (2.0 * tb[k] + h);
            } else {
                al = p.uc.alpha[a.stage];
                be[k] = p.uc.beta[a.stage];
            }
            const EPoly e = epoly(fm[0], fm[1], fm[2], fm[3], p.iRT, 1.0, DELTA);
            pe[k][0] = e.c0; pe[k][1] = e.c1x; pe[k][2] = e.c1y;
            pe[k][3] = e.c2xx; pe[k][4] = e.c2xy; pe[k][5] = e.c2yy;
            alpha[k] = (S)al;
            rws[k] = (S)fm[4];
        }
        dsf[0] = !p.perx && i == 0 && p.bc[0] == 2;
        dsf[1] = !p.perx && i == p.nx - 1 && p.bc[1] == 2;
        dsf[2] = !p.pery && j == 0 && p.bc[2] == 2;
        dsf[3] = !p.pery && j == p.ny - 1 && p.bc[3] == 2;
        const double idx = p.uniform ? p.inv_dx : p.g.inv_dx[i];
        const double idy = p.uniform ? p.inv_dy : p.g.inv_dy[j];
        cx = (S)(-idx);
        cy = (S)(-idy);
        const double c1 = p.tau_field ? (12.0 * tau_o - dt) / (12.0 * tau_o + 3.0 * dt) : p.uc.c1;
        const double e1 = p.tau_field ? 4.0 * dt / (12.0 * tau_o + 3.0 * dt) : p.uc.e1;
        const double *mx = a.momX + 4 * cell;
        const EPoly ex = epoly(mx[0], mx[1], mx[2], mx[3], p.iRT, 1.0, DELTA);
        double EO[6], aLd;
        if (a.stage == 0) {
            // T3S3: tilde f^+(t_n) = (5/4 c1 - 1/4) fhat + 5/4 e1 E^n (eq. f_tilde_1_3);
            // T2S3: ftilde^+ = ((2 tau - dt) ftilde + 2 dt E) / (2 tau + dt)
            double kxd = p.uc.kx0, ked = p.uc.ke0;
            if (p.tau_field) {
                const Stage0Coef c0 = stage0_coef(p.t2, tau_o, dt);
                kxd = c0.kx;
                ked = c0.ke;
            }
            const double k = ked - rounding_of<S>(kxd);
            EO[0] = k * ex.c0; EO[1] = k * ex.c1x; EO[2] = k * ex.c1y;
            EO[3] = k * ex.c2xx; EO[4] = k * ex.c2xy; EO[5] = k * ex.c2yy;
            kx_own = (S)kxd;
            aLd = p.uc.aL0;
        } else {
            double a_f = p.uc.a_f, a_En = p.uc.a_En, a_G = p.uc.a_G, a_Ep = p.uc.a_Ep;
            if (p.tau_field) {
                const double kw = 6.0 * dt / (6.0 * tau_o + dt);
                a_f = (4.0 - 6.0 * c1) / 7.0;
                a_En = -6.0 / 7.0 * e1;
                a_G = 9.0 / 7.0 - 0.75 * kw;
                a_Ep = 0.75 * kw;
            }
            const double *mf = a.momF + 4 * cell;
            const EPoly en = epoly(mf[0], mf[1], mf[2], mf[3], p.iRT, 1.0, DELTA);
            a_En -= rounding_of<S>(a_f);
            a_Ep -= rounding_of<S>(a_G);
            EO[0] = a_En * en.c0 + a_Ep * ex.c0; EO[1] = a_En * en.c1x + a_Ep * ex.c1x;
            EO[2] = a_En * en.c1y + a_Ep * ex.c1y; EO[3] = a_En * en.c2xx + a_Ep * ex.c2xx;
            EO[4] = a_En * en.c2xy + a_Ep * ex.c2xy; EO[5] = a_En * en.c2yy + a_Ep * ex.c2yy;
            kx_own = (S)a_G;
            kf_own = (S)a_f;
            aLd = 4.0 * dt / 7.0;
        }
        aL = (S)aLd;
        // equilibrium part of L: -(xi/dx)(beta_e E_e - beta_w E_w) - (eta/dy)(beta_n E_n - beta_s E_s)
        const double kx = -idx * aLd, ky = -idy * aLd;
        double A[6], B[6];
#pragma unroll
        for (int c = 0; c < 6; c++) {
            A[c] = be[1] * pe[1][c] - be[0] * pe[0][c];
            B[c] = be[3] * pe[3][c] - be[2] * pe[2][c];
        }
        M[0] = (S)EO[0];
        M[1] = (S)(EO[1] + kx * A[0]);
        M[2] = (S)(EO[2] + ky * B[0]);
        M[3] = (S)(EO[3] + kx * A[1]);
        M[4] = (S)(EO[4] + kx * A[2] + ky * B[1]);
        M[5] = (S)(EO[5] + ky * B[2]);
        M[6] = (S)(kx * A[3]);
        M[7] = (S)(kx * A[4] + ky * B[3]);
        M[8] = (S)(kx * A[5] + ky * B[4]);
        M[9] = (S)(ky * B[5]);
    }
    const S r0s = (S)(DELTA ? p.rho0 : 0.0);
    const S *__restrict__ X = (const S *)a.X;
    const S *__restrict__ F = (const S *)a.F;
    const S *__restrict__ FX = (const S *)a.fxv;
    const S *__restrict__ FY = (const S *)a.fyv;
    S *__restrict__ out = (S *)a.out;
    const size_t n = (size_t)p.ncell;
    double m0 = 0, m1 = 0, m2 = 0;   // partial cell moments of the output
    constexpr int U = 4;             // velocities whose loads are issued together
    for (int qa = q0; qa < q1; qa += U) {
        const int ql = (qa - q0) % LQ_TQ;
        if (ql == 0) {
            __syncthreads();
            lq_copy_recs<S>(p, recs, qa, min(LQ_TQ, (q1 - qa + U - 1) / U * U));
            __syncthreads();
        }
        S fw[U], fe[U], fs[U], fn[U], xo[U], fo[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const size_t q = (size_t)min(qa + u, q1 - 1);
            fw[u] = FX[q * nxf + fxw];
            fe[u] = FX[q * nxf + fxe];
            fs[u] = FY[q * nyf + fys];
            fn[u] = FY[q * nyf + fyn];
            xo[u] = X[q * n + cell];
            fo[u] = a.stage != 0 ? F[q * n + cell] : (S)0;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int q = qa + u;
            if (q >= q1) break;
            const QRec<S> &rq = recs[ql + u];
            const int sg = rq.sg;
            const S *mo = rq.mono;
            S w_ = fw[u], e_ = fe[u], s_ = fs[u], n_ = fn[u];
            // velocities leaving a diffuse wall: fbar = E(rho_w, u_w)
            if (dsf[0] && (sg & 1)) w_ = rws[0] * rq.we[0] - r0s;
            if (dsf[1] && (sg & 2)) e_ = rws[1] * rq.we[1] - r0s;
            if (dsf[2] && (sg & 4)) s_ = rws[2] * rq.we[2] - r0s;
            if (dsf[3] && (sg & 8)) n_ = rws[3] * rq.we[3] - r0s;
            const S La = fmaS(mo[0] * cx, fmaS(alpha[1], e_, -alpha[0] * w_),
                              mo[1] * cy * fmaS(alpha[3], n_, -alpha[2] * s_));
            S Mq = M[0];
#pragma unroll
            for (int k = 0; k < 9; k++) Mq = fmaS(mo[k], M[k + 1], Mq);
            const S sq = DELTA ? (S)1 : rq.wq;
            S R = kx_own * xo[u];
            if (a.stage != 0) R = fmaS(kf_own, fo[u], R);
            const S y = fmaS(aL, La, fmaS(sq, Mq, R));
            if (valid) out[(size_t)q * n + cell] = y;
            // non-finite flag, tested on the first velocity of the chunk (see dugks_sync)
            if (valid && q == q0 && !__builtin_isfinite(y)) *p.bad = 1;
            const double *w3 = rq.wm;
            const double yd = (double)y;
            m0 = __builtin_fma(w3[0], yd, m0);
            m1 = __builtin_fma(w3[1], yd, m1);
            m2 = __builtin_fma(w3[2], yd, m2);
        }
    }
    if (!valid) return;
    double *cp = a.cell_part + ((long long)chunk * p.ncell + cell) * 4;
    cp[0] = m0; cp[1] = m1; cp[2] = m2; cp[3] = 0.0;
}

// ---------------------------------------------------------------------------
// lq_cell_reduce: one thread per cell.
// ---------------------------------------------------------------------------
__device__ void lq_cell_reduce_body(const SweepParams &p, const LQStage &a, bool delta, long long cell)
{
    if (cell >= p.ncell) return;
    double s0 = 0, sx = 0, sy = 0;
    for (int c = 0; c < p.lq_nuchunk; c++) {
        const double *v = a.cell_part + ((long long)c * p.ncell + cell) * 4;
        s0 += v[0];
        sx += v[1];
        sy += v[2];
    }
    double *o = a.mom_out + 4 * cell;
    if (delta) {
        o[1] = p.rho0 * p.M0m1 + s0;
        o[0] = p.rho0 + o[1];
        o[2] = p.rho0 * p.M1x + sx;
        o[3] = p.rho0 * p.M1y + sy;
    } else {
        o[0] = o[1] = s0;
        o[2] = sx;
        o[3] = sy;
    }
}

// Cell moments [cell][4] of a stored state (after set_state / init).
template <class S, bool DELTA>
__global__ void k_state_moments(const SweepParams p, const S *__restrict__ x, double *__restrict__ mom)
{
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= p.ncell) return;
    double a0 = 0, ax = 0, ay = 0;
    for (int q = 0; q < p.nq; q++) {
        const double v = (double)x[q * p.ncell + cell];
        const double m = DELTA ? p.w[q] : 1.0;
        a0 = __builtin_fma(m, v, a0);
        ax = __builtin_fma(m * p.xi[q], v, ax);
        ay = __builtin_fma(m * p.eta[q], v, ay);
    }
    double *o = mom + 4 * cell;
    if (DELTA) {
        o[1] = p.rho0 * p.M0m1 + a0;
        o[0] = p.rho0 + o[1];
        o[2] = p.rho0 * p.M1x + ax;
        o[3] = p.rho0 * p.M1y + ay;
    } else {
        o[0] = o[1] = a0;
        o[2] = ax;
        o[3] = ay;
    }
}

// ---------------------------------------------------------------------------
// Kernels: single instance (params by value, implicit work) and batched
// (params table + work list of (instance, tile, chunk)).
// ---------------------------------------------------------------------------
template <class S, bool DELTA>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
lq_faces(const SweepParams p, const LQStage a)
{
    const int ntile = lq_ntile(p);
    // XCD-aware order: consecutive blocks go to different XCDs, so each XCD
    // takes a contiguous band of (tile, chunk) indices; neighbouring tiles of
    // one chunk then share their ring rows and face lines in one L2
    const int nb = ntile * p.lq_nchunk, b = blockIdx.x, nx8 = p.nxcd;
    const int per = nb / nx8, rem = nb % nx8;
    const int x = b % nx8, slot = b / nx8;
    const int t = x * per + (x < rem ? x : rem) + slot;
    lq_faces_body<S, DELTA>(p, a, t % ntile, t / ntile);
}

template <class S, bool DELTA>
__global__ void __launch_bounds__(256) lq_update(const SweepParams p, const LQStage a)
{
    const int nblk = (int)((p.ncell + 255) / 256);
    lq_update_body<S, DELTA>(p, a, blockIdx.x % nblk, blockIdx.x / nblk);
}

template <bool DELTA>
__global__ void __launch_bounds__(256) lq_face_reduce(const SweepParams p, const LQStage a)
{
    lq_face_reduce_body(p, a, DELTA, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

template <bool DELTA>
__global__ void __launch_bounds__(256) lq_cell_reduce(const SweepParams p, const LQStage a)
{
    lq_cell_reduce_body(p, a, DELTA, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

template <class S, bool DELTA>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
lq_faces_batched(const SweepParams *__restrict__ P,
                                                        const LQStage *__restrict__ A,
                                                        const int4 *__restrict__ work)
{
    const int4 w = work[blockIdx.x];
    lq_faces_body<S, DELTA>(P[w.x], A[w.x], w.y, w.z);
}

template <class S, bool DELTA>
__global__ void __launch_bounds__(256) lq_update_batched(const SweepParams *__restrict__ P,
                                                         const LQStage *__restrict__ A,
                                                         const int4 *__restrict__ work)
{
    const int4 w = work[blockIdx.x];
    lq_update_body<S, DELTA>(P[w.x], A[w.x], w.y, w.z);
}

template <bool DELTA>
__global__ void __launch_bounds__(256) lq_face_reduce_batched(const SweepParams *__restrict__ P,
                                                              const LQStage *__restrict__ A,
                                                              const int4 *__restrict__ work)
{
    const int4 w = work[blockIdx.x];
    lq_face_reduce_body(P[w.x], A[w.x], DELTA, (long long)w.y * blockDim.x + threadIdx.x);
}

template <bool DELTA>
__global__ void __launch_bounds__(256) lq_cell_reduce_batched(const SweepParams *__restrict__ P,
                                                              const LQStage *__restrict__ A,
                                                              const int4 *__restrict__ work)
{
    const int4 w = work[blockIdx.x];
    lq_cell_reduce_body(P[w.x], A[w.x], DELTA, (long long)w.y * blockDim.x + threadIdx.x);
}

template <class S, bool DELTA>
static hipError_t lq_batched_t(const SweepParams *P, const LQStage *A, const int4 *wt, int nt,
                               const int4 *wf, int nf, const int4 *wu, int nu, const int4 *wc, int nc,
                               int nthreads, size_t smem, hipStream_t s)
{
    if (nt > 0) hipLaunchKernelGGL((lq_faces_batched<S, DELTA>), dim3(nt), dim3(nthreads), smem, s, P, A, wt);
    if (nf > 0) hipLaunchKernelGGL((lq_face_reduce_batched<DELTA>), dim3(nf), dim3(256), 0, s, P, A, wf);
    if (nu > 0) hipLaunchKernelGGL((lq_update_batched<S, DELTA>), dim3(nu), dim3(256), 0, s, P, A, wu);
    if (nc > 0) hipLaunchKernelGGL((lq_cell_reduce_batched<DELTA>), dim3(nc), dim3(256), 0, s, P, A, wc);
    return hipGetLastError();
}

hipError_t launch_lq_stage_batched(bool delta, const SweepParams *P, const LQStage *A,
                                   const int4 *work_tiles, int ntiles, const int4 *work_faces, int nfaces,
                                   const int4 *work_upd, int nupd, const int4 *work_cells, int ncells,
                                   int nthreads, size_t smem, hipStream_t s)
{
    return delta ? lq_batched_t<float, true>(P, A, work_tiles, ntiles, work_faces, nfaces, work_upd, nupd,
                                             work_cells, ncells, nthreads, smem, s)
                 : lq_batched_t<double, false>(P, A, work_tiles, ntiles, work_faces, nfaces, work_upd, nupd,
                                               work_cells, ncells, nthreads, smem, s);
}

size_t lq_smem_bytes(const SweepParams &p, bool delta)
{
    // B planes over the tile and halo (padded rows) and the interface
    // exchange (the per-velocity records are static LDS of the kernels)
    const size_t plane = (size_t)lq_plane(p.tile_x, p.tile_y);
    const size_t nt = (size_t)p.tile_x * p.tile_y;
    return (delta ? 4 : 8) * (plane * p.lq_qs + 4 * (size_t)p.lq_qs * nt);
}

template <class S, bool DELTA>
static hipError_t lq_stage_t(const SweepParams &p, const LQStage &a, hipStream_t s, int part)
{
    const int ntile = lq_ntile(p);
    const dim3 blk(p.tile_x * p.tile_y);
    const size_t smem = lq_smem_bytes(p, DELTA);
    const long long nface = (long long)(p.nx + 1) * p.ny + (long long)p.nx * (p.ny + 1);
    if (part == 0 || part < 0)
        hipLaunchKernelGGL((lq_faces<S, DELTA>), dim3(ntile * p.lq_nchunk), blk, smem, s, p, a);
    if (part == 1 || part < 0)
        hipLaunchKernelGGL((lq_face_reduce<DELTA>), dim3((unsigned)((nface + 255) / 256)), dim3(256), 0, s, p, a);
    if (part == 2 || part < 0)
        hipLaunchKernelGGL((lq_update<S, DELTA>), dim3((unsigned)((p.ncell + 255) / 256) * p.lq_nuchunk), dim3(256),
                           0, s, p, a);
    if (part == 3 || part < 0)
        hipLaunchKernelGGL((lq_cell_reduce<DELTA>), dim3((unsigned)((p.ncell + 255) / 256)), dim3(256), 0, s, p, a);
    return hipGetLastError();
}

hipError_t launch_lq_stage(bool delta, const SweepParams &p, const LQStage &a, hipStream_t s, int part)
{
    return delta ? lq_stage_t<float, true>(p, a, s, part) : lq_stage_t<double, false>(p, a, s, part);
}

int lq_blocks_per_cu(bool delta, bool faces, int nthreads, size_t smem)
{
    const void *f = delta ? (faces ? (const void *)lq_faces<float, true> : (const void *)lq_update<float, true>)
                          : (faces ? (const void *)lq_faces<double, false> : (const void *)lq_update<double, false>);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, nthreads, smem) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

hipError_t set_lq_smem(bool delta, size_t bytes)
{
    const void *fns[4];
    if (delta) {
        fns[0] = (const void *)lq_faces<float, true>;
        fns[1] = (const void *)lq_update<float, true>;
        fns[2] = (const void *)lq_faces_batched<float, true>;
        fns[3] = (const void *)lq_update_batched<float, true>;
    } else {
        fns[0] = (const void *)lq_faces<double, false>;
        fns[1] = (const void *)lq_update<double, false>;
        fns[2] = (const void *)lq_faces_batched<double, false>;
        fns[3] = (const void *)lq_update_batched<double, false>;
    }
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_state_moments(const SweepParams &p, bool delta, const void *state, double *mom,
                                hipStream_t s)
{
    const dim3 g((unsigned)((p.ncell + 255) / 256));
    if (delta)
        hipLaunchKernelGGL((k_state_moments<float, true>), g, dim3(256), 0, s, p, (const float *)state, mom);
    else
        hipLaunchKernelGGL((k_state_moments<double, false>), g, dim3(256), 0, s, p, (const double *)state, mom);
    return hipGetLastError();
}

}  // namespace dk
