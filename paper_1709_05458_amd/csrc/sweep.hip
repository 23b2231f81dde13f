// Sweep kernels of the T3S3-DUGKS step for lattices whose velocities are
// integer vectors times a scale (D2Q9 of the paper's "Discrete particle
// velocities" section, and a D2Q37 lattice).  One kernel launch is one stage:
//   STAGE 0 (stage A, steps (1)-(2)):  X = fhat(t_n)      -> out = tilde f(t')
//   STAGE 1 (stage C, steps (3)-(4)):  X = tilde f(t'),
//                                      F = fhat(t_n)      -> out = fhat(t_{n+1})
//
// Layout: SoA, element (q, cell) at q*ncell + cell, cell = j*nx + i.
// A workgroup owns a tile of TX x TY cells, one cell per thread.  It stages
// the pre-reconstruction variable B (eq. f_bar_1_6 for stage A, eq. fbp_5_12
// for stage C) of every velocity over the tile plus a 2-cell halo in LDS.
// The cell moments needed for B's equilibrium part are recomputed from the
// loaded values, so no moment arrays are streamed.  Each thread then forms,
// per velocity, the interface values at its four faces (eqs. interfaceEvof,
// flux_DS), sums the interface moments over q in double, and keeps the part of
// the micro-flux that is linear in the interface values; the equilibrium part
// of the recovered interface distribution (eq. recover2f) is added once the
// interface moments are complete.
#include "dugks_internal.h"
#include "lattices.h"

#include <type_traits>
#include <utility>

#include "launchers.h"
#include "sweep_common.h"

namespace dk {

// ---------------------------------------------------------------------------
// Per-thread state of one stage sweep.
// ---------------------------------------------------------------------------
template <class Lat, class S, bool DELTA>
struct ThreadState {
    static constexpr int Q = Lat::Q;
    S La[Q];          // linear part of the micro-flux
    S R[Q];           // own-cell part of the stage output
    double mr[4], mx[4], my[4];   // interface moment sums (storage units) W,E,S,N
    double num[4];                // diffuse walls: arriving flux sums
    S aw, ae, as_, an;            // recovery weights alpha of the four faces
    S cx, cy;                     // -1/dx, -1/dy of the own cell
};

// Interface moment sums in double.  FP32-delta: sum w_q (1, ex, ey) x_q with
// the products w_q ex, w_q ey read from a per-velocity table (scalar loads),
// so that each term is one conversion and one to three FMAs.
template <class Lat, class S, bool DELTA, int q>
__device__ __forceinline__ void accumulate(ThreadState<Lat, S, DELTA> &t, int face, S v,
                                           const double *__restrict__ wm)
{
    constexpr int EX = Lat::ex(q), EY = Lat::ey(q);
    const double d = (double)v;
    if (DELTA) {
        t.mr[face] = __builtin_fma(wm[3 * q], d, t.mr[face]);
        if (EX) t.mx[face] = __builtin_fma(wm[3 * q + 1], d, t.mx[face]);
        if (EY) t.my[face] = __builtin_fma(wm[3 * q + 2], d, t.my[face]);
    } else {
        t.mr[face] += d;
        if (EX) t.mx[face] = __builtin_fma((double)EX, d, t.mx[face]);
        if (EY) t.my[face] = __builtin_fma((double)EY, d, t.my[face]);
    }
}

// Fast path: uniform grid, tile away from walls.  coef[q*24 + 0..11] are the
// x-face weights over cells (i-2..i+1) x (j-1..j+1) of face i (between cells
// i-1 and i), coef[q*24 + 12..23] the y-face weights over (i-1..i+1) x
// (j-2..j+1) of face j; they fold the upwind choice, the characteristic foot
// point and the 3-point derivatives into one linear combination.
template <class Lat, class S, bool DELTA, int q>
__device__ __forceinline__ void faces_fast(ThreadState<Lat, S, DELTA> &t, const S *lds, int plane,
                                           int HX, int base, const S *__restrict__ coef,
                                           const double *__restrict__ wm, S xq_s, S yq_s)
{
    constexpr int EX = Lat::ex(q), EY = Lat::ey(q);
    const S *P = lds + q * plane + base;
    const S *C = coef + q * 24;
    S vw = 0, ve = 0, vs = 0, vn = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if ((EX > 0 && k == 3) || (EX < 0 && k == 0)) continue;
#pragma unroll
        for (int b = 0; b < 3; b++) {
            const S c = C[k * 3 + b];
            vw = fmaS(c, P[(b - 1) * HX + (k - 2)], vw);
            ve = fmaS(c, P[(b - 1) * HX + (k - 1)], ve);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if ((EY > 0 && k == 3) || (EY < 0 && k == 0)) continue;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const S c = C[12 + k * 3 + a];
            vs = fmaS(c, P[(k - 2) * HX + (a - 1)], vs);
            vn = fmaS(c, P[(k - 1) * HX + (a - 1)], vn);
        }
    }
    accumulate<Lat, S, DELTA, q>(t, 0, vw, wm);
    accumulate<Lat, S, DELTA, q>(t, 1, ve, wm);
    accumulate<Lat, S, DELTA, q>(t, 2, vs, wm);
    accumulate<Lat, S, DELTA, q>(t, 3, vn, wm);
    S l = 0;
    if (EX) l = fmaS(xq_s * t.cx, t.ae * ve - t.aw * vw, l);
    if (EY) l = fmaS(yq_s * t.cy, t.an * vn - t.as_ * vs, l);
    t.La[q] = l;
    // keep the scheduler from hoisting the next velocity's loads above this
    // one (that raises register pressure far beyond what the data needs)
    __builtin_amdgcn_sched_barrier(0);
}

// General path (walls, non-uniform spacing).  Face values are formed in
// double from the LDS plane(s).  Leaving velocities at a diffuse wall are
// deferred until the wall density is known.
template <class Lat, class S, bool DELTA, int q>
__device__ __forceinline__ void faces_general(ThreadState<Lat, S, DELTA> &t, const SweepParams &p,
                                              const S *lds, int plane, int HX, int hxo, int hyo,
                                              int i, int j, double h, double rho_own, double wq,
                                              const double *__restrict__ wm, S xq_s, S yq_s)
{
    constexpr int EX = Lat::ex(q), EY = Lat::ey(q);
    constexpr int O = Lat::opp(q);
    constexpr int OX = Lat::ex(O), OY = Lat::ey(O);
    const double cl = p.clat;
    const double xq = cl * EX, yq = cl * EY;
    const S *P = lds + q * plane;
    const S *PO = lds + O * plane;
    const int nx = p.nx, ny = p.ny;
    double v[4];
    bool defer[4] = {false, false, false, false};

    // ---- x-faces: W = face i (cells i-1 | i), E = face i+1 ----
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int fi = i + s;
        const int hxr = hxo + s;   // LDS column of cell fi
        const double dy = -yq * h;
        double val = 0.0;
        if (!p.perx && fi == 0) {
            if (EX <= 0) {
                val = expand_general(p, P, HX, hxr, hyo, 0, j, p.g.dxr[0] - xq * h, dy);
            } else if (p.bc[0] == 1) {
                const double bb = 2.0 * rho_own * (xq * p.uw[0][0] + yq * p.uw[0][1]) / p.RT;
                val = expand_general(p, PO, HX, hxr, hyo, 0, j, p.g.dxr[0] - cl * OX * h, -cl * OY * h) +
                      (DELTA ? bb : wq * bb);
            } else {
                defer[s] = true;
            }
            if (EX < 0) {   // arriving at the west wall: xi.n = -xi_x > 0
                t.num[0] += -xq * (DELTA ? wq * val : val);
            }
        } else if (!p.perx && fi == nx) {
            if (EX >= 0) {
                val = expand_general(p, P, HX, hxr - 1, hyo, nx - 1, j, p.g.dxl[nx] - xq * h, dy);
            } else if (p.bc[1] == 1) {
                const double bb = 2.0 * rho_own * (xq * p.uw[1][0] + yq * p.uw[1][1]) / p.RT;
                val = expand_general(p, PO, HX, hxr - 1, hyo, nx - 1, j, p.g.dxl[nx] - cl * OX * h,
                                     -cl * OY * h) +
                      (DELTA ? bb : wq * bb);
            } else {
                defer[s] = true;
            }
            if (EX > 0) t.num[1] += xq * (DELTA ? wq * val : val);
        } else {
            const int giL = wrapi(fi - 1, nx), giR = wrapi(fi, nx);
            if (EX > 0) {
                val = expand_general(p, P, HX, hxr - 1, hyo, giL, j, p.g.dxl[fi] - xq * h, dy);
            } else if (EX < 0) {
                val = expand_general(p, P, HX, hxr, hyo, giR, j, p.g.dxr[fi] - xq * h, dy);
            } else {
                const double a = expand_general(p, P, HX, hxr - 1, hyo, giL, j, p.g.dxl[fi], dy);
                const double b = expand_general(p, P, HX, hxr, hyo, giR, j, p.g.dxr[fi], dy);
                val = 0.5 * (a + b);
            }
        }
        v[s] = val;
    }
    // ---- y-faces: S = face j (cells j-1 | j), N = face j+1 ----
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int fj = j + s;
        const int hyr = hyo + s;
        const double dx = -xq * h;
        double val = 0.0;
        if (!p.pery && fj == 0) {
            if (EY <= 0) {
                val = expand_general(p, P, HX, hxo, hyr, i, 0, dx, p.g.dyr[0] - yq * h);
            } else if (p.bc[2] == 1) {
                const double bb = 2.0 * rho_own * (xq * p.uw[2][0] + yq * p.uw[2][1]) / p.RT;
                val = expand_general(p, PO, HX, hxo, hyr, i, 0, -cl * OX * h, p.g.dyr[0] - cl * OY * h) +
                      (DELTA ? bb : wq * bb);
            } else {
                defer[2 + s] = true;
            }
            if (EY < 0) t.num[2] += -yq * (DELTA ? wq * val : val);
        } else if (!p.pery && fj == ny) {
            if (EY >= 0) {
                val = expand_general(p, P, HX, hxo, hyr - 1, i, ny - 1, dx, p.g.dyl[ny] - yq * h);
            } else if (p.bc[3] == 1) {
                const double bb = 2.0 * rho_own * (xq * p.uw[3][0] + yq * p.uw[3][1]) / p.RT;
                val = expand_general(p, PO, HX, hxo, hyr - 1, i, ny - 1, -cl * OX * h,
                                     p.g.dyl[ny] - cl * OY * h) +
                      (DELTA ? bb : wq * bb);
            } else {
                defer[2 + s] = true;
            }
            if (EY > 0) t.num[3] += yq * (DELTA ? wq * val : val);
        } else {
            const int gjS = wrapi(fj - 1, ny), gjN = wrapi(fj, ny);
            if (EY > 0) {
                val = expand_general(p, P, HX, hxo, hyr - 1, i, gjS, dx, p.g.dyl[fj] - yq * h);
            } else if (EY < 0) {
                val = expand_general(p, P, HX, hxo, hyr, i, gjN, dx, p.g.dyr[fj] - yq * h);
            } else {
                const double a = expand_general(p, P, HX, hxo, hyr - 1, i, gjS, dx, p.g.dyl[fj]);
                const double b = expand_general(p, P, HX, hxo, hyr, i, gjN, dx, p.g.dyr[fj]);
                val = 0.5 * (a + b);
            }
        }
        v[2 + s] = val;
    }
    const S vw = (S)v[0], ve = (S)v[1], vs = (S)v[2], vn = (S)v[3];
    if (!defer[0]) accumulate<Lat, S, DELTA, q>(t, 0, vw, wm);
    if (!defer[1]) accumulate<Lat, S, DELTA, q>(t, 1, ve, wm);
    if (!defer[2]) accumulate<Lat, S, DELTA, q>(t, 2, vs, wm);
    if (!defer[3]) accumulate<Lat, S, DELTA, q>(t, 3, vn, wm);
    S l = 0;
    if (EX) l = fmaS(xq_s * t.cx, t.ae * ve - t.aw * vw, l);
    if (EY) l = fmaS(yq_s * t.cy, t.an * vn - t.as_ * vs, l);
    t.La[q] = l;
    __builtin_amdgcn_sched_barrier(0);
}

template <class Lat, class S, bool DELTA, int q>
__device__ __forceinline__ void load_q(const S *__restrict__ X, long long n, long long cell, S *v)
{
    v[q] = X[q * n + cell];
}

template <class Lat, class S, bool DELTA, int q>
__device__ __forceinline__ void moment_q(const S *v, const double *__restrict__ wm, double &a0,
                                         double &ax, double &ay)
{
    constexpr int EX = Lat::ex(q), EY = Lat::ey(q);
    const double d = (double)v[q];
    if (DELTA) {
        a0 = __builtin_fma(wm[3 * q], d, a0);
        if (EX) ax = __builtin_fma(wm[3 * q + 1], d, ax);
        if (EY) ay = __builtin_fma(wm[3 * q + 2], d, ay);
    } else {
        a0 += d;
        if (EX) ax = __builtin_fma((double)EX, d, ax);
        if (EY) ay = __builtin_fma((double)EY, d, ay);
    }
}

// ---------------------------------------------------------------------------
// The stage kernel.  GENERAL = false handles tiles of a uniform grid that are
// clear of walls (precomputed face weights); GENERAL = true handles the other
// tiles (walls, one-sided stencils, non-uniform spacing).  Each instance
// returns at once on the tiles of the other kind.
// ---------------------------------------------------------------------------
template <class Lat, class S, bool DELTA, int STAGE, bool GENERAL>
__device__ __forceinline__ void
sweep_small_body(const SweepParams &p, const double h, const S *__restrict__ X,
                 const S *__restrict__ F, S *__restrict__ out, const S *__restrict__ coef, int tx, int ty)
{
    constexpr int Q = Lat::Q;
    using Seq = std::make_integer_sequence<int, Q>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    S *lds = reinterpret_cast<S *>(smem_raw);

    const int TX = p.tile_x, TY = p.tile_y;
    const int i0 = tx * TX, j0 = ty * TY;

    const int HX = TX + 4;
    const int plane = HX * (TY + 4);
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lx = tid % TX, ly = tid / TX;
    const int i = i0 + lx, j = j0 + ly;
    const bool valid = (i < p.nx) && (j < p.ny);
    const long long n = p.ncell;
    const double dt = p.dt, cl = p.clat;
    const double *__restrict__ W = p.w;
    const double *__restrict__ WM = p.wmom;
    const long long ocell = (long long)j * p.nx + i;
    const double tau_o = (p.tau_field && valid) ? p.tau[ocell] : p.tau0;
    const double c1 = p.tau_field ? (12.0 * tau_o - dt) / (12.0 * tau_o + 3.0 * dt) : p.uc.c1;
    const double e1 = p.tau_field ? 4.0 * dt / (12.0 * tau_o + 3.0 * dt) : p.uc.e1;

    ThreadState<Lat, S, DELTA> t;
    double o_rho = 1.0;

    // ---- load phase: B over tile + halo; the first slot of every thread is
    //      its own cell, whose share of the stage output R is formed here ----
    for (int c = tid; c < plane; c += nthr) {
        int hx, hy;
        halo_pos(c, TX, TY, hx, hy);
        int gi = i0 + hx - 2, gj = j0 + hy - 2;
        bool in = true;
        if (p.perx) gi = wrapi(gi, p.nx); else in = in && gi >= 0 && gi < p.nx;
        if (p.pery) gj = wrapi(gj, p.ny); else in = in && gj >= 0 && gj < p.ny;
        S v[Q];
        double a0 = 0, ax = 0, ay = 0;
        const long long cell = (long long)gj * p.nx + gi;
        if (in) {
            [&]<int... qs>(std::integer_sequence<int, qs...>) {
                (load_q<Lat, S, DELTA, qs>(X, n, cell, v), ...);
                (moment_q<Lat, S, DELTA, qs>(v, WM, a0, ax, ay), ...);
            }(Seq{});
        } else {
#pragma unroll
            for (int q = 0; q < Q; q++) v[q] = (S)0;
            a0 = DELTA ? 0.0 : 1.0;
        }
        double rho, drho, mx, my;
        phys_moments(p, DELTA, a0, ax, ay, rho, drho, mx, my);
        if (!in) { rho = 1.0; drho = DELTA ? 0.0 : 1.0; mx = my = 0.0; }
        const double tau = (p.tau_field && in) ? p.tau[cell] : p.tau0;
        double cc, ce;
        if (!p.tau_field) {
            cc = p.uc.cc[STAGE];
            ce = p.uc.ce[STAGE];
        } else if (STAGE == 0) {   // eq. f_bar_1_6 (T3S3) or fbar^{+,dt/2} of Remark I (T2S3)
            const Stage0Coef c0 = stage0_coef(p.t2, tau, dt);
            cc = c0.cc;
            ce = c0.ce;
        } else {   // eq. fbp_5_12 with the coefficients that map tilde f onto fbar^{+,5dt/12}
            cc = (24.0 * tau - 5.0 * dt) / (24.0 * tau + 4.0 * dt);
            ce = 9.0 * dt / (24.0 * tau + 4.0 * dt);
        }
        const EPoly ep_cell = epoly(rho, drho, mx, my, p.iRT, cl, DELTA);
        EPolyS<S> e;
        e.set(ep_cell, ce);
        const S ccs = (S)cc;
        S *dst = lds + hy * HX + hx;
        [&]<int... qs>(std::integer_sequence<int, qs...>) {
            ((dst[qs * plane] = fmaS(ccs, v[qs],
                                     DELTA ? e.template eval<Lat::ex(qs), Lat::ey(qs)>()
                                           : (S)W[qs] * e.template eval<Lat::ex(qs), Lat::ey(qs)>())),
             ...);
        }(Seq{});
        if (c == tid && valid) {
            o_rho = rho;
            if (STAGE == 0) {
                // T3S3: tilde f^+(t_n) = 5/4 fbar^{+,dt/6} - 1/4 fhat  (eq. f_tilde_1_3);
                // T2S3: ftilde^+ = ((2 tau - dt) ftilde + 2 dt E) / (2 tau + dt)
                double kxd = p.uc.kx0, ked = p.uc.ke0;
                if (p.tau_field) {
                    const Stage0Coef c0 = stage0_coef(p.t2, tau_o, dt);
                    kxd = c0.kx;
                    ked = c0.ke;
                }
                EPolyS<S> en;
                en.set(ep_cell, ked - rounding_of<S>(kxd));
                const S kx = (S)kxd;
                [&]<int... qs>(std::integer_sequence<int, qs...>) {
                    ((t.R[qs] = fmaS(kx, v[qs],
                                     DELTA ? en.template eval<Lat::ex(qs), Lat::ey(qs)>()
                                           : (S)W[qs] * en.template eval<Lat::ex(qs), Lat::ey(qs)>())),
                     ...);
                }(Seq{});
            } else {
                // fhat(t_{n+1}) = fhat/4 + 3/4 fbar^{+,dt/6} + 3/4 dt Omega(t') + 9/7 (tilde f(t') -
                // tilde f^+(t_n)) + 4 dt/7 L**  (eqs. fhp, collisionterm, feqIntD3rdHat2_DS; the T2
                // update of step 2 gives 3 dt/7 L* = 9/7 (tilde f(t') - tilde f^+(t_n)))
                S fh[Q];
                double b0 = 0, bx = 0, by = 0;
                [&]<int... qs>(std::integer_sequence<int, qs...>) {
                    (load_q<Lat, S, DELTA, qs>(F, n, ocell, fh), ...);
                    (moment_q<Lat, S, DELTA, qs>(fh, WM, b0, bx, by), ...);
                }(Seq{});
                double rn, drn, mxn, myn;
                phys_moments(p, DELTA, b0, bx, by, rn, drn, mxn, myn);
                double a_f = p.uc.a_f, a_En = p.uc.a_En, a_G = p.uc.a_G, a_Ep = p.uc.a_Ep;
                if (p.tau_field) {
                    const double kw = 6.0 * dt / (6.0 * tau_o + dt);
                    a_f = (4.0 - 6.0 * c1) / 7.0;
                    a_En = -6.0 / 7.0 * e1;
                    a_G = 9.0 / 7.0 - 0.75 * kw;
                    a_Ep = 0.75 * kw;
                }
                EPolyS<S> en, ep;
                en.set(epoly(rn, drn, mxn, myn, p.iRT, cl, DELTA), a_En - rounding_of<S>(a_f));
                ep.set(ep_cell, a_Ep - rounding_of<S>(a_G));
                const S sf = (S)a_f, sg = (S)a_G;
                [&]<int... qs>(std::integer_sequence<int, qs...>) {
                    ((t.R[qs] = fmaS(sf, fh[qs], fmaS(sg, v[qs],
                        (DELTA ? (S)1 : (S)W[qs]) *
                            (en.template eval<Lat::ex(qs), Lat::ey(qs)>() +
                             ep.template eval<Lat::ex(qs), Lat::ey(qs)>())))),
                     ...);
                }(Seq{});
            }
            if (GENERAL) {   // park R in the output to free registers for the general path
#pragma unroll
                for (int q = 0; q < Q; q++) out[q * n + ocell] = t.R[q];
            }
        }
    }
    __syncthreads();
    if (!valid) return;   // no further barrier below
    const S aL = (S)(STAGE == 0 ? p.uc.aL0 : 4.0 * dt / 7.0);

    // ---- interface recovery weights of the four faces (eq. recover2f) -------
    double tb[4];
    if (p.tau_field) {
        const int im = p.perx ? wrapi(i - 1, p.nx) : (i > 0 ? i - 1 : i);
        const int ip = p.perx ? wrapi(i + 1, p.nx) : (i < p.nx - 1 ? i + 1 : i);
        const int jm = p.pery ? wrapi(j - 1, p.ny) : (j > 0 ? j - 1 : j);
        const int jp = p.pery ? wrapi(j + 1, p.ny) : (j < p.ny - 1 ? j + 1 : j);
        tb[0] = 0.5 * (tau_o + p.tau[(long long)j * p.nx + im]);
        tb[1] = 0.5 * (tau_o + p.tau[(long long)j * p.nx + ip]);
        tb[2] = 0.5 * (tau_o + p.tau[(long long)jm * p.nx + i]);
        tb[3] = 0.5 * (tau_o + p.tau[(long long)jp * p.nx + i]);
    } else {
        tb[0] = tb[1] = tb[2] = tb[3] = p.tau0;
    }
    double alpha[4], beta[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if (p.tau_field) {
            alpha[k] = 2.0 * tb[k] / (2.0 * tb[k] + h);
            beta[k] = h / (2.0 * tb[k] + h);
        } else {
            alpha[k] = p.uc.alpha[STAGE];
            beta[k] = p.uc.beta[STAGE];
        }
    }
    t.aw = (S)alpha[0]; t.ae = (S)alpha[1]; t.as_ = (S)alpha[2]; t.an = (S)alpha[3];
    const double idx = p.uniform ? p.inv_dx : p.g.inv_dx[i];
    const double idy = p.uniform ? p.inv_dy : p.g.inv_dy[j];
    t.cx = (S)(-idx);
    t.cy = (S)(-idy);
#pragma unroll
    for (int k = 0; k < 4; k++) { t.mr[k] = t.mx[k] = t.my[k] = 0.0; t.num[k] = 0.0; }

    // ---- interface values, moments and linear flux part, all q --------------
    const S cls = (S)cl;
    if (!GENERAL) {
        const int base = (ly + 2) * HX + (lx + 2);
        [&]<int... qs>(std::integer_sequence<int, qs...>) {
            (faces_fast<Lat, S, DELTA, qs>(t, lds, plane, HX, base, coef, WM,
                                           cls * (S)Lat::ex(qs), cls * (S)Lat::ey(qs)), ...);
        }(Seq{});
    } else {
        // always_inline: left out of line (it is large for Q = 37), this fold
        // makes the parameters, the thread state and the closure addressable,
        // and every read of them then goes through scratch memory
        [&]<int... qs>(std::integer_sequence<int, qs...>) __attribute__((always_inline)) {
            (faces_general<Lat, S, DELTA, qs>(t, p, lds, plane, HX, lx + 2, ly + 2, i, j, h, o_rho,
                                              W[qs], WM, cls * (S)Lat::ex(qs), cls * (S)Lat::ey(qs)),
             ...);
        }(Seq{});
    }

    // ---- diffuse walls: wall density from zero net mass flux ---------------
    double rw[4] = {0, 0, 0, 0};
    bool dsf[4];
    dsf[0] = GENERAL && !p.perx && i == 0 && p.bc[0] == 2;
    dsf[1] = GENERAL && !p.perx && i == p.nx - 1 && p.bc[1] == 2;
    dsf[2] = GENERAL && !p.pery && j == 0 && p.bc[2] == 2;
    dsf[3] = GENERAL && !p.pery && j == p.ny - 1 && p.bc[3] == 2;
    double M[4][3];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        M[k][0] = t.mr[k];
        M[k][1] = t.mx[k];
        M[k][2] = t.my[k];
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        // physical moments of face k
        double rho, drho, mx, my;
        phys_moments(p, DELTA, M[k][0], M[k][1], M[k][2], rho, drho, mx, my);
        if (GENERAL && dsf[k]) {
            rw[k] = (t.num[k] + p.ds_num_off[k]) / p.ds_den[k];
            const double r0 = DELTA ? p.rho0 : 0.0;
            rho += rw[k] * p.ds_m[k][0] - r0 * p.ds_w[k][0];
            drho += rw[k] * p.ds_m[k][0] - r0 * p.ds_w[k][0];
            mx += rw[k] * p.ds_m[k][1] - r0 * p.ds_w[k][1];
            my += rw[k] * p.ds_m[k][2] - r0 * p.ds_w[k][2];
        }
        M[k][0] = rho; M[k][1] = drho; M[k][2] = mx;
        // reuse slot: store my in t.my
        t.my[k] = my;
    }
    // Equilibrium part beta_b E_b of the recovered interface values enters
    // L_q as -(xi_x/dx)(beta_e E_e - beta_w E_w) - (xi_y/dy)(beta_n E_n - beta_s E_s);
    // with xi = clat e this is one cubic polynomial in the integer vector e.
    Cubic<S> cub;
    {
        const EPoly ew = epoly(M[0][0], M[0][1], M[0][2], t.my[0], p.iRT, cl, DELTA);
        const EPoly ee = epoly(M[1][0], M[1][1], M[1][2], t.my[1], p.iRT, cl, DELTA);
        const EPoly es = epoly(M[2][0], M[2][1], M[2][2], t.my[2], p.iRT, cl, DELTA);
        const EPoly en = epoly(M[3][0], M[3][1], M[3][2], t.my[3], p.iRT, cl, DELTA);
        const double kx = -idx * cl, ky = -idy * cl;
        const double a0 = beta[1] * ee.c0 - beta[0] * ew.c0, a1 = beta[1] * ee.c1x - beta[0] * ew.c1x,
                     a2 = beta[1] * ee.c1y - beta[0] * ew.c1y, a3 = beta[1] * ee.c2xx - beta[0] * ew.c2xx,
                     a4 = beta[1] * ee.c2xy - beta[0] * ew.c2xy, a5 = beta[1] * ee.c2yy - beta[0] * ew.c2yy;
        const double b0 = beta[3] * en.c0 - beta[2] * es.c0, b1 = beta[3] * en.c1x - beta[2] * es.c1x,
                     b2 = beta[3] * en.c1y - beta[2] * es.c1y, b3 = beta[3] * en.c2xx - beta[2] * es.c2xx,
                     b4 = beta[3] * en.c2xy - beta[2] * es.c2xy, b5 = beta[3] * en.c2yy - beta[2] * es.c2yy;
        cub.x = (S)(kx * a0);
        cub.y = (S)(ky * b0);
        cub.xx = (S)(kx * a1);
        cub.xy = (S)(kx * a2 + ky * b1);
        cub.yy = (S)(ky * b2);
        cub.xxx = (S)(kx * a3);
        cub.xxy = (S)(kx * a4 + ky * b3);
        cub.xyy = (S)(kx * a5 + ky * b4);
        cub.yyy = (S)(ky * b5);
    }
    const bool anyds = GENERAL && (dsf[0] || dsf[1] || dsf[2] || dsf[3]);
    const S r0s = (S)(DELTA ? p.rho0 : 0.0);
    const int nq = Q;

    // ---- finish: L = La + equilibrium part (+ deferred wall terms); output --
    S vrest = 0;   // output of the rest velocity, for the non-finite flag
    [&]<int... qs>(std::integer_sequence<int, qs...>) {
        (([&] {
             constexpr int q = qs;
             constexpr int EX = Lat::ex(q), EY = Lat::ey(q);
             const S xq = cls * (S)EX, yq = cls * (S)EY;
             S L = t.La[q];
             if (DELTA) L += cub.template eval<EX, EY>();
             else L = fmaS((S)W[q], cub.template eval<EX, EY>(), L);
             if (GENERAL && anyds) {
                 // leaving velocities of diffuse walls: fbar = E(rho_w, u_w)
                 if (EX > 0 && dsf[0]) L = fmaS(-(xq * t.cx) * t.aw, (S)rw[0] * (S)p.wall_E[0 * nq + q] - r0s, L);
                 if (EX < 0 && dsf[1]) L = fmaS((xq * t.cx) * t.ae, (S)rw[1] * (S)p.wall_E[1 * nq + q] - r0s, L);
                 if (EY > 0 && dsf[2]) L = fmaS(-(yq * t.cy) * t.as_, (S)rw[2] * (S)p.wall_E[2 * nq + q] - r0s, L);
                 if (EY < 0 && dsf[3]) L = fmaS((yq * t.cy) * t.an, (S)rw[3] * (S)p.wall_E[3 * nq + q] - r0s, L);
             }
             const S Rq = GENERAL ? out[q * n + ocell] : t.R[q];
             const S v = fmaS(aL, L, Rq);
             out[q * n + ocell] = v;
             if constexpr (Lat::opp(q) == q) vrest = v;
         }()),
         ...);
    }(Seq{});
    // non-finite flag: a non-finite value anywhere in the cell's neighbourhood
    // reaches every velocity through the moments, so the rest velocity is tested
    if (!__builtin_isfinite(vrest)) *p.bad = 1;
}

// Single instance: tiles from the block index (XCD-aware order); each kind of
// tile is handled by its own instantiation.  MAXT bounds the block: at 256 (a
// tile of up to 256 cells, one wave per SIMD) the compiler may use the whole
// 512-entry register file (arch VGPRs + AGPRs) instead of spilling to scratch;
// the launcher takes that bound where LDS admits only one block per CU.
template <class Lat, class S, bool DELTA, int STAGE, bool GENERAL, int MAXT>
__global__ void __launch_bounds__(MAXT)
sweep_small(const SweepParams p, const double h, const S *__restrict__ X,
            const S *__restrict__ F, S *__restrict__ out, const S *__restrict__ coef, const Ring r)
{
    int tx, ty;
    if (GENERAL && r.on) ring_tile_of(r, p.nxcd, blockIdx.x, tx, ty);
    else tile_of_block(p, tx, ty);
    if (tile_is_fast(p, tx * p.tile_x, ty * p.tile_y, p.tile_x, p.tile_y) == GENERAL) return;
    sweep_small_body<Lat, S, DELTA, STAGE, GENERAL>(p, h, X, F, out, coef, tx, ty);
}

static Ring ring_of(const SweepParams &p)
{
    return ring_make(p.uniform != 0, p.perx != 0, p.pery != 0, p.nx, p.ny, p.tile_x, p.tile_y);
}

// Many instances in one launch: block b works on work[b] = (instance, tile x,
// tile y), with the instance's parameters and buffers read from device tables.
template <class Lat, class S, bool DELTA, int STAGE, bool GENERAL>
__global__ void __launch_bounds__(512)
sweep_small_batched(const SweepParams *__restrict__ P, const StageIO *__restrict__ io,
                    const int4 *__restrict__ work)
{
    const int4 w = work[blockIdx.x];
    const SweepParams &p = P[w.x];
    const StageIO &a = io[w.x];
    sweep_small_body<Lat, S, DELTA, STAGE, GENERAL>(p, a.h, (const S *)a.X, (const S *)a.F, (S *)a.out,
                                                   (const S *)a.coef, w.y, w.z);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <class Lat, class S, bool DELTA, int STAGE>
static hipError_t launch_t(const SweepParams &p, double h, const void *X, const void *F, void *out,
                           const void *coef, hipStream_t s, int parts)
{
    dim3 grid(((p.nx + p.tile_x - 1) / p.tile_x) * ((p.ny + p.tile_y - 1) / p.tile_y));
    dim3 block(p.tile_x * p.tile_y);
    size_t smem = sizeof(S) * Lat::Q * (size_t)(p.tile_x + 4) * (p.tile_y + 4);
    // tiles of the fast kind exist unless the grid is non-uniform; tiles of the
    // general kind exist unless the domain is uniform and fully periodic
    const bool any_fast = p.uniform && (parts & 1);
    const bool any_general = !(p.uniform && p.perx && p.pery) && (parts & 2);
    const bool small = p.tile_x * p.tile_y <= 256;
    const Ring none{0, 0, 0, 0, 0, 0, 0};
    if (any_fast) {
        if (small)
            hipLaunchKernelGGL((sweep_small<Lat, S, DELTA, STAGE, false, 256>), grid, block, smem, s, p, h,
                               (const S *)X, (const S *)F, (S *)out, (const S *)coef, none);
        else
            hipLaunchKernelGGL((sweep_small<Lat, S, DELTA, STAGE, false, 512>), grid, block, smem, s, p, h,
                               (const S *)X, (const S *)F, (S *)out, (const S *)coef, none);
    }
    if (any_general) {
        // a uniform grid with walls: one block per tile of the ring only
        const Ring r = ring_of(p);
        const dim3 ggrid(r.on ? (unsigned)r.ng : grid.x);
        if (r.on && r.ng == 0) return hipGetLastError();
        // two waves per SIMD pay only where two blocks fit in a CU's 160 KB of
        // LDS (D2Q37 FP32-delta on a 16 x 16 tile: 508 ring tiles of 2048^2
        // in one round of blocks instead of two, 15% faster per step despite
        // the spills at that bound); otherwise one wave with every register
        const bool two_blocks = 2 * smem <= 160u * 1024u;
        if (small && !two_blocks)
            hipLaunchKernelGGL((sweep_small<Lat, S, DELTA, STAGE, true, 256>), ggrid, block, smem, s, p, h,
                               (const S *)X, (const S *)F, (S *)out, (const S *)coef, r);
        else
            hipLaunchKernelGGL((sweep_small<Lat, S, DELTA, STAGE, true, 512>), ggrid, block, smem, s, p, h,
                               (const S *)X, (const S *)F, (S *)out, (const S *)coef, r);
    }
    return hipGetLastError();
}

template <class Lat, class S, bool DELTA>
static hipError_t smem_t(size_t bytes)
{
    const void *fns[12] = {(const void *)sweep_small<Lat, S, DELTA, 0, false, 256>,
                          (const void *)sweep_small<Lat, S, DELTA, 1, false, 256>,
                          (const void *)sweep_small<Lat, S, DELTA, 0, true, 256>,
                          (const void *)sweep_small<Lat, S, DELTA, 1, true, 256>,
                          (const void *)sweep_small<Lat, S, DELTA, 0, false, 512>,
                          (const void *)sweep_small<Lat, S, DELTA, 1, false, 512>,
                          (const void *)sweep_small<Lat, S, DELTA, 0, true, 512>,
                          (const void *)sweep_small<Lat, S, DELTA, 1, true, 512>,
                          (const void *)sweep_small_batched<Lat, S, DELTA, 0, false>,
                          (const void *)sweep_small_batched<Lat, S, DELTA, 1, false>,
                          (const void *)sweep_small_batched<Lat, S, DELTA, 0, true>,
                          (const void *)sweep_small_batched<Lat, S, DELTA, 1, true>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class Lat, class S, bool DELTA, int STAGE>
static hipError_t launch_batched_t(const SweepParams *P, const StageIO *io, const int4 *work, int nfast,
                                   const int4 *work_gen, int ngen, int nthreads, size_t smem, hipStream_t s)
{
    if (nfast > 0)
        hipLaunchKernelGGL((sweep_small_batched<Lat, S, DELTA, STAGE, false>), dim3(nfast), dim3(nthreads),
                           smem, s, P, io, work);
    if (ngen > 0)
        hipLaunchKernelGGL((sweep_small_batched<Lat, S, DELTA, STAGE, true>), dim3(ngen), dim3(nthreads),
                           smem, s, P, io, work_gen);
    return hipGetLastError();
}

// Entry points of one lattice and precision (declared in launchers.h; the
// dispatch by value is in dispatch.hip).
template <class Lat, class S, bool DELTA>
hipError_t small_stage(int stage, const SweepParams &p, double h, const void *X, const void *F, void *out,
                       const void *coef, hipStream_t s, int parts)
{
    return stage == 0 ? launch_t<Lat, S, DELTA, 0>(p, h, X, F, out, coef, s, parts)
                      : launch_t<Lat, S, DELTA, 1>(p, h, X, F, out, coef, s, parts);
}

template <class Lat, class S, bool DELTA>
hipError_t small_stage_batched(int stage, const SweepParams *P, const StageIO *io, const int4 *work_fast,
                               int nfast, const int4 *work_gen, int ngen, int nthreads, size_t smem,
                               hipStream_t s)
{
    return stage == 0 ? launch_batched_t<Lat, S, DELTA, 0>(P, io, work_fast, nfast, work_gen, ngen, nthreads, smem, s)
                      : launch_batched_t<Lat, S, DELTA, 1>(P, io, work_fast, nfast, work_gen, ngen, nthreads, smem, s);
}

template <class Lat, class S, bool DELTA>
hipError_t small_smem(size_t bytes)
{
    return smem_t<Lat, S, DELTA>(bytes);
}

// The build compiles this file once per lattice and precision (DK_LAT = 9 or
// 37, DK_DELTA = 1 for FP32-delta), so the four sets of kernels compile in
// parallel.
#if defined(DK_LAT) && defined(DK_DELTA)
using InstLat = std::conditional_t<DK_LAT == 9, LatD2Q9, LatD2Q37>;
using InstS = std::conditional_t<DK_DELTA != 0, float, double>;
template hipError_t small_stage<InstLat, InstS, DK_DELTA != 0>(int, const SweepParams &, double, const void *,
                                                                const void *, void *, const void *,
                                                                hipStream_t, int);
template hipError_t small_stage_batched<InstLat, InstS, DK_DELTA != 0>(int, const SweepParams *,
                                                                        const StageIO *, const int4 *, int,
                                                                        const int4 *, int, int, size_t,
                                                                        hipStream_t);
template hipError_t small_smem<InstLat, InstS, DK_DELTA != 0>(size_t);
#endif

}  // namespace dk
