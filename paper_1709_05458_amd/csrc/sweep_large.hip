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
        cc = (12.0 * tau - dt) / (12.0 * tau + 3.0 * dt);
        ce = 4.0 * dt / (12.0 * tau + 3.0 * dt);
    } else {
        cc = (24.0 * tau - 5.0 * dt) / (24.0 * tau + 4.0 * dt);
        ce = 9.0 * dt / (24.0 * tau + 4.0 * dt);
    }
}

// E_q(moments) / s_q - r0 for runtime velocity (xq, yq), from EPoly coefficients
// built with clat = 1.
template <class S>
__device__ __forceinline__ S eval_rt(const S *c, S xq, S yq)
{
    S v = c[0];
    v = fmaS(xq, c[1], v);
    v = fmaS(yq, c[2], v);
    v = fmaS(xq * xq, c[3], v);
    v = fmaS(xq * yq, c[4], v);
    v = fmaS(yq * yq, c[5], v);
    return v;
}

// Shared memory of a large-Q block: QS planes of B over the halo tile, and per
// halo cell the scaled equilibrium coefficients (6) and the transform weight.
template <class S>
struct LQShared {
    S *planes;   // [QS][plane]
    S *ecoef;    // [7][plane]
};

// Fill LDS planes q0 .. q0+nqs-1 with B = cc X + ce E over the halo tile.
template <class S, bool DELTA>
__device__ __forceinline__ void lq_fill(const SweepParams &p, const LQStage &a, LQShared<S> sh,
                                        int i0, int j0, int q0, int nqs)
{
    const int TX = p.tile_x, TY = p.tile_y, HX = TX + 4;
    const int plane = HX * (TY + 4);
    const S *__restrict__ X = (const S *)a.X;
    const long long n = p.ncell;
    for (int c = threadIdx.x; c < plane; c += blockDim.x) {
        const int hx = c % HX, hy = c / HX;
        int gi = i0 + hx - 2, gj = j0 + hy - 2;
        bool in = true;
        if (p.perx) gi = wrapi(gi, p.nx); else in = in && gi >= 0 && gi < p.nx;
        if (p.pery) gj = wrapi(gj, p.ny); else in = in && gj >= 0 && gj < p.ny;
        S ec[6];
#pragma unroll
        for (int k = 0; k < 6; k++) ec[k] = sh.ecoef[k * plane + c];
        const S cc = sh.ecoef[6 * plane + c];
        const long long cell = (long long)gj * p.nx + gi;
        for (int s = 0; s < nqs; s++) {
            const int q = q0 + s;
            S v = (S)0;
            if (in) {
                const S e = eval_rt(ec, (S)p.xi[q], (S)p.eta[q]);
                v = fmaS(cc, X[q * n + cell], DELTA ? e : (S)p.w[q] * e);
            }
            sh.planes[s * plane + c] = v;
        }
    }
}

// Once per block: equilibrium coefficients (scaled by ce) and cc of every halo cell.
template <class S, bool DELTA>
__device__ __forceinline__ void lq_prepare(const SweepParams &p, const LQStage &a, LQShared<S> sh,
                                           int i0, int j0)
{
    const int TX = p.tile_x, TY = p.tile_y, HX = TX + 4;
    const int plane = HX * (TY + 4);
    for (int c = threadIdx.x; c < plane; c += blockDim.x) {
        const int hx = c % HX, hy = c / HX;
        int gi = i0 + hx - 2, gj = j0 + hy - 2;
        bool in = true;
        if (p.perx) gi = wrapi(gi, p.nx); else in = in && gi >= 0 && gi < p.nx;
        if (p.pery) gj = wrapi(gj, p.ny); else in = in && gj >= 0 && gj < p.ny;
        double ec[6] = {0, 0, 0, 0, 0, 0}, cc = 0.0;
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
        for (int k = 0; k < 6; k++) sh.ecoef[k * plane + c] = (S)ec[k];
        sh.ecoef[6 * plane + c] = (S)cc;
    }
}

// Interface value of x-face fi (cells fi-1 | fi) in row j for velocity (xq, yq);
// hxr is the LDS column of cell fi.  Returns false for a velocity leaving a
// diffuse wall (value set later from the wall density).
template <class S>
__device__ __forceinline__ bool lq_xface(const SweepParams &p, const S *P, int HX, int fi, int hxr,
                                         int hyo, int j, double xq, double yq, double h, double &v)
{
    const double dy = -yq * h;
    if (!p.perx && fi == 0) {
        if (xq > 0.0) return false;
        v = expand_general(p, P, HX, hxr, hyo, 0, j, p.g.dxr[0] - xq * h, dy);
    } else if (!p.perx && fi == p.nx) {
        if (xq < 0.0) return false;
        v = expand_general(p, P, HX, hxr - 1, hyo, p.nx - 1, j, p.g.dxl[p.nx] - xq * h, dy);
    } else {
        const int giL = wrapi(fi - 1, p.nx), giR = wrapi(fi, p.nx);
        if (xq > 0.0) {
            v = expand_general(p, P, HX, hxr - 1, hyo, giL, j, p.g.dxl[fi] - xq * h, dy);
        } else if (xq < 0.0) {
            v = expand_general(p, P, HX, hxr, hyo, giR, j, p.g.dxr[fi] - xq * h, dy);
        } else {
            v = 0.5 * (expand_general(p, P, HX, hxr - 1, hyo, giL, j, p.g.dxl[fi], dy) +
                       expand_general(p, P, HX, hxr, hyo, giR, j, p.g.dxr[fi], dy));
        }
    }
    return true;
}

template <class S>
__device__ __forceinline__ bool lq_yface(const SweepParams &p, const S *P, int HX, int fj, int hyr,
                                         int hxo, int i, double xq, double yq, double h, double &v)
{
    const double dx = -xq * h;
    if (!p.pery && fj == 0) {
        if (yq > 0.0) return false;
        v = expand_general(p, P, HX, hxo, hyr, i, 0, dx, p.g.dyr[0] - yq * h);
    } else if (!p.pery && fj == p.ny) {
        if (yq < 0.0) return false;
        v = expand_general(p, P, HX, hxo, hyr - 1, i, p.ny - 1, dx, p.g.dyl[p.ny] - yq * h);
    } else {
        const int gjS = wrapi(fj - 1, p.ny), gjN = wrapi(fj, p.ny);
        if (yq > 0.0) {
            v = expand_general(p, P, HX, hxo, hyr - 1, i, gjS, dx, p.g.dyl[fj] - yq * h);
        } else if (yq < 0.0) {
            v = expand_general(p, P, HX, hxo, hyr, i, gjN, dx, p.g.dyr[fj] - yq * h);
        } else {
            v = 0.5 * (expand_general(p, P, HX, hxo, hyr - 1, i, gjS, dx, p.g.dyl[fj]) +
                       expand_general(p, P, HX, hxo, hyr, i, gjN, dx, p.g.dyr[fj]));
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// lq_faces
// ---------------------------------------------------------------------------
template <class S, bool DELTA>
__device__ void lq_faces_body(const SweepParams &p, const LQStage &a, int tile, int chunk)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int TX = p.tile_x, TY = p.tile_y, HX = TX + 4;
    const int plane = HX * (TY + 4);
    LQShared<S> sh;
    sh.planes = reinterpret_cast<S *>(smem_raw);
    sh.ecoef = sh.planes + p.lq_qs * plane;
    const int gx = (p.nx + TX - 1) / TX;
    const int i0 = (tile % gx) * TX, j0 = (tile / gx) * TY;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int i = i0 + lx, j = j0 + ly;
    const bool valid = i < p.nx && j < p.ny;
    const int q0 = chunk * p.lq_chunk, q1 = min(p.nq, q0 + p.lq_chunk);

    lq_prepare<S, DELTA>(p, a, sh, i0, j0);
    // owned faces: W (x-face i), S (y-face j), and the E / N domain-boundary faces
    const bool ownE = !p.perx && i == p.nx - 1;
    const bool ownN = !p.pery && j == p.ny - 1;
    double acc[4][4];   // faces W, S, E, N x (sum m x, sum m xi x, sum m eta x, diffuse numerator)
#pragma unroll
    for (int f = 0; f < 4; f++)
#pragma unroll
        for (int k = 0; k < 4; k++) acc[f][k] = 0.0;
    const double h = a.h;
    for (int qa = q0; qa < q1; qa += p.lq_qs) {
        const int nqs = min(p.lq_qs, q1 - qa);
        __syncthreads();
        lq_fill<S, DELTA>(p, a, sh, i0, j0, qa, nqs);
        __syncthreads();
        if (!valid) continue;
        for (int s = 0; s < nqs; s++) {
            const int q = qa + s;
            const double xq = p.xi[q], yq = p.eta[q];
            const double m = DELTA ? p.w[q] : 1.0;
            const S *P = sh.planes + s * plane;
            double v;
            // west face of the cell
            if (lq_xface(p, P, HX, i, lx + 2, ly + 2, j, xq, yq, h, v)) {
                acc[0][0] = __builtin_fma(m, v, acc[0][0]);
                acc[0][1] = __builtin_fma(m * xq, v, acc[0][1]);
                acc[0][2] = __builtin_fma(m * yq, v, acc[0][2]);
                if (!p.perx && i == 0 && xq < 0.0) acc[0][3] = __builtin_fma(-xq * m, v, acc[0][3]);
            }
            if (lq_yface(p, P, HX, j, ly + 2, lx + 2, i, xq, yq, h, v)) {
                acc[1][0] = __builtin_fma(m, v, acc[1][0]);
                acc[1][1] = __builtin_fma(m * xq, v, acc[1][1]);
                acc[1][2] = __builtin_fma(m * yq, v, acc[1][2]);
                if (!p.pery && j == 0 && yq < 0.0) acc[1][3] = __builtin_fma(-yq * m, v, acc[1][3]);
            }
            if (ownE && lq_xface(p, P, HX, i + 1, lx + 3, ly + 2, j, xq, yq, h, v)) {
                acc[2][0] = __builtin_fma(m, v, acc[2][0]);
                acc[2][1] = __builtin_fma(m * xq, v, acc[2][1]);
                acc[2][2] = __builtin_fma(m * yq, v, acc[2][2]);
                if (xq > 0.0) acc[2][3] = __builtin_fma(xq * m, v, acc[2][3]);
            }
            if (ownN && lq_yface(p, P, HX, j + 1, ly + 3, lx + 2, i, xq, yq, h, v)) {
                acc[3][0] = __builtin_fma(m, v, acc[3][0]);
                acc[3][1] = __builtin_fma(m * xq, v, acc[3][1]);
                acc[3][2] = __builtin_fma(m * yq, v, acc[3][2]);
                if (yq > 0.0) acc[3][3] = __builtin_fma(yq * m, v, acc[3][3]);
            }
        }
    }
    if (!valid) return;
    const long long nface = (long long)(p.nx + 1) * p.ny + (long long)p.nx * (p.ny + 1);
    double *part = a.face_part + (long long)chunk * nface * 4;
    long long fid[4] = {xface_id(p, i, j), yface_id(p, i, j), xface_id(p, i + 1, j), yface_id(p, i, j + 1)};
    const bool own[4] = {true, true, ownE, ownN};
#pragma unroll
    for (int f = 0; f < 4; f++)
        if (own[f])
#pragma unroll
            for (int k = 0; k < 4; k++) part[4 * fid[f] + k] = acc[f][k];
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
// lq_update
// ---------------------------------------------------------------------------
template <class S, bool DELTA>
__device__ void lq_update_body(const SweepParams &p, const LQStage &a, int tile, int chunk)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int TX = p.tile_x, TY = p.tile_y, HX = TX + 4;
    const int plane = HX * (TY + 4);
    LQShared<S> sh;
    sh.planes = reinterpret_cast<S *>(smem_raw);
    sh.ecoef = sh.planes + p.lq_qs * plane;
    const int gx = (p.nx + TX - 1) / TX;
    const int i0 = (tile % gx) * TX, j0 = (tile / gx) * TY;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int i = i0 + lx, j = j0 + ly;
    const bool valid = i < p.nx && j < p.ny;
    const int q0 = chunk * p.lq_chunk, q1 = min(p.nq, q0 + p.lq_chunk);
    const long long n = p.ncell;
    const long long cell = (long long)j * p.nx + i;
    const double dt = p.dt, h = a.h;

    lq_prepare<S, DELTA>(p, a, sh, i0, j0);

    // per-thread face data: equilibrium coefficients (scaled by beta), alpha,
    // diffuse-wall densities; own-cell output coefficients
    S eb[4][6];
    S alpha_s[4];
    double rw[4] = {0, 0, 0, 0};
    bool dsf[4] = {false, false, false, false};
    S ownE[6], ownE2[6];   // stage A: 5/4 e1 E^n ; stage C: a_En E^n, a_Ep E'
    S kx_own = 0, kf_own = 0, aL = 0;
    S cx = 0, cy = 0;
    if (valid) {
        const long long fid[4] = {xface_id(p, i, j), xface_id(p, i + 1, j), yface_id(p, i, j),
                                  yface_id(p, i, j + 1)};
        const double tau_o = p.tau_field ? p.tau[cell] : p.tau0;
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
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const double *fm = a.face_mom + 8 * fid[k];
            double al, be;
            if (p.tau_field) {
                al = 2.0 * tb[k] / (2.0 * tb[k] + h);
                be = h / (2.0 * tb[k] + h);
            } else {
                al = p.uc.alpha[a.stage];
                be = p.uc.beta[a.stage];
            }
            const EPoly e = epoly(fm[0], fm[1], fm[2], fm[3], p.iRT, 1.0, DELTA);
            eb[k][0] = (S)(be * e.c0); eb[k][1] = (S)(be * e.c1x); eb[k][2] = (S)(be * e.c1y);
            eb[k][3] = (S)(be * e.c2xx); eb[k][4] = (S)(be * e.c2xy); eb[k][5] = (S)(be * e.c2yy);
            alpha_s[k] = (S)al;
            rw[k] = fm[4];
        }
        dsf[0] = !p.perx && i == 0 && p.bc[0] == 2;
        dsf[1] = !p.perx && i == p.nx - 1 && p.bc[1] == 2;
        dsf[2] = !p.pery && j == 0 && p.bc[2] == 2;
        dsf[3] = !p.pery && j == p.ny - 1 && p.bc[3] == 2;
        cx = (S)(-(p.uniform ? p.inv_dx : p.g.inv_dx[i]));
        cy = (S)(-(p.uniform ? p.inv_dy : p.g.inv_dy[j]));
        const double c1 = p.tau_field ? (12.0 * tau_o - dt) / (12.0 * tau_o + 3.0 * dt) : p.uc.c1;
        const double e1 = p.tau_field ? 4.0 * dt / (12.0 * tau_o + 3.0 * dt) : p.uc.e1;
        const double *mx = a.momX + 4 * cell;
        const EPoly ex = epoly(mx[0], mx[1], mx[2], mx[3], p.iRT, 1.0, DELTA);
        if (a.stage == 0) {
            // tilde f^+(t_n) = (5/4 c1 - 1/4) fhat + 5/4 e1 E^n (eq. f_tilde_1_3)
            const double k = 1.25 * e1;
            ownE[0] = (S)(k * ex.c0); ownE[1] = (S)(k * ex.c1x); ownE[2] = (S)(k * ex.c1y);
            ownE[3] = (S)(k * ex.c2xx); ownE[4] = (S)(k * ex.c2xy); ownE[5] = (S)(k * ex.c2yy);
            kx_own = (S)(1.25 * c1 - 0.25);
            aL = (S)(dt / 3.0);
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
            ownE[0] = (S)(a_En * en.c0); ownE[1] = (S)(a_En * en.c1x); ownE[2] = (S)(a_En * en.c1y);
            ownE[3] = (S)(a_En * en.c2xx); ownE[4] = (S)(a_En * en.c2xy); ownE[5] = (S)(a_En * en.c2yy);
            ownE2[0] = (S)(a_Ep * ex.c0); ownE2[1] = (S)(a_Ep * ex.c1x); ownE2[2] = (S)(a_Ep * ex.c1y);
            ownE2[3] = (S)(a_Ep * ex.c2xx); ownE2[4] = (S)(a_Ep * ex.c2xy); ownE2[5] = (S)(a_Ep * ex.c2yy);
            kx_own = (S)a_G;
            kf_own = (S)a_f;
            aL = (S)(4.0 * dt / 7.0);
        }
    }
    const S r0s = (S)(DELTA ? p.rho0 : 0.0);
    const S *__restrict__ X = (const S *)a.X;
    const S *__restrict__ F = (const S *)a.F;
    S *__restrict__ out = (S *)a.out;
    double m0 = 0, m1 = 0, m2 = 0;   // partial cell moments of the output

    for (int qa = q0; qa < q1; qa += p.lq_qs) {
        const int nqs = min(p.lq_qs, q1 - qa);
        __syncthreads();
        lq_fill<S, DELTA>(p, a, sh, i0, j0, qa, nqs);
        __syncthreads();
        if (!valid) continue;
        for (int s = 0; s < nqs; s++) {
            const int q = qa + s;
            const double xq = p.xi[q], yq = p.eta[q];
            const S xs = (S)xq, ys = (S)yq;
            const S sq = DELTA ? (S)1 : (S)p.w[q];
            const S *P = sh.planes + s * plane;
            double vv[4];
            bool ok[4];
            ok[0] = lq_xface(p, P, HX, i, lx + 2, ly + 2, j, xq, yq, h, vv[0]);
            ok[1] = lq_xface(p, P, HX, i + 1, lx + 3, ly + 2, j, xq, yq, h, vv[1]);
            ok[2] = lq_yface(p, P, HX, j, ly + 2, lx + 2, i, xq, yq, h, vv[2]);
            ok[3] = lq_yface(p, P, HX, j + 1, ly + 3, lx + 2, i, xq, yq, h, vv[3]);
            S fb[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                S bar;
                if (ok[k]) bar = (S)vv[k];
                else bar = dsf[k] ? (S)rw[k] * (S)p.wall_E[k * p.nq + q] - r0s : (S)0;
                fb[k] = fmaS(alpha_s[k], bar, sq * eval_rt(eb[k], xs, ys));
            }
            const S L = fmaS(xs * cx, fb[1] - fb[0], ys * cy * (fb[3] - fb[2]));
            S R;
            const S xo = X[q * n + cell];
            if (a.stage == 0) {
                R = fmaS(kx_own, xo, sq * eval_rt(ownE, xs, ys));
            } else {
                const S fo = F[q * n + cell];
                R = fmaS(kf_own, fo, fmaS(kx_own, xo, sq * (eval_rt(ownE, xs, ys) + eval_rt(ownE2, xs, ys))));
            }
            const S y = fmaS(aL, L, R);
            out[q * n + cell] = y;
            const double m = DELTA ? p.w[q] : 1.0;
            const double yd = (double)y;
            m0 = __builtin_fma(m, yd, m0);
            m1 = __builtin_fma(m * xq, yd, m1);
            m2 = __builtin_fma(m * yq, yd, m2);
        }
    }
    if (!valid) return;
    double *cp = a.cell_part + ((long long)chunk * n + cell) * 4;
    cp[0] = m0; cp[1] = m1; cp[2] = m2; cp[3] = 0.0;
}

// ---------------------------------------------------------------------------
// lq_cell_reduce: one thread per cell.
// ---------------------------------------------------------------------------
__device__ void lq_cell_reduce_body(const SweepParams &p, const LQStage &a, bool delta, long long cell)
{
    if (cell >= p.ncell) return;
    double s0 = 0, sx = 0, sy = 0;
    for (int c = 0; c < p.lq_nchunk; c++) {
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
__global__ void __launch_bounds__(256) lq_faces(const SweepParams p, const LQStage a)
{
    const int ntile = ((p.nx + p.tile_x - 1) / p.tile_x) * ((p.ny + p.tile_y - 1) / p.tile_y);
    lq_faces_body<S, DELTA>(p, a, blockIdx.x % ntile, blockIdx.x / ntile);
}

template <class S, bool DELTA>
__global__ void __launch_bounds__(256) lq_update(const SweepParams p, const LQStage a)
{
    const int ntile = ((p.nx + p.tile_x - 1) / p.tile_x) * ((p.ny + p.tile_y - 1) / p.tile_y);
    lq_update_body<S, DELTA>(p, a, blockIdx.x % ntile, blockIdx.x / ntile);
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
__global__ void __launch_bounds__(256) lq_faces_batched(const SweepParams *__restrict__ P,
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
                               const int4 *wf, int nf, const int4 *wc, int nc, int nthreads, size_t smem,
                               hipStream_t s)
{
    if (nt > 0) hipLaunchKernelGGL((lq_faces_batched<S, DELTA>), dim3(nt), dim3(nthreads), smem, s, P, A, wt);
    if (nf > 0) hipLaunchKernelGGL((lq_face_reduce_batched<DELTA>), dim3(nf), dim3(256), 0, s, P, A, wf);
    if (nt > 0) hipLaunchKernelGGL((lq_update_batched<S, DELTA>), dim3(nt), dim3(nthreads), smem, s, P, A, wt);
    if (nc > 0) hipLaunchKernelGGL((lq_cell_reduce_batched<DELTA>), dim3(nc), dim3(256), 0, s, P, A, wc);
    return hipGetLastError();
}

hipError_t launch_lq_stage_batched(bool delta, const SweepParams *P, const LQStage *A,
                                   const int4 *work_tiles, int ntiles, const int4 *work_faces, int nfaces,
                                   const int4 *work_cells, int ncells, int nthreads, size_t smem,
                                   hipStream_t s)
{
    return delta ? lq_batched_t<float, true>(P, A, work_tiles, ntiles, work_faces, nfaces, work_cells, ncells,
                                             nthreads, smem, s)
                 : lq_batched_t<double, false>(P, A, work_tiles, ntiles, work_faces, nfaces, work_cells,
                                               ncells, nthreads, smem, s);
}

size_t lq_smem_bytes(const SweepParams &p, bool delta)
{
    const size_t plane = (size_t)(p.tile_x + 4) * (p.tile_y + 4);
    return (delta ? 4 : 8) * plane * (p.lq_qs + 7);
}

template <class S, bool DELTA>
static hipError_t lq_stage_t(const SweepParams &p, const LQStage &a, hipStream_t s, int part)
{
    const int ntile = ((p.nx + p.tile_x - 1) / p.tile_x) * ((p.ny + p.tile_y - 1) / p.tile_y);
    const dim3 blk(p.tile_x * p.tile_y);
    const size_t smem = lq_smem_bytes(p, DELTA);
    const long long nface = (long long)(p.nx + 1) * p.ny + (long long)p.nx * (p.ny + 1);
    if (part == 0 || part < 0)
        hipLaunchKernelGGL((lq_faces<S, DELTA>), dim3(ntile * p.lq_nchunk), blk, smem, s, p, a);
    if (part == 1 || part < 0)
        hipLaunchKernelGGL((lq_face_reduce<DELTA>), dim3((unsigned)((nface + 255) / 256)), dim3(256), 0, s, p, a);
    if (part == 2 || part < 0)
        hipLaunchKernelGGL((lq_update<S, DELTA>), dim3(ntile * p.lq_nchunk), blk, smem, s, p, a);
    if (part == 3 || part < 0)
        hipLaunchKernelGGL((lq_cell_reduce<DELTA>), dim3((unsigned)((p.ncell + 255) / 256)), dim3(256), 0, s, p, a);
    return hipGetLastError();
}

hipError_t launch_lq_stage(bool delta, const SweepParams &p, const LQStage &a, hipStream_t s, int part)
{
    return delta ? lq_stage_t<float, true>(p, a, s, part) : lq_stage_t<double, false>(p, a, s, part);
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
