// Discrete adjoint of one T3S3-DUGKS step (any grid, walls and velocity
// set), in double.  For a step out = F(fhat; tau) the kernels map
// lambda_out = dL/d out to dL/d fhat and add dL/d tau, following the forward
// sequence of steps (1)-(4) backwards:
//   out = fhat/4 + 3/4 B + 3/4 W + dt/7 (3 L* + 4 L**)        (feqIntD3rdHat2_DS)
//   L** = D(f**), f** = a2 fbar** + b2 E(mom fbar**), fbar** = R_h2(B')
//   B' = c3 G + (1 - c3) E(mom G), W = -k (G - E(mom G))        (fbp_5_12, collisionterm)
//   G = 5/4 B - 1/4 fhat + dt/3 L*, L* = D(f*), ... R_h1(B)     (f_tilde_1_3, T2 step)
//   B = c1 fhat + (1 - c1) E(mom fhat)                          (f_bar_1_6)
// R_h is the interface expansion (one weight per window cell, upwind side
// fixed by the sign of the velocity), D the micro-flux; their transposes are
// taken in gather form (each cell / face sums what it fed), so no atomics are
// used and the result is deterministic.
//
// On periodic uniform grids the face values use fixed window weights per
// velocity (adj_face, gather_B); on walls and stretched grids the general
// kernels (adj_face_g, adj_gather_g) expand about each upwind cell with its
// own stencils and differentiate the wall rules.
//
// Every cell (or face) kernel runs a block of four waves over 64 cells: wave
// s takes the velocities q = s, s + 4, ... (the same in every lane, so the
// per-velocity weights are scalar loads), and sums over all velocities
// (moments, the adjoint of the equilibrium) are combined across the four
// waves through LDS in a fixed order.  At 256^2 cells that is four waves per
// SIMD instead of one.
#include "sweep_common.h"
#include "../../include/dugks.h"

namespace dk {

// periodic index of i in [-2, n + 1] (stencil offsets of at most two cells;
// grids have n >= 3)
__device__ __forceinline__ int wrp(int i, int n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// waves per block (velocity groups) and cells per block
constexpr int AL = 4;
constexpr int AC = 64;

// The cell (or face) of a thread and its velocity group.  Threads past the
// end take the last item (every thread takes part in the sums) and store
// nothing.
struct Lane {
    long long c;
    int s;
    bool ok;
};
__device__ __forceinline__ Lane lane_of(long long count)
{
    Lane l;
    l.s = __builtin_amdgcn_readfirstlane(threadIdx.x / AC);
    const long long c = (long long)blockIdx.x * AC + threadIdx.x % AC;
    l.ok = c < count;
    l.c = l.ok ? c : count - 1;
    return l;
}

// Sums of N values per cell over the block's four waves (wave order fixed).
template <int N>
__device__ __forceinline__ void wave_sum(double (&v)[N])
{
    __shared__ double buf[N][AL][AC];
    const int w = threadIdx.x / AC, l = threadIdx.x % AC;
#pragma unroll
    for (int k = 0; k < N; k++) buf[k][w][l] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; k++) v[k] = (buf[k][0][l] + buf[k][1][l]) + (buf[k][2][l] + buf[k][3][l]);
    __syncthreads();
}

// gradient of E_q(rho, m) with respect to (rho, mx, my), scaled by w_q:
// dE/drho = w (1 - (xi.u)^2/(2RT^2) + u^2/(2RT)), dE/dm = w (xi/RT + (xi.u) xi/RT^2 - u/RT)
__device__ __forceinline__ void grad_E(const AdjArgs &a, int q, double ux, double uy, double &gr,
                                       double &gx, double &gy)
{
    const double x = a.xi[q], y = a.eta[q], w = a.w[q];
    const double eu = x * ux + y * uy;
    gr = w * (1.0 - 0.5 * eu * eu * a.iRT * a.iRT + 0.5 * (ux * ux + uy * uy) * a.iRT);
    gx = w * (x * a.iRT + eu * x * a.iRT * a.iRT - ux * a.iRT);
    gy = w * (y * a.iRT + eu * y * a.iRT * a.iRT - uy * a.iRT);
}

__device__ __forceinline__ double eq_val(const AdjArgs &a, int q, double rho, double ux, double uy)
{
    const double eu = a.xi[q] * ux + a.eta[q] * uy;
    return a.w[q] * rho * (1.0 + eu * a.iRT + 0.5 * eu * eu * a.iRT * a.iRT -
                           0.5 * (ux * ux + uy * uy) * a.iRT);
}

// The lane's k-th velocity q = s + AL k.  Past the last velocity it is
// clamped to the last one and marked off: its loads stay in bounds and its
// terms are dropped, so that with the velocity count fixed at compile time the
// loop has a fixed trip count (used where a lane loads one value per
// velocity; the face and cell kernels, whose loads per velocity are windows
// of 12 or 24 values, keep a loop that stops at the last velocity, since
// issuing every window at once took more registers than it saved).
struct Vel {
    int q;
    bool on;
};
__device__ __forceinline__ Vel vel_of(const Lane &L, int k, int nq)
{
    const int q = L.s + AL * k;
    return q < nq ? Vel{q, true} : Vel{nq - 1, false};
}

// ---------------------------------------------------------------------------
// Primal intermediates of one step from fhat (storage units) and G (stage A
// output): B, moments of fhat, B' and moments of G, all in double.
// ---------------------------------------------------------------------------
template <class S, bool DELTA, int QC>
__global__ void __launch_bounds__(AL * AC) adj_prep(const AdjArgs a, double rho0, const S *__restrict__ fhat,
                                                    const S *__restrict__ G, double *__restrict__ fh_d,
                                                    double *__restrict__ B, double *__restrict__ M,
                                                    double *__restrict__ G_d, double *__restrict__ B2,
                                                    double *__restrict__ M2)
{
    const Lane L = lane_of(a.n);
    const long long c = L.c;
    const double tau = a.tau[c], dt = a.dt;
    const double c1 = (12.0 * tau - dt) / (12.0 * tau + 3.0 * dt);
    const double c3 = (24.0 * tau - 5.0 * dt) / (24.0 * tau + 4.0 * dt);
    auto val = [&](const S *src, int q) {
        return DELTA ? a.w[q] * ((double)src[q * a.n + c] + rho0) : (double)src[q * a.n + c];
    };
    if constexpr (QC > 0) {
        // both states' values of the lane's velocities, loaded together; one
        // sum over the waves for both sets of moments
        constexpr int NR = (QC + AL - 1) / AL;
        double vf[NR], vg[NR];
#pragma unroll
        for (int k = 0; k < NR; k++) {
            const Vel V = vel_of(L, k, QC);
            vf[k] = val(fhat, V.q);
            vg[k] = val(G, V.q);
        }
        double m6[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < NR; k++) {
            const Vel V = vel_of(L, k, QC);
            const double f = V.on ? vf[k] : 0.0, g = V.on ? vg[k] : 0.0;
            m6[0] += f;
            m6[1] += a.xi[V.q] * f;
            m6[2] += a.eta[V.q] * f;
            m6[3] += g;
            m6[4] += a.xi[V.q] * g;
            m6[5] += a.eta[V.q] * g;
        }
        wave_sum(m6);
        if (!L.ok) return;
        if (L.s == 0) {
            for (int k = 0; k < 3; k++) {
                M[3 * c + k] = m6[k];
                M2[3 * c + k] = m6[3 + k];
            }
        }
        const double ux = m6[1] / m6[0], uy = m6[2] / m6[0], gx = m6[4] / m6[3], gy = m6[5] / m6[3];
#pragma unroll
        for (int k = 0; k < NR; k++) {
            const Vel V = vel_of(L, k, QC);
            if (!V.on) break;
            const long long o = (long long)V.q * a.n + c;
            fh_d[o] = vf[k];
            G_d[o] = vg[k];
            B[o] = c1 * vf[k] + (1.0 - c1) * eq_val(a, V.q, m6[0], ux, uy);
            B2[o] = c3 * vg[k] + (1.0 - c3) * eq_val(a, V.q, m6[3], gx, gy);
        }
        return;
    }
    for (int pass = 0; pass < 2; pass++) {
        const S *src = pass ? G : fhat;
        double *dst = pass ? G_d : fh_d;
        double r = 0, mx = 0, my = 0;
        for (int q = L.s; q < a.nq; q += AL) {
            const double v = val(src, q);
            if (L.ok) dst[q * a.n + c] = v;
            r += v;
            mx += a.xi[q] * v;
            my += a.eta[q] * v;
        }
        double m3[3] = {r, mx, my};
        wave_sum(m3);
        r = m3[0];
        mx = m3[1];
        my = m3[2];
        double *Mo = pass ? M2 : M;
        if (L.ok && L.s == 0) {
            Mo[3 * c] = r;
            Mo[3 * c + 1] = mx;
            Mo[3 * c + 2] = my;
        }
        const double ux = mx / r, uy = my / r, cc = pass ? c3 : c1;
        double *Bo = pass ? B2 : B;
        for (int q = L.s; q < a.nq; q += AL)
            if (L.ok) Bo[q * a.n + c] = cc * val(src, q) + (1.0 - cc) * eq_val(a, q, r, ux, uy);
    }
}

// interface value of face (axis, i, j) for velocity q from the window of Bs
__device__ __forceinline__ double face_bar(const AdjArgs &a, const double *Bs, const double *cw, int axis,
                                           int i, int j, int q)
{
    const double *C = cw + 24 * q + (axis ? 12 : 0);
    const double *Bq = Bs + q * a.n;
    double v = 0.0;
    if (axis == 0) {   // x-face between cells i-1 and i of row j: cells (i-2+k, j-1+b)
        for (int k = 0; k < 4; k++)
            for (int b = 0; b < 3; b++)
                v = __builtin_fma(C[k * 3 + b], Bq[(long long)wrp(j - 1 + b, a.ny) * a.nx + wrp(i - 2 + k, a.nx)], v);
    } else {           // y-face between rows j-1 and j of column i: cells (i-1+b, j-2+k)
        for (int k = 0; k < 4; k++)
            for (int b = 0; b < 3; b++)
                v = __builtin_fma(C[k * 3 + b], Bq[(long long)wrp(j - 2 + k, a.ny) * a.nx + wrp(i - 1 + b, a.nx)], v);
    }
    return v;
}

// ---------------------------------------------------------------------------
// Face adjoint of one stage.  Thread = face (x-faces then y-faces, indexed by
// the cell whose west / south face it is).  lamL(c, q) is the adjoint of the
// micro-flux at cell c: scaleL * lamsrc(c, q).
// Outputs lam_fbar [axis][q][cell] and the tau sensitivity of the face.
// ---------------------------------------------------------------------------
template <int QC>
__global__ void __launch_bounds__(AL * AC) adj_face(const AdjArgs a, int stage, const double *__restrict__ Bs, const double *__restrict__ lamsrc,
                         double scaleL, double *__restrict__ lam_fbar, double *__restrict__ dtau_face)
{
    // QC > 0: the velocity count at compile time; face values and flux
    // adjoints stay in registers and each output is written once
    const int nq = QC > 0 ? QC : a.nq;
    const Lane L = lane_of(a.n);
    const int axis = blockIdx.y;
    const long long c = L.c, t = axis * a.n + c;
    const int i = (int)(c % a.nx), j = (int)(c / a.nx);
    const long long cl = axis ? (long long)wrp(j - 1, a.ny) * a.nx + i : (long long)j * a.nx + wrp(i - 1, a.nx);
    const double *cw = stage ? a.cC : a.cA;
    const double h = stage ? a.h2 : a.h1;
    const double tb = 0.5 * (a.tau[c] + a.tau[cl]);
    const double al = 2.0 * tb / (2.0 * tb + h), be = h / (2.0 * tb + h);
    const double dal = 2.0 * h / ((2.0 * tb + h) * (2.0 * tb + h));   // d alpha / d tau_b
    const double inv = axis ? a.idy : a.idx;
    // the lane's velocities: q = L.s + AL k
    constexpr int NR = QC > 0 ? (QC + AL - 1) / AL : 1;
    double vq[NR], lq[NR];
    // pass 1: interface moments
    double r = 0, mx = 0, my = 0;
#pragma unroll
    for (int k = 0; k < (QC > 0 ? NR : (nq + AL - 1) / AL); k++) {
        const int q = L.s + AL * k;
        if (q >= nq) break;
        const double v = face_bar(a, Bs, cw, axis, i, j, q);
        if (QC > 0) vq[QC > 0 ? k : 0] = v;
        r += v;
        mx += a.xi[q] * v;
        my += a.eta[q] * v;
    }
    {
        double m3[3] = {r, mx, my};
        wave_sum(m3);
        r = m3[0];
        mx = m3[1];
        my = m3[2];
    }
    const double ux = mx / r, uy = my / r;
    // pass 2: adjoint of the recovery f = al fbar + be E(mom fbar) and of D
    double gR = 0, gX = 0, gY = 0, dt_b = 0;
#pragma unroll
    for (int k = 0; k < (QC > 0 ? NR : (nq + AL - 1) / AL); k++) {
        const int q = L.s + AL * k;
        if (q >= nq) break;
        const double xn = axis ? a.eta[q] : a.xi[q];
        const double lf = xn * inv * scaleL * (lamsrc[q * a.n + c] - lamsrc[q * a.n + cl]);
        double er, ex, ey;
        grad_E(a, q, ux, uy, er, ex, ey);
        gR = __builtin_fma(be * lf, er, gR);
        gX = __builtin_fma(be * lf, ex, gX);
        gY = __builtin_fma(be * lf, ey, gY);
        const double v = QC > 0 ? vq[QC > 0 ? k : 0] : face_bar(a, Bs, cw, axis, i, j, q);
        dt_b = __builtin_fma(lf * dal, v - eq_val(a, q, r, ux, uy), dt_b);
        if (QC > 0)
            lq[QC > 0 ? k : 0] = lf;
        else if (L.ok)
            lam_fbar[((long long)axis * nq + q) * a.n + c] = al * lf;
    }
    {
        double g4[4] = {gR, gX, gY, dt_b};
        wave_sum(g4);
        gR = g4[0];
        gX = g4[1];
        gY = g4[2];
        dt_b = g4[3];
    }
    if (!L.ok) return;
#pragma unroll
    for (int k = 0; k < (QC > 0 ? NR : (nq + AL - 1) / AL); k++) {
        const int q = L.s + AL * k;
        if (q >= nq) break;
        const double base = QC > 0 ? al * lq[QC > 0 ? k : 0] : lam_fbar[((long long)axis * nq + q) * a.n + c];
        lam_fbar[((long long)axis * nq + q) * a.n + c] = base + (gR + gX * a.xi[q] + gY * a.eta[q]);
    }
    if (L.s == 0) dtau_face[t] = dt_b;
}

// transposed expansion: adjoint of B at cell (x0, y0), velocity q
__device__ __forceinline__ double gather_B(const AdjArgs &a, const double *cw, const double *lam_fbar,
                                           int x0, int y0, int q)
{
    const double *Cx = cw + 24 * q, *Cy = Cx + 12;
    const double *lx = lam_fbar + (long long)q * a.n;
    const double *ly = lam_fbar + ((long long)a.nq + q) * a.n;
    double v = 0.0;
    for (int k = 0; k < 4; k++)
        for (int b = 0; b < 3; b++) {
            const int i = wrp(x0 + 2 - k, a.nx), j = wrp(y0 + 1 - b, a.ny);
            v = __builtin_fma(Cx[k * 3 + b], lx[(long long)j * a.nx + i], v);
            const int iy = wrp(x0 + 1 - b, a.nx), jy = wrp(y0 + 2 - k, a.ny);
            v = __builtin_fma(Cy[k * 3 + b], ly[(long long)jy * a.nx + iy], v);
        }
    return v;
}

// half of the tau sensitivity of the four faces of a cell
__device__ __forceinline__ double faces_tau(const AdjArgs &a, const double *dtf, int i, int j)
{
    const long long c = (long long)j * a.nx + i;
    return 0.5 * (dtf[c] + dtf[(long long)j * a.nx + wrp(i + 1, a.nx)] + dtf[a.n + c] +
                  dtf[a.n + (long long)wrp(j + 1, a.ny) * a.nx + i]);
}

// ---------------------------------------------------------------------------
// Walls and stretched grids.  Faces are numbered as in the forward sweep:
// x-face (fi, j) = j (nx + 1) + fi, then y-face (i, fj) = nxf + fj nx + i; on a
// periodic axis the last face is the first one and is not formed.  The
// interface value of velocity q at a face is the expansion (eq. flux_DS) of B
// about its upwind cell with that cell's 3-point stencils (one-sided next to a
// wall); at a wall the velocities leaving it take the wall's value (eq. BB,
// or the diffuse-scattering rule) and a velocity parallel to the wall the
// whole expansion of the wall cell.
// ---------------------------------------------------------------------------
// d(expansion about cell (iu, ju) at offsets (dx, dy)) / d B(cell at offset
// (kx, ky) from it), with kx, ky in [-2, 2]
__device__ __forceinline__ double expand_weight(const AdjArgs &a, int iu, int ju, int kx, int ky, double dx,
                                                double dy)
{
    const int k = kx - a.sx_off[iu], l = ky - a.sy_off[ju];
    const bool kv = k >= 0 && k < 3, lv = l >= 0 && l < 3;
    double w = (kx == 0 && ky == 0) ? 1.0 : 0.0;
    if (ky == 0 && kv) w += dx * a.sx_d1[3 * iu + k] + a.kappa * dx * dx * a.sx_d2[3 * iu + k];
    if (kx == 0 && lv) w += dy * a.sy_d1[3 * ju + l] + a.kappa * dy * dy * a.sy_d2[3 * ju + l];
    if (kv && lv) w += 2.0 * a.kappa * dx * dy * a.sx_d1[3 * iu + k] * a.sy_d1[3 * ju + l];
    return w;
}

// the expansion itself (its weights applied to the stencil of the cell)
__device__ __forceinline__ double expand_at(const AdjArgs &a, const double *Bq, int iu, int ju, double dx,
                                            double dy)
{
    double v = 0.0;
    for (int ky = -2; ky <= 2; ky++)
        for (int kx = -2; kx <= 2; kx++) {
            const double w = expand_weight(a, iu, ju, kx, ky, dx, dy);
            if (w == 0.0) continue;
            const int i = a.perx ? wrp(iu + kx, a.nx) : iu + kx, j = a.pery ? wrp(ju + ky, a.ny) : ju + ky;
            v = __builtin_fma(w, Bq[(long long)j * a.nx + i], v);
        }
    return v;
}

// storage-free description of one face of the natural numbering
struct FaceG {
    int axis;        // 0: x-face, 1: y-face
    int cl, cu;      // the cells below / above (west / east, south / north); -1 outside
    int side;        // wall side (0 W, 1 E, 2 S, 3 N) or -1
    int il, jl, iu, ju;   // column and row of cl and cu (valid where the cell is)
};

__device__ __forceinline__ bool face_of(const AdjArgs &a, long long f, FaceG &g)
{
    const long long nxf = (long long)(a.nx + 1) * a.ny;
    g.side = -1;
    if (f < nxf) {
        const int j = (int)(f / (a.nx + 1)), fi = (int)(f % (a.nx + 1));
        if (a.perx && fi == a.nx) return false;
        g.axis = 0;
        g.jl = g.ju = j;
        g.iu = fi;
        g.il = a.perx ? wrp(fi - 1, a.nx) : fi - 1;
        if (!a.perx && fi == 0) g.side = 0;
        if (!a.perx && fi == a.nx) g.side = 1;
    } else {
        const long long t = f - nxf;
        const int fj = (int)(t / a.nx), i = (int)(t % a.nx);
        if (a.pery && fj == a.ny) return false;
        g.axis = 1;
        g.il = g.iu = i;
        g.ju = fj;
        g.jl = a.pery ? wrp(fj - 1, a.ny) : fj - 1;
        if (!a.pery && fj == 0) g.side = 2;
        if (!a.pery && fj == a.ny) g.side = 3;
    }
    g.cl = (g.side == 0 || g.side == 2) ? -1 : g.jl * a.nx + g.il;
    g.cu = (g.side == 1 || g.side == 3) ? -1 : g.ju * a.nx + g.iu;
    return true;
}

// the face's outward wall normal component of velocity q (sides 0..3)
__device__ __forceinline__ double wall_xn(const AdjArgs &a, int side, int q)
{
    return side == 0 ? -a.xi[q] : side == 1 ? a.xi[q] : side == 2 ? -a.eta[q] : a.eta[q];
}

// w_q P_q(u_w): the equilibrium of unit density at the wall's velocity
__device__ __forceinline__ double wall_e1(const AdjArgs &a, int side, int q)
{
    const double ux = a.uw[side][0], uy = a.uw[side][1];
    const double eu = a.xi[q] * ux + a.eta[q] * uy, uu = ux * ux + uy * uy;
    return a.w[q] * (1.0 + eu * a.iRT + 0.5 * eu * eu * a.iRT * a.iRT - 0.5 * uu * a.iRT);
}

// Expanded interface value of velocity q at face g (walls: the arriving and
// parallel velocities only; 0 for the leaving ones).
__device__ __forceinline__ double face_expand(const AdjArgs &a, const FaceG &g, const double *Bq, int q, double h)
{
    const double ex = a.xi[q], ey = a.eta[q];
    const double cn = g.axis ? ey : ex;   // velocity component normal to the face
    if (g.axis == 0) {
        const double dy = -ey * h;
        if (g.side == 0) return ex > 0.0 ? 0.0 : expand_at(a, Bq, g.iu, g.ju, a.dxr[g.iu] - ex * h, dy);
        if (g.side == 1) return ex < 0.0 ? 0.0 : expand_at(a, Bq, g.il, g.jl, a.dxl[g.il + 1] - ex * h, dy);
        if (cn > 0.0) return expand_at(a, Bq, g.il, g.jl, a.dxl[g.il + 1] - ex * h, dy);
        if (cn < 0.0) return expand_at(a, Bq, g.iu, g.ju, a.dxr[g.iu] - ex * h, dy);
        return 0.5 * (expand_at(a, Bq, g.il, g.jl, a.dxl[g.il + 1], dy) + expand_at(a, Bq, g.iu, g.ju, a.dxr[g.iu], dy));
    }
    const double dx = -ex * h;
    if (g.side == 2) return ey > 0.0 ? 0.0 : expand_at(a, Bq, g.iu, g.ju, dx, a.dyr[g.ju] - ey * h);
    if (g.side == 3) return ey < 0.0 ? 0.0 : expand_at(a, Bq, g.il, g.jl, dx, a.dyl[g.jl + 1] - ey * h);
    if (cn > 0.0) return expand_at(a, Bq, g.il, g.jl, dx, a.dyl[g.jl + 1] - ey * h);
    if (cn < 0.0) return expand_at(a, Bq, g.iu, g.ju, dx, a.dyr[g.ju] - ey * h);
    return 0.5 * (expand_at(a, Bq, g.il, g.jl, dx, a.dyl[g.jl + 1]) + expand_at(a, Bq, g.iu, g.ju, dx, a.dyr[g.ju]));
}

// Face adjoint of one stage on any grid: thread per face of the natural
// numbering.  Out: lam_fbar [q][face] (the adjoint of the expanded interface
// values; zero for velocities leaving a wall, whose adjoint has been passed
// to what the wall rule takes them from), dtau_face [face] and, at
// bounce-back walls, lam_rho [face] (adjoint of the density of the wall
// cell's stage input).  lam_fbar doubles as the scratch of the face values.
__global__ void __launch_bounds__(256) adj_face_g(const AdjArgs a, int stage, const double *__restrict__ Bs,
                                                  const double *__restrict__ Mx, const double *__restrict__ lamsrc,
                                                  double scaleL, double *__restrict__ lam_fbar,
                                                  double *__restrict__ dtau_face, double *__restrict__ lam_rho)
{
    const long long nface = (long long)(a.nx + 1) * a.ny + (long long)a.nx * (a.ny + 1);
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nface) return;
    FaceG g;
    if (!face_of(a, f, g)) return;
    const int nq = a.nq;
    const double h = stage ? a.h2 : a.h1;
    double *V = lam_fbar + f;   // V[q * nface]
    // tau at the face: the mean of its cells, the wall cell's at a wall
    const double tb = g.cl < 0 ? a.tau[g.cu] : g.cu < 0 ? a.tau[g.cl] : 0.5 * (a.tau[g.cl] + a.tau[g.cu]);
    const double al = 2.0 * tb / (2.0 * tb + h), be = h / (2.0 * tb + h);
    const double dal = 2.0 * h / ((2.0 * tb + h) * (2.0 * tb + h));
    const int wc = g.cl < 0 ? g.cu : g.cl;   // the cell next to a wall
    const int kind = g.side >= 0 ? a.bc[g.side] : 0;
    // pass 1: interface values, the wall rule, moments
    double num = 0.0, den = 0.0;
    for (int q = 0; q < nq; q++) {
        const double v = face_expand(a, g, Bs + (long long)q * a.n, q, h);
        V[q * nface] = v;
        if (g.side >= 0) {
            const double xn = wall_xn(a, g.side, q);
            if (xn > 0.0) num += xn * v;
            if (xn < 0.0) den += -xn * wall_e1(a, g.side, q);
        }
    }
    if (g.side >= 0) {
        for (int q = 0; q < nq; q++) {
            if (wall_xn(a, g.side, q) >= 0.0) continue;
            double v;
            if (kind == DUGKS_BC_BOUNCE_BACK) {
                const double xu = a.xi[q] * a.uw[g.side][0] + a.eta[q] * a.uw[g.side][1];
                v = V[a.opp[q] * nface] + 2.0 * Mx[3 * wc] * a.w[q] * xu * a.iRT;
            } else {
                v = num / den * wall_e1(a, g.side, q);
            }
            V[q * nface] = v;
        }
    }
    double r = 0, mx = 0, my = 0;
    for (int q = 0; q < nq; q++) {
        const double v = V[q * nface];
        r += v;
        mx += a.xi[q] * v;
        my += a.eta[q] * v;
    }
    const double ux = mx / r, uy = my / r;
    // pass 2: adjoint of the micro-flux and of the recovery f = al fbar + be E
    const double iu_ = g.cu >= 0 ? (g.axis ? a.inv_dy[g.ju] : a.inv_dx[g.iu]) : 0.0;
    const double il_ = g.cl >= 0 ? (g.axis ? a.inv_dy[g.jl] : a.inv_dx[g.il]) : 0.0;
    double gR = 0, gX = 0, gY = 0, dt_b = 0;
    for (int q = 0; q < nq; q++) {
        const double xn = g.axis ? a.eta[q] : a.xi[q];
        const double su = g.cu >= 0 ? lamsrc[(long long)q * a.n + g.cu] * iu_ : 0.0;
        const double sl = g.cl >= 0 ? lamsrc[(long long)q * a.n + g.cl] * il_ : 0.0;
        const double lf = xn * scaleL * (su - sl);
        double er, ex, ey;
        grad_E(a, q, ux, uy, er, ex, ey);
        gR = __builtin_fma(be * lf, er, gR);
        gX = __builtin_fma(be * lf, ex, gX);
        gY = __builtin_fma(be * lf, ey, gY);
        const double v = V[q * nface];
        dt_b = __builtin_fma(lf * dal, v - eq_val(a, q, r, ux, uy), dt_b);
        V[q * nface] = al * lf;
    }
    for (int q = 0; q < nq; q++) V[q * nface] += gR + gX * a.xi[q] + gY * a.eta[q];
    // adjoint of the wall rule: what the leaving velocities were taken from
    double lrho = 0.0;
    if (g.side >= 0) {
        if (kind == DUGKS_BC_BOUNCE_BACK) {
            for (int q = 0; q < nq; q++) {
                if (wall_xn(a, g.side, q) >= 0.0) continue;
                const double l = V[q * nface];
                const double xu = a.xi[q] * a.uw[g.side][0] + a.eta[q] * a.uw[g.side][1];
                V[a.opp[q] * nface] += l;
                lrho = __builtin_fma(l, 2.0 * a.w[q] * xu * a.iRT, lrho);
                V[q * nface] = 0.0;
            }
        } else {
            double lrw = 0.0;
            for (int q = 0; q < nq; q++)
                if (wall_xn(a, g.side, q) < 0.0) lrw = __builtin_fma(V[q * nface], wall_e1(a, g.side, q), lrw);
            for (int q = 0; q < nq; q++) {
                const double xn = wall_xn(a, g.side, q);
                if (xn > 0.0) V[q * nface] += lrw * xn / den;
                if (xn < 0.0) V[q * nface] = 0.0;
            }
        }
    }
    dtau_face[f] = dt_b;
    lam_rho[f] = lrho;
}

// Transposed expansion on any grid, thread per (cell, velocity): lamBg(c, q)
// = sum over the faces whose interface value of q was expanded about a cell
// whose stencil holds c, of that expansion's weight on c times lam_fbar.
__global__ void __launch_bounds__(256) adj_gather_g(const AdjArgs a, int stage, const double *__restrict__ lam_fbar,
                                                    double *__restrict__ lamBg)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)a.n * a.nq) return;
    const int q = (int)(t / a.n);
    const long long c = t - (long long)q * a.n;
    const int ci = (int)(c % a.nx), cj = (int)(c / a.nx);
    const long long nxf = (long long)(a.nx + 1) * a.ny;
    const long long nface = nxf + (long long)a.nx * (a.ny + 1);
    const double h = stage ? a.h2 : a.h1;
    const double ex = a.xi[q], ey = a.eta[q];
    const double *L = lam_fbar + (long long)q * nface;
    double acc = 0.0;
    for (int dy_ = -2; dy_ <= 2; dy_++) {
        int ju = cj - dy_;
        if (a.pery) ju = wrp(ju, a.ny); else if (ju < 0 || ju >= a.ny) continue;
        for (int dx_ = -2; dx_ <= 2; dx_++) {
            int iu = ci - dx_;
            if (a.perx) iu = wrp(iu, a.nx); else if (iu < 0 || iu >= a.nx) continue;
            // c sits at offset (dx_, dy_) from the expansion cell (iu, ju)
            const bool wW = !a.perx && iu == 0, wE = !a.perx && iu == a.nx - 1;
            const bool wS = !a.pery && ju == 0, wN = !a.pery && ju == a.ny - 1;
            // x-faces expanded about (iu, ju): east if ex > 0, west if ex < 0,
            // both halves if ex = 0 (the whole value at a wall face)
            const double dyx = -ey * h;
            if (ex >= 0.0) {
                const double wt = ex > 0.0 ? 1.0 : (wE ? 1.0 : 0.5);
                const int fi = (a.perx && iu + 1 == a.nx) ? 0 : iu + 1;
                const double wgt = expand_weight(a, iu, ju, dx_, dy_, a.dxl[iu + 1] - ex * h, dyx);
                if (wgt != 0.0) acc = __builtin_fma(wt * wgt, L[(long long)ju * (a.nx + 1) + fi], acc);
            }
            if (ex <= 0.0) {
                const double wt = ex < 0.0 ? 1.0 : (wW ? 1.0 : 0.5);
                const double wgt = expand_weight(a, iu, ju, dx_, dy_, a.dxr[iu] - ex * h, dyx);
                if (wgt != 0.0) acc = __builtin_fma(wt * wgt, L[(long long)ju * (a.nx + 1) + iu], acc);
            }
            const double dxy = -ex * h;
            if (ey >= 0.0) {
                const double wt = ey > 0.0 ? 1.0 : (wN ? 1.0 : 0.5);
                const int fj = (a.pery && ju + 1 == a.ny) ? 0 : ju + 1;
                const double wgt = expand_weight(a, iu, ju, dx_, dy_, dxy, a.dyl[ju + 1] - ey * h);
                if (wgt != 0.0) acc = __builtin_fma(wt * wgt, L[nxf + (long long)fj * a.nx + iu], acc);
            }
            if (ey <= 0.0) {
                const double wt = ey < 0.0 ? 1.0 : (wS ? 1.0 : 0.5);
                const double wgt = expand_weight(a, iu, ju, dx_, dy_, dxy, a.dyr[ju] - ey * h);
                if (wgt != 0.0) acc = __builtin_fma(wt * wgt, L[nxf + (long long)ju * a.nx + iu], acc);
            }
        }
    }
    lamBg[t] = acc;
}

// tau sensitivity a cell takes from its faces (half of an interior face's,
// all of a wall face's) and the density adjoint of its bounce-back wall faces
__device__ __forceinline__ void cell_faces_g(const AdjArgs &a, const double *dtf, const double *lam_rho, int i,
                                             int j, double &dtc, double &lrho)
{
    const long long nxf = (long long)(a.nx + 1) * a.ny;
    const long long fw = (long long)j * (a.nx + 1) + i;
    const long long fe = (long long)j * (a.nx + 1) + ((a.perx && i + 1 == a.nx) ? 0 : i + 1);
    const long long fs = nxf + (long long)j * a.nx + i;
    const long long fn = nxf + (long long)((a.pery && j + 1 == a.ny) ? 0 : j + 1) * a.nx + i;
    const bool wW = !a.perx && i == 0, wE = !a.perx && i == a.nx - 1;
    const bool wS = !a.pery && j == 0, wN = !a.pery && j == a.ny - 1;
    dtc = (wW ? 1.0 : 0.5) * dtf[fw] + (wE ? 1.0 : 0.5) * dtf[fe] + (wS ? 1.0 : 0.5) * dtf[fs] +
          (wN ? 1.0 : 0.5) * dtf[fn];
    lrho = (wW ? lam_rho[fw] : 0.0) + (wE ? lam_rho[fe] : 0.0) + (wS ? lam_rho[fs] : 0.0) +
           (wN ? lam_rho[fn] : 0.0);
}

// ---------------------------------------------------------------------------
// Cell adjoint of stage C: from lambda_out and the stage C face adjoint to
// lambda of L* (lamLs), the partial adjoints of B (lamB) and fhat (lamF).
// ---------------------------------------------------------------------------
template <int QC, bool GEN>
__global__ void __launch_bounds__(AL * AC) adj_cellC(const AdjArgs a, const double *__restrict__ lam_out, const double *__restrict__ lam_fbar,
                          const double *__restrict__ dtau_face, const double *__restrict__ G_d,
                          const double *__restrict__ M2, double *__restrict__ lamLs, double *__restrict__ lamB,
                          double *__restrict__ lamF, double *__restrict__ dtau, const double *__restrict__ lam_rho,
                          const double *__restrict__ lamBg)
{
    const Lane L = lane_of(a.n);
    const long long c = L.c;
    const int i = (int)(c % a.nx), j = (int)(c / a.nx);
    const double tau = a.tau[c], dt = a.dt;
    const double c3 = (24.0 * tau - 5.0 * dt) / (24.0 * tau + 4.0 * dt);
    const double dc3 = 216.0 * dt / ((24.0 * tau + 4.0 * dt) * (24.0 * tau + 4.0 * dt));
    const double kw = 6.0 * dt / (6.0 * tau + dt);
    const double dkw = -36.0 * dt / ((6.0 * tau + dt) * (6.0 * tau + dt));
    const double r = M2[3 * c], ux = M2[3 * c + 1] / r, uy = M2[3 * c + 2] / r;
    double gR = 0, gX = 0, gY = 0, dtc = 0.0, lrho = 0.0;
    if (GEN) cell_faces_g(a, dtau_face, lam_rho, i, j, dtc, lrho);
    else dtc = faces_tau(a, dtau_face, i, j);
    if (L.s != 0) dtc = lrho = 0.0;
    // the density of G at bounce-back walls (its adjoint enters every q as gR does)
    gR = lrho;
    // lam_G (partial) into lamLs as scratch
    const int nq = QC > 0 ? QC : a.nq;
#pragma unroll
    for (int k = 0; k < (QC > 0 ? (QC + AL - 1) / AL : (nq + AL - 1) / AL); k++) {
        const int q = L.s + AL * k;
        if (q >= nq) break;
        const double lB2 = GEN ? lamBg[(long long)q * a.n + c] : gather_B(a, a.cC, lam_fbar, i, j, q);
        const double lW = 0.75 * lam_out[q * a.n + c];
        const double e = eq_val(a, q, r, ux, uy);
        const double gme = G_d[q * a.n + c] - e;
        dtc += lB2 * dc3 * gme - lW * dkw * gme;
        const double coefE = (1.0 - c3) * lB2 + kw * lW;   // weight of E'_q
        double er, ex, ey;
        grad_E(a, q, ux, uy, er, ex, ey);
        gR = __builtin_fma(coefE, er, gR);
        gX = __builtin_fma(coefE, ex, gX);
        gY = __builtin_fma(coefE, ey, gY);
        if (L.ok) lamLs[q * a.n + c] = c3 * lB2 - kw * lW;
    }
    {
        double g4[4] = {gR, gX, gY, dtc};
        wave_sum(g4);
        gR = g4[0];
        gX = g4[1];
        gY = g4[2];
        dtc = g4[3];
    }
    if (!L.ok) return;
#pragma unroll
    for (int k = 0; k < (QC > 0 ? (QC + AL - 1) / AL : (nq + AL - 1) / AL); k++) {
        const int q = L.s + AL * k;
        if (q >= nq) break;
        const double lG = lamLs[q * a.n + c] + gR + gX * a.xi[q] + gY * a.eta[q];
        const double lo = lam_out[q * a.n + c];
        lamLs[q * a.n + c] = (3.0 * dt / 7.0) * lo + (dt / 3.0) * lG;   // adjoint of L*
        lamB[q * a.n + c] = 0.75 * lo + 1.25 * lG;                      // from out and tilde f^+
        lamF[q * a.n + c] = 0.25 * lo - 0.25 * lG;
    }
    if (L.s == 0) dtau[c] += dtc;
}

// ---------------------------------------------------------------------------
// Cell adjoint of stage A: lambda(fhat(t_n)).
// ---------------------------------------------------------------------------
template <int QC, bool GEN>
__global__ void __launch_bounds__(AL * AC) adj_cellA(const AdjArgs a, const double *__restrict__ lam_fbar, const double *__restrict__ dtau_face,
                          const double *__restrict__ fh_d, const double *__restrict__ M,
                          const double *__restrict__ lamB, const double *__restrict__ lamF,
                          double *__restrict__ lam_in, double *__restrict__ dtau, const double *__restrict__ lam_rho,
                          const double *__restrict__ lamBg)
{
    const Lane L = lane_of(a.n);
    const long long c = L.c;
    const int i = (int)(c % a.nx), j = (int)(c / a.nx);
    const double tau = a.tau[c], dt = a.dt;
    const double c1 = (12.0 * tau - dt) / (12.0 * tau + 3.0 * dt);
    const double dc1 = 48.0 * dt / ((12.0 * tau + 3.0 * dt) * (12.0 * tau + 3.0 * dt));
    const double r = M[3 * c], ux = M[3 * c + 1] / r, uy = M[3 * c + 2] / r;
    double gR = 0, gX = 0, gY = 0, dtc = 0.0, lrho = 0.0;
    if (GEN) cell_faces_g(a, dtau_face, lam_rho, i, j, dtc, lrho);
    else dtc = faces_tau(a, dtau_face, i, j);
    if (L.s != 0) dtc = lrho = 0.0;
    // the density of fhat at bounce-back walls (its adjoint enters every q as gR does)
    gR = lrho;
    const int nq = QC > 0 ? QC : a.nq;
#pragma unroll
    for (int k = 0; k < (QC > 0 ? (QC + AL - 1) / AL : (nq + AL - 1) / AL); k++) {
        const int q = L.s + AL * k;
        if (q >= nq) break;
        const double lB = lamB[q * a.n + c] +
                          (GEN ? lamBg[(long long)q * a.n + c] : gather_B(a, a.cA, lam_fbar, i, j, q));
        const double e = eq_val(a, q, r, ux, uy);
        dtc += lB * dc1 * (fh_d[q * a.n + c] - e);
        double er, ex, ey;
        grad_E(a, q, ux, uy, er, ex, ey);
        const double ce = (1.0 - c1) * lB;
        gR = __builtin_fma(ce, er, gR);
        gX = __builtin_fma(ce, ex, gX);
        gY = __builtin_fma(ce, ey, gY);
        if (L.ok) lam_in[q * a.n + c] = lamF[q * a.n + c] + c1 * lB;
    }
    {
        double g4[4] = {gR, gX, gY, dtc};
        wave_sum(g4);
        gR = g4[0];
        gX = g4[1];
        gY = g4[2];
        dtc = g4[3];
    }
    if (!L.ok) return;
#pragma unroll
    for (int k = 0; k < (QC > 0 ? (QC + AL - 1) / AL : (nq + AL - 1) / AL); k++) {
        const int q = L.s + AL * k;
        if (q >= nq) break;
        lam_in[q * a.n + c] += gR + gX * a.xi[q] + gY * a.eta[q];
    }
    if (L.s == 0) dtau[c] += dtc;
}

// seed: lambda = dL/dfhat of L = sum_j a_j rho_j + b_j . u_j at the final state
__global__ void adj_seed(const AdjArgs a, const double *__restrict__ fh_d, const double *__restrict__ dL_drho,
                         const double *__restrict__ dL_du, double *__restrict__ lam)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    double r = 0, mx = 0, my = 0;
    for (int q = 0; q < a.nq; q++) {
        const double v = fh_d[q * a.n + c];
        r += v;
        mx += a.xi[q] * v;
        my += a.eta[q] * v;
    }
    const double ux = mx / r, uy = my / r;
    const double ar = dL_drho ? dL_drho[c] : 0.0, bx = dL_du[c], by = dL_du[a.n + c];
    for (int q = 0; q < a.nq; q++)
        lam[q * a.n + c] = ar + (bx * (a.xi[q] - ux) + by * (a.eta[q] - uy)) / r;
}

// adjoint of fhat = f + dt/(4 tau) (f - E(mom f)) at t = 0
__global__ void adj_init(const AdjArgs a, const double *__restrict__ f0, const double *__restrict__ lam,
                         double *__restrict__ dL_df0, double *__restrict__ dtau)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    double r = 0, mx = 0, my = 0;
    for (int q = 0; q < a.nq; q++) {
        const double v = f0[q * a.n + c];
        r += v;
        mx += a.xi[q] * v;
        my += a.eta[q] * v;
    }
    const double ux = mx / r, uy = my / r, tau = a.tau[c];
    const double k = a.dt / (4.0 * tau), dk = -a.dt / (4.0 * tau * tau);
    double gR = 0, gX = 0, gY = 0, dtc = 0;
    for (int q = 0; q < a.nq; q++) {
        const double l = lam[q * a.n + c];
        double er, ex, ey;
        grad_E(a, q, ux, uy, er, ex, ey);
        gR = __builtin_fma(l, er, gR);
        gX = __builtin_fma(l, ex, gX);
        gY = __builtin_fma(l, ey, gY);
        dtc = __builtin_fma(l * dk, f0[q * a.n + c] - eq_val(a, q, r, ux, uy), dtc);
    }
    for (int q = 0; q < a.nq; q++)
        dL_df0[q * a.n + c] = (1.0 + k) * lam[q * a.n + c] - k * (gR + gX * a.xi[q] + gY * a.eta[q]);
    dtau[c] += dtc;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline dim3 g1(long long n) { return dim3((unsigned)((n + 255) / 256)); }
// blocks of AL waves over AC cells (faces: one grid row per axis)
static inline dim3 gc(long long n, int rows = 1) { return dim3((unsigned)((n + AC - 1) / AC), rows); }

hipError_t adj_launch_prep(const AdjArgs &a, bool delta, double rho0, const void *fhat, const void *G,
                           double *fh_d, double *B, double *M, double *G_d, double *B2, double *M2, hipStream_t s)
{
    // the velocity count fixed at compile time for D2Q9
    if (delta && a.nq == 9)
        hipLaunchKernelGGL((adj_prep<float, true, 9>), gc(a.n), dim3(AL * AC), 0, s, a, rho0, (const float *)fhat,
                           (const float *)G, fh_d, B, M, G_d, B2, M2);
    else if (delta)
        hipLaunchKernelGGL((adj_prep<float, true, 0>), gc(a.n), dim3(AL * AC), 0, s, a, rho0, (const float *)fhat,
                           (const float *)G, fh_d, B, M, G_d, B2, M2);
    else if (a.nq == 9)
        hipLaunchKernelGGL((adj_prep<double, false, 9>), gc(a.n), dim3(AL * AC), 0, s, a, rho0, (const double *)fhat,
                           (const double *)G, fh_d, B, M, G_d, B2, M2);
    else
        hipLaunchKernelGGL((adj_prep<double, false, 0>), gc(a.n), dim3(AL * AC), 0, s, a, rho0, (const double *)fhat,
                           (const double *)G, fh_d, B, M, G_d, B2, M2);
    return hipGetLastError();
}

// face adjoint with the velocity count fixed at compile time for D2Q9 (at 37
// velocities the unrolled kernel no longer fits the register file)
static void launch_adj_face(const AdjArgs &a, int stage, const double *Bs, const double *lamsrc, double scaleL,
                            double *lam_fbar, double *dtau_face, hipStream_t s)
{
    if (a.nq == 9)
        hipLaunchKernelGGL(adj_face<9>, gc(a.n, 2), dim3(AL * AC), 0, s, a, stage, Bs, lamsrc, scaleL, lam_fbar,
                           dtau_face);
    else
        hipLaunchKernelGGL(adj_face<0>, gc(a.n, 2), dim3(AL * AC), 0, s, a, stage, Bs, lamsrc, scaleL, lam_fbar,
                           dtau_face);
}

hipError_t adj_launch_step(const AdjArgs &a, const double *lam_out, double *lam_in, const double *fh_d,
                           const double *B, const double *M, const double *G_d, const double *B2,
                           const double *M2, double *lam_fbar, double *dtau_face, double *lamLs, double *lamB,
                           double *lamF, double *dtau, double *lam_rho, double *lamBg, hipStream_t s)
{
    if (a.general) {
        const long long nface = (long long)(a.nx + 1) * a.ny + (long long)a.nx * (a.ny + 1);
        // stage C (reverse of steps (3)-(4))
        hipLaunchKernelGGL(adj_face_g, g1(nface), dim3(256), 0, s, a, 1, B2, M2, lam_out, 4.0 * a.dt / 7.0, lam_fbar,
                           dtau_face, lam_rho);
        hipLaunchKernelGGL(adj_gather_g, g1((long long)a.n * a.nq), dim3(256), 0, s, a, 1, lam_fbar, lamBg);
        hipLaunchKernelGGL((adj_cellC<0, true>), gc(a.n), dim3(AL * AC), 0, s, a, lam_out, lam_fbar, dtau_face, G_d,
                           M2, lamLs, lamB, lamF, dtau, lam_rho, lamBg);
        // stage A (reverse of steps (1)-(2))
        hipLaunchKernelGGL(adj_face_g, g1(nface), dim3(256), 0, s, a, 0, B, M, lamLs, 1.0, lam_fbar, dtau_face,
                           lam_rho);
        hipLaunchKernelGGL(adj_gather_g, g1((long long)a.n * a.nq), dim3(256), 0, s, a, 0, lam_fbar, lamBg);
        hipLaunchKernelGGL((adj_cellA<0, true>), gc(a.n), dim3(AL * AC), 0, s, a, lam_fbar, dtau_face, fh_d, M, lamB,
                           lamF, lam_in, dtau, lam_rho, lamBg);
        return hipGetLastError();
    }
    // stage C (reverse of steps (3)-(4)); the cell adjoints with the velocity
    // count fixed at compile time for D2Q9 (their gathers are issued together)
    launch_adj_face(a, 1, B2, lam_out, 4.0 * a.dt / 7.0, lam_fbar, dtau_face, s);
    if (a.nq == 9)
        hipLaunchKernelGGL((adj_cellC<9, false>), gc(a.n), dim3(AL * AC), 0, s, a, lam_out, lam_fbar, dtau_face, G_d,
                           M2, lamLs, lamB, lamF, dtau, nullptr, nullptr);
    else
        hipLaunchKernelGGL((adj_cellC<0, false>), gc(a.n), dim3(AL * AC), 0, s, a, lam_out, lam_fbar, dtau_face, G_d,
                           M2, lamLs, lamB, lamF, dtau, nullptr, nullptr);
    // stage A (reverse of steps (1)-(2))
    launch_adj_face(a, 0, B, lamLs, 1.0, lam_fbar, dtau_face, s);
    if (a.nq == 9)
        hipLaunchKernelGGL((adj_cellA<9, false>), gc(a.n), dim3(AL * AC), 0, s, a, lam_fbar, dtau_face, fh_d, M, lamB,
                           lamF, lam_in, dtau, nullptr, nullptr);
    else
        hipLaunchKernelGGL((adj_cellA<0, false>), gc(a.n), dim3(AL * AC), 0, s, a, lam_fbar, dtau_face, fh_d, M, lamB,
                           lamF, lam_in, dtau, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t adj_launch_seed(const AdjArgs &a, const double *fh_d, const double *dL_drho, const double *dL_du,
                           double *lam, hipStream_t s)
{
    hipLaunchKernelGGL(adj_seed, g1(a.n), dim3(256), 0, s, a, fh_d, dL_drho, dL_du, lam);
    return hipGetLastError();
}

hipError_t adj_launch_init(const AdjArgs &a, const double *f0, const double *lam, double *dL_df0, double *dtau,
                           hipStream_t s)
{
    hipLaunchKernelGGL(adj_init, g1(a.n), dim3(256), 0, s, a, f0, lam, dL_df0, dtau);
    return hipGetLastError();
}

}  // namespace dk
