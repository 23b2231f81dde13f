// Discrete adjoint of one T3S3-DUGKS step (periodic, uniform grid, any
// velocity set), in double.  For a step out = F(fhat; tau) the kernels map
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
// Every cell (or face) kernel runs a block of four waves over 64 cells: wave
// s takes the velocities q = s, s + 4, ... (the same in every lane, so the
// per-velocity weights are scalar loads), and sums over all velocities
// (moments, the adjoint of the equilibrium) are combined across the four
// waves through LDS in a fixed order.  At 256^2 cells that is four waves per
// SIMD instead of one.
#include "sweep_common.h"

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

// ---------------------------------------------------------------------------
// Primal intermediates of one step from fhat (storage units) and G (stage A
// output): B, moments of fhat, B' and moments of G, all in double.
// ---------------------------------------------------------------------------
template <class S, bool DELTA>
__global__ void adj_prep(const AdjArgs a, double rho0, const S *__restrict__ fhat, const S *__restrict__ G,
                         double *__restrict__ fh_d, double *__restrict__ B, double *__restrict__ M,
                         double *__restrict__ G_d, double *__restrict__ B2, double *__restrict__ M2)
{
    const Lane L = lane_of(a.n);
    const long long c = L.c;
    const double tau = a.tau[c], dt = a.dt;
    const double c1 = (12.0 * tau - dt) / (12.0 * tau + 3.0 * dt);
    const double c3 = (24.0 * tau - 5.0 * dt) / (24.0 * tau + 4.0 * dt);
    for (int pass = 0; pass < 2; pass++) {
        const S *src = pass ? G : fhat;
        double *dst = pass ? G_d : fh_d;
        auto val = [&](int q) {
            return DELTA ? a.w[q] * ((double)src[q * a.n + c] + rho0) : (double)src[q * a.n + c];
        };
        double r = 0, mx = 0, my = 0;
        for (int q = L.s; q < a.nq; q += AL) {
            const double v = val(q);
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
            if (L.ok) Bo[q * a.n + c] = cc * val(q) + (1.0 - cc) * eq_val(a, q, r, ux, uy);
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
// Cell adjoint of stage C: from lambda_out and the stage C face adjoint to
// lambda of L* (lamLs), the partial adjoints of B (lamB) and fhat (lamF).
// ---------------------------------------------------------------------------
template <int QC>
__global__ void __launch_bounds__(AL * AC) adj_cellC(const AdjArgs a, const double *__restrict__ lam_out, const double *__restrict__ lam_fbar,
                          const double *__restrict__ dtau_face, const double *__restrict__ G_d,
                          const double *__restrict__ M2, double *__restrict__ lamLs, double *__restrict__ lamB,
                          double *__restrict__ lamF, double *__restrict__ dtau)
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
    double gR = 0, gX = 0, gY = 0, dtc = L.s == 0 ? faces_tau(a, dtau_face, i, j) : 0.0;
    // lam_G (partial) into lamLs as scratch
    const int nq = QC > 0 ? QC : a.nq;
#pragma unroll
    for (int k = 0; k < (QC > 0 ? (QC + AL - 1) / AL : (nq + AL - 1) / AL); k++) {
        const int q = L.s + AL * k;
        if (q >= nq) break;
        const double lB2 = gather_B(a, a.cC, lam_fbar, i, j, q);
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
template <int QC>
__global__ void __launch_bounds__(AL * AC) adj_cellA(const AdjArgs a, const double *__restrict__ lam_fbar, const double *__restrict__ dtau_face,
                          const double *__restrict__ fh_d, const double *__restrict__ M,
                          const double *__restrict__ lamB, const double *__restrict__ lamF,
                          double *__restrict__ lam_in, double *__restrict__ dtau)
{
    const Lane L = lane_of(a.n);
    const long long c = L.c;
    const int i = (int)(c % a.nx), j = (int)(c / a.nx);
    const double tau = a.tau[c], dt = a.dt;
    const double c1 = (12.0 * tau - dt) / (12.0 * tau + 3.0 * dt);
    const double dc1 = 48.0 * dt / ((12.0 * tau + 3.0 * dt) * (12.0 * tau + 3.0 * dt));
    const double r = M[3 * c], ux = M[3 * c + 1] / r, uy = M[3 * c + 2] / r;
    double gR = 0, gX = 0, gY = 0, dtc = L.s == 0 ? faces_tau(a, dtau_face, i, j) : 0.0;
    const int nq = QC > 0 ? QC : a.nq;
#pragma unroll
    for (int k = 0; k < (QC > 0 ? (QC + AL - 1) / AL : (nq + AL - 1) / AL); k++) {
        const int q = L.s + AL * k;
        if (q >= nq) break;
        const double lB = lamB[q * a.n + c] + gather_B(a, a.cA, lam_fbar, i, j, q);
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
    if (delta)
        hipLaunchKernelGGL((adj_prep<float, true>), gc(a.n), dim3(AL * AC), 0, s, a, rho0, (const float *)fhat,
                           (const float *)G, fh_d, B, M, G_d, B2, M2);
    else
        hipLaunchKernelGGL((adj_prep<double, false>), gc(a.n), dim3(AL * AC), 0, s, a, rho0, (const double *)fhat,
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
                           double *lamF, double *dtau, hipStream_t s)
{
    // stage C (reverse of steps (3)-(4)); the cell adjoints with the velocity
    // count fixed at compile time for D2Q9 (their gathers are issued together)
    launch_adj_face(a, 1, B2, lam_out, 4.0 * a.dt / 7.0, lam_fbar, dtau_face, s);
    if (a.nq == 9)
        hipLaunchKernelGGL(adj_cellC<9>, gc(a.n), dim3(AL * AC), 0, s, a, lam_out, lam_fbar, dtau_face, G_d, M2,
                           lamLs, lamB, lamF, dtau);
    else
        hipLaunchKernelGGL(adj_cellC<0>, gc(a.n), dim3(AL * AC), 0, s, a, lam_out, lam_fbar, dtau_face, G_d, M2,
                           lamLs, lamB, lamF, dtau);
    // stage A (reverse of steps (1)-(2))
    launch_adj_face(a, 0, B, lamLs, 1.0, lam_fbar, dtau_face, s);
    if (a.nq == 9)
        hipLaunchKernelGGL(adj_cellA<9>, gc(a.n), dim3(AL * AC), 0, s, a, lam_fbar, dtau_face, fh_d, M, lamB, lamF,
                           lam_in, dtau);
    else
        hipLaunchKernelGGL(adj_cellA<0>, gc(a.n), dim3(AL * AC), 0, s, a, lam_fbar, dtau_face, fh_d, M, lamB, lamF,
                           lam_in, dtau);
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
