// Kernels of the scheme and reading variants, structured like the paper's
// computational sequence rather than fused: the general member a of the
// time-discretization family (section "Time discretization": A = a/2, K from
// A = (3K-2)/(6K-3), eq. EEWithP with P_n, P', P_{n+1}), the second-order
// step of Remark I, and three interface reconstructions:
//   RECON_POINT         cell values as centre values, one midpoint per face
//                       (eq. flux_DS with the coefficient kappa on the
//                       quadratic term, the library's default reading);
//   RECON_CELL_AVERAGE  cell values as cell averages (the paper's definition
//                       of f_j), the quadratic whose averages over the
//                       3-point stencils match them, and the two-point Gauss
//                       rule for the face integral of eq. microflux;
//   RECON_S2            the original DUGKS reconstruction the paper compares
//                       with: linear interpolation at the face centre minus
//                       xi h times the face gradient.
// FP64, uniform periodic grids, any velocity set.  One stage is: cell
// moments -> B = c X + (1 - c) E -> interface values at the face points,
// their moments and recovery (eq. recover2f) -> micro-flux and the stage
// combination.  Speed is not the point of this path: it runs the variants
// for the validation studies, next to the fused kernels of the default.
#include "dugks_internal.h"

namespace dk {

__device__ __forceinline__ double v_eq(const VarArgs &a, int q, double rho, double ux, double uy)
{
    const double eu = a.xi[q] * ux + a.eta[q] * uy;
    const double uu = ux * ux + uy * uy;
    return a.w[q] * rho * (1.0 + eu / a.RT + eu * eu / (2.0 * a.RT * a.RT) - uu / (2.0 * a.RT));
}

__device__ __forceinline__ double v_tau(const VarArgs &a, long long cell)
{
    return a.tau ? a.tau[cell] : a.tau0;
}

__device__ __forceinline__ int v_wrap(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// rho, u of every cell: M[0][cell] = rho, M[1] = ux, M[2] = uy
__global__ void v_moments(const VarArgs a, const double *__restrict__ X, double *__restrict__ M)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    double r = 0, mx = 0, my = 0;
    for (int q = 0; q < a.nq; q++) {
        const double v = X[q * a.n + c];
        r += v;
        mx += a.xi[q] * v;
        my += a.eta[q] * v;
    }
    M[c] = r;
    M[a.n + c] = mx / r;
    M[2 * a.n + c] = my / r;
}

// B = c X + (1 - c) E(M) with c = (p0 tau + p1) / (p2 tau + p3)
__global__ void v_mix(const VarArgs a, const double *__restrict__ X, const double *__restrict__ M,
                      double p0, double p1, double p2, double p3, double *__restrict__ B)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    const double t = v_tau(a, c);
    const double k = (p0 * t + p1) / (p2 * t + p3);
    const double r = M[c], ux = M[a.n + c], uy = M[2 * a.n + c];
    for (int q = 0; q < a.nq; q++) B[q * a.n + c] = k * X[q * a.n + c] + (1.0 - k) * v_eq(a, q, r, ux, uy);
}

// value at the offset (dx, dy) from the centre of cell (i, j) of the
// quadratic reconstructed from the 3 x 3 block of plane P around it
__device__ double v_expand(const VarArgs &a, const double *__restrict__ P, int i, int j, double dx, double dy)
{
    const int im = v_wrap(i - 1, a.nx), ip = v_wrap(i + 1, a.nx);
    const int jm = v_wrap(j - 1, a.ny), jp = v_wrap(j + 1, a.ny);
    auto at = [&](int ii, int jj) { return P[(long long)jj * a.nx + ii]; };
    const double c0 = at(i, j);
    const double Bx = (at(ip, j) - at(im, j)) / (2.0 * a.dx);
    const double By = (at(i, jp) - at(i, jm)) / (2.0 * a.dy);
    const double Bxx = (at(ip, j) - 2.0 * c0 + at(im, j)) / (a.dx * a.dx);
    const double Byy = (at(i, jp) - 2.0 * c0 + at(i, jm)) / (a.dy * a.dy);
    const double Bxy = (at(ip, jp) - at(im, jp) - at(ip, jm) + at(im, jm)) / (4.0 * a.dx * a.dy);
    double V = c0;
    if (a.recon == RECON_CELL_AVERAGE) {
        // centre value of the quadratic whose cell averages are the data: the
        // row average along x, less the y-curvature averaged over the cell
        V = (26.0 * c0 - at(ip, j) - at(im, j)) / 24.0 - a.dy * a.dy / 24.0 * Byy;
    }
    return V + dx * Bx + dy * By + a.kappa * (dx * dx * Bxx + 2.0 * dx * dy * Bxy + dy * dy * Byy);
}

// S2: face between cells (iL, jL) and (iR, jR) along axis ax (0: x, 1: y)
__device__ double v_s2(const VarArgs &a, const double *__restrict__ P, int ax, int iL, int jL, int iR, int jR,
                       double ex, double ey, double h)
{
    auto at = [&](int ii, int jj) { return P[(long long)v_wrap(jj, a.ny) * a.nx + v_wrap(ii, a.nx)]; };
    const double bL = at(iL, jL), bR = at(iR, jR);
    const double fb = 0.5 * (bL + bR);
    if (ax == 0) {
        const double gn = (bR - bL) / a.dx;
        const double gt = 0.5 * ((at(iL, jL + 1) - at(iL, jL - 1)) + (at(iR, jR + 1) - at(iR, jR - 1))) / (2.0 * a.dy);
        return fb - ex * h * gn - ey * h * gt;
    }
    const double gn = (bR - bL) / a.dy;
    const double gt = 0.5 * ((at(iL + 1, jL) - at(iL - 1, jL)) + (at(iR + 1, jR) - at(iR - 1, jR))) / (2.0 * a.dx);
    return fb - ey * h * gn - ex * h * gt;
}

// One thread per face point.  Face f of axis 0 is the x-face on the west
// side of cell f (cells f-1 | f along x, periodic); axis 1 the y-face on
// the south side.  F[q][pt][face]: first the interface values fbar of every
// velocity, then, once their moments are known, the recovered f (eq.
// recover2f) with the mean relaxation time of the two cells.
__global__ void v_faces(const VarArgs a, int ax, const double *__restrict__ B, double h, double *__restrict__ F)
{
    const int npt = a.recon == RECON_CELL_AVERAGE ? 2 : 1;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= a.n * npt) return;
    const int pt = (int)(id / a.n);
    const long long face = id % a.n;
    const int i = (int)(face % a.nx), j = (int)(face / a.nx);
    // the two cells: L = west / south, R = the cell of the face index
    const int iL = ax == 0 ? v_wrap(i - 1, a.nx) : i, jL = ax == 0 ? j : v_wrap(j - 1, a.ny);
    const int iR = i, jR = j;
    // face point relative to the centres of L (R is one cell further along ax)
    const double gp = npt == 2 ? (pt == 0 ? -1.0 : 1.0) * 0.5 / sqrt(3.0) : 0.0;
    const double nL = 0.5 * (ax == 0 ? a.dx : a.dy);   // face along the axis, from L's centre
    const double tL = gp * (ax == 0 ? a.dy : a.dx);     // along the face
    const long long stride = (long long)npt * a.n;
    double *Fp = F + (long long)pt * a.n + face;
    double r = 0, mx = 0, my = 0;
    for (int q = 0; q < a.nq; q++) {
        const double *P = B + q * a.n;
        const double ex = a.xi[q], ey = a.eta[q];
        const double en = ax == 0 ? ex : ey;
        double v;
        if (a.recon == RECON_S2) {
            v = v_s2(a, P, ax, iL, jL, iR, jR, ex, ey, h);
        } else {
            // offsets of the foot point x_b - xi h from the centre of L and of R
            const double dnL = nL - en * h, dnR = -nL - en * h;
            const double dtt = tL - (ax == 0 ? ey : ex) * h;
            auto from = [&](int ci, int cj, double dn) {
                return ax == 0 ? v_expand(a, P, ci, cj, dn, dtt) : v_expand(a, P, ci, cj, dtt, dn);
            };
            if (en > 0.0) v = from(iL, jL, dnL);
            else if (en < 0.0) v = from(iR, jR, dnR);
            else v = 0.5 * (from(iL, jL, dnL) + from(iR, jR, dnR));
        }
        Fp[q * stride] = v;
        r += v;
        mx += ex * v;
        my += ey * v;
    }
    const double ux = mx / r, uy = my / r;
    const double tb = 0.5 * (v_tau(a, (long long)jL * a.nx + iL) + v_tau(a, (long long)jR * a.nx + iR));
    for (int q = 0; q < a.nq; q++) {
        const double e = v_eq(a, q, r, ux, uy);
        Fp[q * stride] = (2.0 * tb * Fp[q * stride] + h * e) / (2.0 * tb + h);
    }
}

// Micro-flux (eq. microflux: the face mean of the recovered values) and the
// stage combination, one thread per cell:
//   mode 0 (family, stage A): L* -> Ls; out = tilde f(t') = tilde f^+ + a dt L*
//   mode 1 (family, stage C): out = fhat^+ + P' dt Omega(t') + dt (w1 L* + w2 L**)
//   mode 2 (Remark I step):   out = ((2 tau - dt) ft + 2 dt E) / (2 tau + dt) + dt L
__global__ void v_update(const VarArgs a, VarFamily fam, int mode, const double *__restrict__ Fx,
                         const double *__restrict__ Fy, const double *__restrict__ S0,
                         const double *__restrict__ M0, const double *__restrict__ G,
                         const double *__restrict__ M1, double *__restrict__ Ls, double *__restrict__ out)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    const int npt = a.recon == RECON_CELL_AVERAGE ? 2 : 1;
    const int i = (int)(c % a.nx), j = (int)(c / a.nx);
    const long long ce = (long long)j * a.nx + v_wrap(i + 1, a.nx), cn = (long long)v_wrap(j + 1, a.ny) * a.nx + i;
    const double t = v_tau(a, c), dt = fam.dt;
    const double r0 = M0[c], u0 = M0[a.n + c], w0 = M0[2 * a.n + c];
    for (int q = 0; q < a.nq; q++) {
        double fw = 0, fe = 0, fs = 0, fn = 0;
        for (int pt = 0; pt < npt; pt++) {
            const long long o = ((long long)q * npt + pt) * a.n;
            fw += Fx[o + c] / npt;
            fe += Fx[o + ce] / npt;
            fs += Fy[o + c] / npt;
            fn += Fy[o + cn] / npt;
        }
        const double L = -(a.xi[q] * a.dy * (fe - fw) + a.eta[q] * a.dx * (fn - fs)) / (a.dx * a.dy);
        const long long k = q * a.n + c;
        const double E0 = v_eq(a, q, r0, u0, w0);
        if (mode == 0) {
            const double ctp = (t - 0.5 * fam.a * dt) / (t + fam.Pn1 * dt);
            Ls[k] = L;
            out[k] = ctp * S0[k] + (1.0 - ctp) * E0 + fam.a * dt * L;
        } else if (mode == 1) {
            const double chp = (t - fam.Pn * dt) / (t + fam.Pn1 * dt);
            const double E1 = v_eq(a, q, M1[c], M1[a.n + c], M1[2 * a.n + c]);
            const double W = -2.0 * dt / (2.0 * t + fam.a * dt) * (G[k] - E1);
            out[k] = chp * S0[k] + (1.0 - chp) * E0 + fam.Pp * W + dt * (fam.w1 * Ls[k] + fam.w2 * L);
        } else {
            const double c2 = (2.0 * t - dt) / (2.0 * t + dt);
            out[k] = c2 * S0[k] + (1.0 - c2) * E0 + dt * L;
        }
        if (q == 0 && !__builtin_isfinite(out[k])) *a.bad = 1;   // non-finite flag (see dugks_sync)
    }
}

hipError_t variant_step(const VarArgs &a, const VarFamily &fam, bool t2, const double *X, double *Y,
                        const VarBuffers &b, hipStream_t s)
{
    const dim3 blk(256), gc((unsigned)((a.n + 255) / 256));
    const int npt = a.recon == RECON_CELL_AVERAGE ? 2 : 1;
    const dim3 gf((unsigned)((a.n * npt + 255) / 256));
    const double dt = fam.dt;
    hipLaunchKernelGGL(v_moments, gc, blk, 0, s, a, X, b.M0);
    if (t2) {
        // Remark I: fbar^+ over h = dt/2 from ftilde, ((4 tau - dt) ft + 3 dt E) / (4 tau + 2 dt)
        hipLaunchKernelGGL(v_mix, gc, blk, 0, s, a, X, b.M0, 4.0, -dt, 4.0, 2.0 * dt, b.B);
        hipLaunchKernelGGL(v_faces, gf, blk, 0, s, a, 0, b.B, 0.5 * dt, b.Fx);
        hipLaunchKernelGGL(v_faces, gf, blk, 0, s, a, 1, b.B, 0.5 * dt, b.Fy);
        hipLaunchKernelGGL(v_update, gc, blk, 0, s, a, fam, 2, b.Fx, b.Fy, X, b.M0, nullptr, nullptr, nullptr, Y);
        return hipGetLastError();
    }
    // step (1): fbar^{+,h1} = f + (h1/2) Omega from fhat, h1 = A dt
    const double h1 = fam.A * dt, h2 = (fam.K - fam.a) * dt;
    hipLaunchKernelGGL(v_mix, gc, blk, 0, s, a, X, b.M0, 1.0, -0.5 * h1, 1.0, fam.Pn1 * dt, b.B);
    hipLaunchKernelGGL(v_faces, gf, blk, 0, s, a, 0, b.B, h1, b.Fx);
    hipLaunchKernelGGL(v_faces, gf, blk, 0, s, a, 1, b.B, h1, b.Fy);
    // step (2): the T2 sub-step of a dt to t'
    hipLaunchKernelGGL(v_update, gc, blk, 0, s, a, fam, 0, b.Fx, b.Fy, X, b.M0, nullptr, nullptr, b.Ls, b.G);
    // step (3): fbar^{+,h2} = f + (h2/2) Omega at t' from tilde f, h2 = (K - a) dt
    hipLaunchKernelGGL(v_moments, gc, blk, 0, s, a, (const double *)b.G, b.M1);
    hipLaunchKernelGGL(v_mix, gc, blk, 0, s, a, (const double *)b.G, b.M1, 2.0, -h2, 2.0, fam.a * dt, b.B);
    hipLaunchKernelGGL(v_faces, gf, blk, 0, s, a, 0, b.B, h2, b.Fx);
    hipLaunchKernelGGL(v_faces, gf, blk, 0, s, a, 1, b.B, h2, b.Fy);
    // step (4): eq. EEWithP
    hipLaunchKernelGGL(v_update, gc, blk, 0, s, a, fam, 1, b.Fx, b.Fy, X, b.M0, (const double *)b.G, b.M1, b.Ls,
                       Y);
    return hipGetLastError();
}

}  // namespace dk
