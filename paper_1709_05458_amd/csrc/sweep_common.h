// Device helpers shared by the small- and large-velocity-set sweep kernels.
#pragma once
#include "dugks_internal.h"
#include "ring.h"

namespace dk {

__device__ __forceinline__ double fmaS(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaS(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ int wrapi(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// Position in the (TX+4) x (TY+4) halo tile of load slot c: the first TX*TY
// slots are the tile interior in thread order, the rest the 2-cell ring.
__device__ __forceinline__ void halo_pos(int c, int TX, int TY, int &hx, int &hy)
{
    const int HX = TX + 4;
    const int n0 = TX * TY;
    if (c < n0) {
        hx = c % TX + 2;
        hy = c / TX + 2;
        return;
    }
    int r = c - n0;
    if (r < 2 * HX) { hy = r / HX; hx = r % HX; return; }
    r -= 2 * HX;
    if (r < 2 * HX) { hy = TY + 2 + r / HX; hx = r % HX; return; }
    r -= 2 * HX;
    if (r < 2 * TY) { hx = r & 1; hy = 2 + (r >> 1); return; }
    r -= 2 * TY;
    hx = TX + 2 + (r & 1);
    hy = 2 + (r >> 1);
}

// Equilibrium of given physical moments in storage units, as coefficients of
// the quadratic polynomial in the integer lattice vector e:
//   E_q / s_q - r0 = c0 + c1x ex + c1y ey + c2xx ex^2 + c2xy ex ey + c2yy ey^2
// (s_q = w_q, r0 = 0 for FP64 storage; s_q = 1, r0 = rho0 for FP32-delta).
struct EPoly {
    double c0, c1x, c1y, c2xx, c2xy, c2yy;
};

// 1/x from the hardware estimate and two Newton steps (within an ulp of the
// rounded quotient for the positive, normal densities it is used on)
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// (iRT and clat are uniform: their products are formed once per thread)
__device__ __forceinline__ EPoly epoly(double rho, double drho, double mx, double my,
                                       double iRT, double clat, bool delta)
{
    const double ir = recip(rho);
    const double ux = mx * ir, uy = my * ir;
    const double uu = __builtin_fma(ux, ux, uy * uy);
    const double c1 = iRT * clat, h2 = 0.5 * c1 * c1;
    EPoly e;
    e.c0 = __builtin_fma(-(rho * (0.5 * iRT)), uu, delta ? drho : rho);
    e.c1x = mx * c1;
    e.c1y = my * c1;
    const double kx = (rho * h2) * ux, ky = (rho * h2) * uy;
    e.c2xx = kx * ux;
    e.c2xy = (kx + kx) * uy;
    e.c2yy = ky * uy;
    return e;
}

template <class S>
struct EPolyS {
    S c0, c1x, c1y, c2xx, c2xy, c2yy;
    __device__ __forceinline__ void set(const EPoly &e, double scale)
    {
        c0 = (S)(e.c0 * scale);
        c1x = (S)(e.c1x * scale);
        c1y = (S)(e.c1y * scale);
        c2xx = (S)(e.c2xx * scale);
        c2xy = (S)(e.c2xy * scale);
        c2yy = (S)(e.c2yy * scale);
    }
    template <int EX, int EY>
    __device__ __forceinline__ S eval() const
    {
        S v = c0;
        if (EX) v = fmaS((S)EX, c1x, v);
        if (EY) v = fmaS((S)EY, c1y, v);
        if (EX) v = fmaS((S)(EX * EX), c2xx, v);
        if (EX && EY) v = fmaS((S)(EX * EY), c2xy, v);
        if (EY) v = fmaS((S)(EY * EY), c2yy, v);
        return v;
    }
    // values at e and at -e from one even (quadratic) and one odd (linear) part
    template <int EX, int EY>
    __device__ __forceinline__ void eval_pair(S &vp, S &vm) const
    {
        S ev = c0;
        if (EX) ev = fmaS((S)(EX * EX), c2xx, ev);
        if (EX && EY) ev = fmaS((S)(EX * EY), c2xy, ev);
        if (EY) ev = fmaS((S)(EY * EY), c2yy, ev);
        if (EX && EY) {
            const S od = fmaS((S)EY, c1y, (S)EX * c1x);
            vp = ev + od;
            vm = ev - od;
        } else if (EX) {
            vp = fmaS((S)EX, c1x, ev);
            vm = fmaS((S)-EX, c1x, ev);
        } else {
            vp = fmaS((S)EY, c1y, ev);
            vm = fmaS((S)-EY, c1y, ev);
        }
    }
};

// Storage rounding of a constant update coefficient a: the kernels multiply
// the own-cell distribution by (S)a, which in FP32 scales it by 1 + O(2^-24)
// in the same direction every step, a drift that adds up over long runs.  The
// equilibrium share of that error is taken back by adding -rounding_of<S>(a)
// times the cell's equilibrium to the FP64 equilibrium terms (zero for FP64).
template <class S>
__device__ __forceinline__ double rounding_of(double a)
{
    return (double)(S)a - a;
}

// sum over the monomials e_x^a e_y^b (1 <= a + b <= 3) of the flux's
// equilibrium part; evaluated with compile-time integer e.
template <class S>
struct Cubic {
    S x, y, xx, xy, yy, xxx, xxy, xyy, yyy;
    template <int EX, int EY>
    __device__ __forceinline__ S eval() const
    {
        S v = (S)0;
        if (EX) v = fmaS((S)EX, x, v);
        if (EY) v = fmaS((S)EY, y, v);
        if (EX) v = fmaS((S)(EX * EX), xx, v);
        if (EX && EY) v = fmaS((S)(EX * EY), xy, v);
        if (EY) v = fmaS((S)(EY * EY), yy, v);
        if (EX) v = fmaS((S)(EX * EX * EX), xxx, v);
        if (EX && EY) v = fmaS((S)(EX * EX * EY), xxy, v);
        if (EX && EY) v = fmaS((S)(EX * EY * EY), xyy, v);
        if (EY) v = fmaS((S)(EY * EY * EY), yyy, v);
        return v;
    }
};

// Physical moments from storage-unit sums (a0 = sum m_q x_q, ax = sum m_q ex x_q, ...).
__device__ __forceinline__ void phys_moments(const SweepParams &p, bool delta, double a0,
                                             double ax, double ay, double &rho, double &drho,
                                             double &mx, double &my)
{
    if (delta) {
        // (fused multiply-adds written out: the same rounding in every kernel)
        drho = __builtin_fma(p.rho0, p.M0m1, a0);
        rho = p.rho0 + drho;
        mx = __builtin_fma(p.clat, ax, p.rho0 * p.M1x);
        my = __builtin_fma(p.clat, ay, p.rho0 * p.M1y);
    } else {
        rho = a0;
        drho = a0;
        mx = p.clat * ax;
        my = p.clat * ay;
    }
}

// ---------------------------------------------------------------------------
// General-path expansion about one cell (derivative form of eq. flux_DS with
// per-cell 3-point weights; one-sided next to walls, Lagrange on non-uniform
// grids).  P points at the LDS plane, (hx, hy) is the upwind cell's position
// in the halo tile and (gi, gj) its global index.
// ---------------------------------------------------------------------------
template <class S>
__device__ __forceinline__ double expand_general(const SweepParams &p, const S *P, int HX, int hx,
                                                 int hy, int gi, int gj, double dx, double dy)
{
    const int ox = p.g.sx_off[gi], oy = p.g.sy_off[gj];
    const double *d1x = p.g.sx_d1 + 3 * gi, *d2x = p.g.sx_d2 + 3 * gi;
    const double *d1y = p.g.sy_d1 + 3 * gj, *d2y = p.g.sy_d2 + 3 * gj;
    double Bx = 0, Bxx = 0, By = 0, Byy = 0, Bxy = 0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const double v = (double)P[hy * HX + hx + ox + k];
        Bx = __builtin_fma(d1x[k], v, Bx);
        Bxx = __builtin_fma(d2x[k], v, Bxx);
    }
#pragma unroll
    for (int l = 0; l < 3; l++) {
        const double v = (double)P[(hy + oy + l) * HX + hx];
        By = __builtin_fma(d1y[l], v, By);
        Byy = __builtin_fma(d2y[l], v, Byy);
    }
#pragma unroll
    for (int l = 0; l < 3; l++) {
        double row = 0;
#pragma unroll
        for (int k = 0; k < 3; k++)
            row = __builtin_fma(d1x[k], (double)P[(hy + oy + l) * HX + hx + ox + k], row);
        Bxy = __builtin_fma(d1y[l], row, Bxy);
    }
    const double B0 = (double)P[hy * HX + hx];
    const double quad = dx * dx * Bxx + 2.0 * dx * dy * Bxy + dy * dy * Byy;
    return B0 + dx * Bx + dy * By + p.kappa * quad;
}


// Workgroups are dealt to the XCDs round-robin (block b runs on XCD b % nxcd).
// Give every XCD a contiguous range of row-major tiles so that neighbouring
// tiles, which read each other's halo, share that XCD's L2.
__device__ __forceinline__ void tile_of_block(const SweepParams &p, int &tx, int &ty)
{
    const int gx = (p.nx + p.tile_x - 1) / p.tile_x;
    const int gy = (p.ny + p.tile_y - 1) / p.tile_y;
    const int nb = gx * gy;
    const int b = blockIdx.x;
    const int nx8 = p.nxcd;
    const int per = nb / nx8, rem = nb % nx8;
    const int x = b % nx8, slot = b / nx8;
    const int t = x * per + (x < rem ? x : rem) + slot;
    tx = t % gx;
    ty = t / gx;
}

__device__ __forceinline__ bool tile_is_fast(const SweepParams &p, int i0, int j0, int TX, int TY)
{
    return tile_fast(p.uniform != 0, p.perx != 0, p.pery != 0, p.nx, p.ny, i0, j0, TX, TY);
}

}  // namespace dk
