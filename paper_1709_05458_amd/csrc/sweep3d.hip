// Three-dimensional T3S3-DUGKS sweep (include/dugks3d.h) on a triply periodic
// box of uniform cells, for gfx950.
//
// One step is two kernels, one per stage; each runs a block of 256 threads
// (four waves) over a tile of 16 x 8 x 2 cells, one cell per thread (rows
// of 16 cells: a wave's own-cell loads and stores cover whole 64-byte
// segments):
//   - the loop over velocities is outermost: the stage's transformed state
//     B_q (fbar^{+,h} of eqs. f_bar_1_6 / fbp_5_12, kept in HBM) of the tile
//     and a halo of two cells is staged in LDS, double-buffered, one barrier
//     per velocity;
//   - every thread forms the six face values of its cell for that velocity
//     from LDS (eqs. interfaceEvof and flux_DS: fixed window weights per
//     axis and velocity, built on the host), adds them into the FP64 moments
//     of each face, and adds the part of the micro-flux that needs no face
//     moments, alpha fbar (eq. recover2f split into alpha fbar + beta E).
//     k3_stage_lat (the library's D3Q19 / D3Q27) knows every window's shape
//     at compile time and reads LDS at immediate offsets; k3_stage (any
//     other order of 19 or 27 velocities) reads offsets and weights from
//     tables;
//   - after the last velocity the face equilibria give the beta E part, and
//     the epilogue applies the stage's update to the thread's cell, sums the
//     output's cell moments (FP64) and writes the next stage's transformed
//     state B, so no kernel re-reads a whole state to form moments:
//       stage A: G = 5/4 B_A - 1/4 fhat + dt/3 L*,  B_C = c3 G + (1-c3) E(G);
//       stage C: fhat' = 4/7 fhat - 6/7 B_A + 9/7 G + 3/4 W + 4dt/7 L**,
//                B_A' = c1 fhat' + (1-c1) E(fhat')
//     (the stage C form is eq. feqIntD3rdHat2_DS with L* taken back out of
//     G = 5/4 B_A - 1/4 fhat + dt/3 L*, W = -6dt/(6 tau + dt) (G - E(G)),
//     eq. collisionterm).
// FP32-delta storage keeps g = f / w - rho0; the window sums and the update
// are FP32 on g, the moments FP64.  The affine maps on g are written so that
// their rounded FP32 coefficients act on differences only (X + k (E - X),
// f + 9/7 (G - f) - 6/7 (B_A - f)): g carries rho0 implicitly, and
// coefficients that do not sum to one in FP32 would change the mass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dugks3d.h"
#include "dugks_internal.h"

namespace dk3 {

constexpr int TX = 16, TY = 8, TZ = 2, HALO = 2;
constexpr int LX = TX + 2 * HALO, LY = TY + 2 * HALO, LZ = TZ + 2 * HALO;
constexpr int NSLOT = LX * LY * LZ;           // 1152 LDS slots per velocity
constexpr int NT = TX * TY * TZ;              // 256 threads
constexpr int SPT = (NSLOT + NT - 1) / NT;    // slots filled per thread
constexpr int MAXW = 36;                      // window entries per (axis, velocity): a 4 x 3 x 3 box

struct Args {
    int nx, ny, nz;
    int ntx, nty, ntiles;
    long long n;
    double dt, rho0, iRT;
    double inv_d[3];    // 1 / cell width per axis
    double h[2];        // reconstruction time of stage A (dt/6) and C (5dt/12)
    const double *xi;   // [3][Q]
    const double *w;    // [Q]
    const double *tau;  // [n]
    const int *wcnt;    // [2][3][Q] entries of each window
    const int *woff;    // [2][3][Q][MAXW] LDS offset of each entry from the cell's own slot
    const double *wd;   // [2][3][Q][MAXW] weights
    const float *wf;
    double cs;          // lattice kernels: xi = cs e_q
};

// Periodic image of v along an axis of n >= 3 cells.  Every coordinate a
// cell inside the box reads lies in [-2, n + 1] (a halo of two), where one
// add or subtract is exact; slots further out (past the last cell of a
// ragged tile) only feed cells outside the box and are clamped in range.
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? min(v - n, n - 1) : v); }

// Tile coordinates of a tile's place in the launch order: x fastest, then y
// within a band of up to YB tile rows, then z, then the bands.  Tiles that
// share a halo along y or z then run close together in time (and on one
// XCD), so the shared planes are still in its L2.
constexpr int YB = 2;
__device__ __forceinline__ void tile_coords(const Args &a, int tile, int &ti, int &tj, int &tk)
{
    const int ntz = a.ntiles / (a.ntx * a.nty);
    const int per_band = a.ntx * ntz * YB;   // tiles of a full band
    const int b = tile / per_band;
    const int r = tile - b * per_band;
    const int hb = min(YB, a.nty - b * YB);   // rows of this band
    ti = r % a.ntx;
    const int s = r / a.ntx;
    tj = b * YB + s % hb;
    tk = s / hb;
}

__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class T>
__device__ __forceinline__ const T *weights(const Args &a);
template <>
__device__ __forceinline__ const float *weights<float>(const Args &a) { return a.wf; }
template <>
__device__ __forceinline__ const double *weights<double>(const Args &a) { return a.wd; }

// Equilibrium of one velocity (components xq, weight wq) in storage units:
// g-form (DELTA: E / w - rho0) or f-form.  r: density, dr = r - rho0, u:
// velocity, uu2 = |u|^2 / (2 RT).
template <class T, bool DELTA>
__device__ __forceinline__ T eq_store(const T xq[3], T wq, T iRT, T r, T dr, const T u[3], T uu2)
{
    const T eu = xq[0] * u[0] + xq[1] * u[1] + xq[2] * u[2];
    const T P = eu * iRT * ((T)1 + (T)0.5 * eu * iRT) - uu2;
    if (DELTA) return dr + r * P;
    return wq * r * ((T)1 + P);
}

// the same from the global velocity table (per-cell kernels)
template <class T, bool DELTA>
__device__ __forceinline__ T eq_tab(const Args &a, int q, int Q, T r, T dr, const T u[3], T uu2)
{
    const T xq[3] = {(T)a.xi[q], (T)a.xi[Q + q], (T)a.xi[2 * Q + q]};
    return eq_store<T, DELTA>(xq, (T)a.w[q], (T)a.iRT, r, dr, u, uu2);
}

// density and velocity from FP64 sums of the storage values: rho = R0 + s0,
// rho u = s (the weights are folded into the sums for DELTA)
__device__ __forceinline__ void moments_of(const Args &a, bool delta, const double s[4], double &rho, double u[3])
{
    rho = (delta ? a.rho0 : 0.0) + s[0];
    const double ir = 1.0 / rho;
    u[0] = s[1] * ir;
    u[1] = s[2] * ir;
    u[2] = s[3] * ir;
}

// ---------------------------------------------------------------------------
// One stage over one tile.  STAGE 0: Bin = B_A; writes G (out1), B_C (out2)
// and the moments of G (Mout).  STAGE 1: Bin = B_C; reads fhat, B_A, G and
// the moments of G; writes fhat' over fhat (out1), B_A' over B_A (out2) and
// the moments of fhat' (Mout).  Every thread reads and writes only its own
// cell of those arrays, so the in-place update is safe.
// ---------------------------------------------------------------------------
template <class S, bool DELTA, int Q, int STAGE>
__global__ void __launch_bounds__(NT) k3_stage(const Args a, const S *__restrict__ Bin, const S *fh, const S *Ba,
                                              const S *__restrict__ G, const double *__restrict__ M1, S *out1,
                                              S *out2, double *__restrict__ Mout)
{
    using T = S;
    __shared__ S lds[2][NSLOT];
    // per velocity: xi (3), w, the moment weight (w for DELTA, else 1) and
    // xi / width (3); read from LDS where used, so that the unrolled loops
    // over velocities do not hold the whole table in scalar registers
    __shared__ double vt[Q][8];
    // XCD-aware order: the blocks one XCD runs (b mod 8) take consecutive tiles
    const int nb8 = (a.ntiles + 7) / 8;
    const int tile = (blockIdx.x % 8) * nb8 + blockIdx.x / 8;
    if (tile >= a.ntiles) return;
    int ti, tj, tk;
    tile_coords(a, tile, ti, tj, tk);
    const int t = threadIdx.x;
    if (t < Q) {
        for (int d = 0; d < 3; d++) {
            vt[t][d] = a.xi[d * Q + t];
            vt[t][5 + d] = a.xi[d * Q + t] * a.inv_d[d];
        }
        vt[t][3] = a.w[t];
        vt[t][4] = DELTA ? a.w[t] : 1.0;
    }
    const int lx = t % TX, ly = (t / TX) % TY, lz = t / (TX * TY);
    const int i = ti * TX + lx, j = tj * TY + ly, k = tk * TZ + lz;
    const bool ok = i < a.nx && j < a.ny && k < a.nz;
    const long long n = a.n;
    const long long c = ((long long)min(k, a.nz - 1) * a.ny + min(j, a.ny - 1)) * a.nx + min(i, a.nx - 1);

    // global cell of each LDS slot this thread fills (periodic images)
    long long gidx[SPT];
#pragma unroll
    for (int r = 0; r < SPT; r++) {
        const int s = t + r * NT;
        gidx[r] = 0;
        if (s < NSLOT) {
            const int sx = s % LX, sy = (s / LX) % LY, sz = s / (LX * LY);
            const int gx = wrap1(ti * TX + sx - HALO, a.nx), gy = wrap1(tj * TY + sy - HALO, a.ny),
                      gz = wrap1(tk * TZ + sz - HALO, a.nz);
            gidx[r] = ((long long)gz * a.ny + gy) * a.nx + gx;
        }
    }
    // the slots of one velocity: loaded into registers, then stored to LDS
    S nxt[SPT];
    auto load = [&](int q) {
#pragma unroll
        for (int r = 0; r < SPT; r++)
            if (r * NT + NT <= NSLOT || t + r * NT < NSLOT) nxt[r] = Bin[(long long)q * n + gidx[r]];
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < SPT; r++)
            if (r * NT + NT <= NSLOT || t + r * NT < NSLOT) lds[buf][t + r * NT] = nxt[r];
    };

    // interface recovery weights of the six faces (eq. recover2f with the
    // mean relaxation time of the two cells, R7): [axis][low, high]
    const int ci = min(i, a.nx - 1), cj = min(j, a.ny - 1), ck = min(k, a.nz - 1);
    const double tau_c = a.tau[c];
    const double h = a.h[STAGE];
    T al[3][2], be[3][2];
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
#pragma unroll
        for (int sd = 0; sd < 2; sd++) {
            const int o = sd ? 1 : -1;
            const int ni = ax == 0 ? wrap1(ci + o, a.nx) : ci, nj = ax == 1 ? wrap1(cj + o, a.ny) : cj,
                      nk = ax == 2 ? wrap1(ck + o, a.nz) : ck;
            const double tb = 0.5 * (tau_c + a.tau[((long long)nk * a.ny + nj) * a.nx + ni]);
            const double rd = 1.0 / (2.0 * tb + h);
            al[ax][sd] = (T)(2.0 * tb * rd);
            be[ax][sd] = (T)(h * rd);
        }
    }

    const int own = ((lz + HALO) * LY + (ly + HALO)) * LX + (lx + HALO);
    constexpr int PITCH[3] = {1, LX, LX * LY};
    const T *wt = weights<T>(a);
    double mf[3][2][4];   // FP64 sums of each face: [axis][low, high][storage sum, 3 momenta]
#pragma unroll
    for (int ax = 0; ax < 3; ax++)
#pragma unroll
        for (int sd = 0; sd < 2; sd++)
#pragma unroll
            for (int m = 0; m < 4; m++) mf[ax][sd][m] = 0.0;
    // per thread and velocity, in LDS: the own-cell part of the stage output
    // minus the alpha part of the micro-flux, then the output itself
    __shared__ T X[Q][NT];
    const double dt = a.dt;
    const T iRT = (T)a.iRT;
    // stage C: the equilibrium of G (its moments from stage A) and kw (eq.
    // collisionterm)
    T r1t = 0, dr1 = 0, u1[3] = {0, 0, 0}, uu1 = 0, kw = 0;
    if (STAGE == 1) {
        const double r1 = M1[c], u1d[3] = {M1[n + c], M1[2 * n + c], M1[3 * n + c]};
        r1t = (T)r1;
        dr1 = (T)(r1 - (DELTA ? a.rho0 : 0.0));
        for (int d = 0; d < 3; d++) u1[d] = (T)u1d[d];
        uu1 = (T)(0.5 * (u1d[0] * u1d[0] + u1d[1] * u1d[1] + u1d[2] * u1d[2]) * a.iRT);
        kw = (T)(6.0 * dt / (6.0 * tau_c + dt));
    }
    // weight of L in the output: dt/3 (stage A), 4 dt/7 (stage C)
    const T wl = (T)(STAGE == 0 ? dt / 3.0 : 4.0 * dt / 7.0);

    load(0);
    store(0);
    __syncthreads();
#pragma unroll 1
    for (int q = 0; q < Q; q++) {
        if (q + 1 < Q) load(q + 1);
        // own-cell inputs of the output (their loads overlap the faces)
        const T f = fh[(long long)q * n + c];
        T b = 0, g = 0;
        if (STAGE == 1) {
            b = Ba[(long long)q * n + c];
            g = G[(long long)q * n + c];
        }
        const S *B = lds[q & 1];
        const double om = vt[q][4];
        const double omx[3] = {om * vt[q][0], om * vt[q][1], om * vt[q][2]};
        T acc = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            const int tb = (STAGE * 3 + ax) * Q + q;
            const int cnt = a.wcnt[tb];
            const int *off = a.woff + tb * MAXW;
            const T *wq = wt + tb * MAXW;
            T vlo = 0, vhi = 0;
            for (int m = 0; m < cnt; m++) {
                const int o = own + off[m];
                vlo = fmat(wq[m], B[o], vlo);
                vhi = fmat(wq[m], B[o + PITCH[ax]], vhi);
            }
            const double dlo = (double)vlo, dhi = (double)vhi;
            mf[ax][0][0] += om * dlo;
            mf[ax][1][0] += om * dhi;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                mf[ax][0][d + 1] = __builtin_fma(omx[d], dlo, mf[ax][0][d + 1]);
                mf[ax][1][d + 1] = __builtin_fma(omx[d], dhi, mf[ax][1][d + 1]);
            }
            acc += (T)vt[q][5 + ax] * (al[ax][1] * vhi - al[ax][0] * vlo);
        }
        T own_part;
        if (STAGE == 0) {
            own_part = (T)1.25 * B[own] - (T)0.25 * f;
        } else {
            const T xq[3] = {(T)vt[q][0], (T)vt[q][1], (T)vt[q][2]};
            const T W = -kw * (g - eq_store<T, DELTA>(xq, (T)vt[q][3], iRT, r1t, dr1, u1, uu1));
            // 4/7 f - 6/7 B_A + 9/7 G as f + 9/7 (G - f) - 6/7 (B_A - f): the
            // rounded coefficients then act on differences only, so the
            // constant (rho0) part of the stored deviations is kept exactly
            own_part = f + (T)(9.0 / 7.0) * (g - f) - (T)(6.0 / 7.0) * (b - f) + (T)0.75 * W;
        }
        X[q][t] = own_part - wl * acc;
        if (q + 1 < Q) store((q + 1) & 1);
        __syncthreads();
    }

    // face equilibria: the beta E part of the micro-flux (L = -(alpha part +
    // beta part)), the output and its moments
    T fr[3][2], fdr[3][2], fu[3][2][3], fuu[3][2];
#pragma unroll
    for (int ax = 0; ax < 3; ax++)
#pragma unroll
        for (int sd = 0; sd < 2; sd++) {
            double rho, u[3];
            moments_of(a, DELTA, mf[ax][sd], rho, u);
            fr[ax][sd] = (T)rho;
            fdr[ax][sd] = (T)(rho - (DELTA ? a.rho0 : 0.0));
            for (int d = 0; d < 3; d++) fu[ax][sd][d] = (T)u[d];
            fuu[ax][sd] = (T)(0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * a.iRT);
        }
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int q = 0; q < Q; q++) {
        const T xq[3] = {(T)vt[q][0], (T)vt[q][1], (T)vt[q][2]}, wq = (T)vt[q][3];
        T lb = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            const T ehi = eq_store<T, DELTA>(xq, wq, iRT, fr[ax][1], fdr[ax][1], fu[ax][1], fuu[ax][1]);
            const T elo = eq_store<T, DELTA>(xq, wq, iRT, fr[ax][0], fdr[ax][0], fu[ax][0], fuu[ax][0]);
            lb += (T)vt[q][5 + ax] * (be[ax][1] * ehi - be[ax][0] * elo);
        }
        const T o = X[q][t] - wl * lb;
        X[q][t] = o;
        const double om = vt[q][4], v = (double)o;
        s4[0] += om * v;
        s4[1] = __builtin_fma(om * vt[q][0], v, s4[1]);
        s4[2] = __builtin_fma(om * vt[q][1], v, s4[2]);
        s4[3] = __builtin_fma(om * vt[q][2], v, s4[3]);
    }
    double rho, u[3];
    moments_of(a, DELTA, s4, rho, u);
    if (!ok) return;
    const double cc = STAGE == 0 ? (24.0 * tau_c - 5.0 * dt) / (24.0 * tau_c + 4.0 * dt)
                                 : (12.0 * tau_c - dt) / (12.0 * tau_c + 3.0 * dt);
    // B = c X + (1 - c) E as X + (1 - c) (E - X), exact for X = E
    const T cet = (T)(1.0 - cc);
    const T rt = (T)rho, drt = (T)(rho - (DELTA ? a.rho0 : 0.0));
    const T ut[3] = {(T)u[0], (T)u[1], (T)u[2]};
    const T uu = (T)(0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * a.iRT);
#pragma unroll 1
    for (int q = 0; q < Q; q++) {
        const T o = X[q][t];
        const T xq[3] = {(T)vt[q][0], (T)vt[q][1], (T)vt[q][2]};
        out1[(long long)q * n + c] = o;
        out2[(long long)q * n + c] = o + cet * (eq_store<T, DELTA>(xq, (T)vt[q][3], iRT, rt, drt, ut, uu) - o);
    }
    Mout[c] = rho;
    Mout[n + c] = u[0];
    Mout[2 * n + c] = u[1];
    Mout[3 * n + c] = u[2];
}

// ---------------------------------------------------------------------------
// The same stage for the library's lattices (D3Q27: xi = c e with
// e = (ix - 1, iy - 1, iz - 1), q = 9 ix + 3 iy + iz; D3Q19: the same order
// without the eight corners).  The sign pattern of every velocity is known
// at compile time, hence so is which cells of the 4 x 3 x 3 window of each
// face carry a weight: the window sums read LDS at immediate offsets (no
// address arithmetic), skip the empty entries, and the weights of the stage
// (only the non-empty entries) sit in LDS.  LDS rows are padded to 48
// slots, which puts the two 16-cell rows of each half-wave on distinct banks.
// ---------------------------------------------------------------------------
struct E3 {
    int c[3];
};
template <int LAT>
__host__ __device__ constexpr E3 lat_e(int q)
{
    int k = 0;
    for (int p = 0; p < 27; p++) {
        const E3 e{{p / 9 - 1, (p / 3) % 3 - 1, p % 3 - 1}};
        if (LAT == 19 && e.c[0] != 0 && e.c[1] != 0 && e.c[2] != 0) continue;
        if (k == q) return e;
        k++;
    }
    return E3{{0, 0, 0}};
}
// the lattice's weights: products of (1/6, 2/3, 1/6) per axis (D3Q27);
// 1/3, 1/18, 1/36 for zero, one and two nonzero components (D3Q19)
template <int LAT>
__host__ __device__ constexpr double lat_w(int q)
{
    const E3 e = lat_e<LAT>(q);
    int nz = 0;
    double w = 1.0;
    for (int a = 0; a < 3; a++) {
        nz += e.c[a] != 0;
        w *= e.c[a] != 0 ? 1.0 / 6.0 : 2.0 / 3.0;
    }
    if (LAT == 19) return nz == 0 ? 1.0 / 3.0 : (nz == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    return w;
}

// window entry m of the low face along axis ax: offset oa in -2..1 along ax,
// ob and oc in -1..1 along the other two axes (in increasing axis order)
__host__ __device__ constexpr void win_offset(int ax, int m, int o[3])
{
    const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
    o[0] = o[1] = o[2] = 0;
    o[ax] = m / 9 - 2;
    o[t1] = (m / 3) % 3 - 1;
    o[t2] = m % 3 - 1;
}
// does the expansion of eq. flux_DS put a weight on window entry m?  About
// the upwind cell U (U = -1 or 0 along ax; both when xi is parallel to the
// face) the displacement is nonzero along ax and along every axis where xi
// is; the expansion touches U, U +- e_a where the displacement along a is
// nonzero, and U + e_a +- e_b where both are.
__host__ __device__ constexpr bool in_window(const E3 e, int ax, int m)
{
    int o[3] = {0, 0, 0};
    win_offset(ax, m, o);
    bool nz[3] = {false, false, false};
    for (int a = 0; a < 3; a++) nz[a] = a == ax || e.c[a] != 0;
    for (int U = -1; U <= 0; U++) {
        if ((e.c[ax] > 0 && U != -1) || (e.c[ax] < 0 && U != 0)) continue;
        int cnt = 0;
        bool ok = true;
        for (int a = 0; a < 3; a++) {
            const int p = o[a] - (a == ax ? U : 0);
            if (p < -1 || p > 1) ok = false;
            if (p != 0) {
                cnt++;
                if (!nz[a]) ok = false;
            }
        }
        if (ok && cnt <= 2) return true;
    }
    return false;
}
// position of every non-empty entry in the compact weight list of a stage
template <int LAT>
struct WinTable {
    short idx[3][LAT][36];
    int total;
};
template <int LAT>
__host__ __device__ constexpr WinTable<LAT> make_win()
{
    WinTable<LAT> w{};
    int k = 0;
    for (int ax = 0; ax < 3; ax++)
        for (int q = 0; q < LAT; q++)
            for (int m = 0; m < 36; m++) {
                w.idx[ax][q][m] = -1;
                if (in_window(lat_e<LAT>(q), ax, m)) w.idx[ax][q][m] = (short)k++;
            }
    w.total = k;
    return w;
}
template <int LAT>
inline constexpr WinTable<LAT> kWin = make_win<LAT>();

template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    [&]<int... I>(std::integer_sequence<int, I...>) {
        (f(std::integral_constant<int, I>{}), ...);
    }(std::make_integer_sequence<int, N>{});
}

constexpr int LXP = 48;   // padded row of the lattice kernels' LDS tile
constexpr int LSZ = LZ * LY * LXP;

// The velocity-dependent part of the equilibrium of lattice velocity e,
// P = xi.u/RT + (xi.u)^2/(2 RT^2) - |u|^2/(2 RT), from cv = cs u / RT and
// uu2 = |u|^2/(2 RT); the products with the components of e (0 or +-1)
// fold at compile time
template <class T, int LAT, int q>
__device__ __forceinline__ T p_lat(const T cv[3], T uu2)
{
    constexpr E3 e = lat_e<LAT>(q);
    T eu = 0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (e.c[d] > 0) eu += cv[d];
        if (e.c[d] < 0) eu -= cv[d];
    }
    return eu * ((T)1 + (T)0.5 * eu) - uu2;
}
// equilibrium of lattice velocity e in storage units (as eq_store)
template <class T, bool DELTA, int LAT, int q>
__device__ __forceinline__ T eq_lat(const T cv[3], T r, T dr, T uu2)
{
    const T P = p_lat<T, LAT, q>(cv, uu2);
    if (DELTA) return dr + r * P;
    return (T)lat_w<LAT>(q) * r * ((T)1 + P);
}

// FP64: at least two waves per SIMD (at 27 velocities stage C would take
// 260 registers, one wave).  FP32 D3Q27 stage C: three (174 registers would
// give two; at 168 a few values spill, and the stage runs 9% faster)
template <class S, bool DELTA, int LAT, int STAGE>
__global__ void __launch_bounds__(NT)
    __attribute__((amdgpu_waves_per_eu(DELTA ? (LAT == 27 && STAGE == 1 ? 3 : 1) : 2, 8))) k3_stage_lat(const Args a, const S *__restrict__ Bin, const S *fh,
                                                  const S *Ba, const S *__restrict__ G,
                                                  const double *__restrict__ M1, S *out1, S *out2,
                                                  double *__restrict__ Mout, const S *__restrict__ wcompact)
{
    using T = S;
    constexpr int Q = LAT;
    constexpr int NW = kWin<LAT>.total;
    __shared__ S lds[2][LSZ];
    // the weights in 16-byte chunks: a wave reads four (FP64: two) uniform
    // weights per LDS instruction, at immediate offsets from one base
    constexpr int VW = 16 / (int)sizeof(T);
    using V = T __attribute__((ext_vector_type(VW)));
    __shared__ V wsh[(NW + VW - 1) / VW];
    const int nb8 = (a.ntiles + 7) / 8;
    const int tile = (blockIdx.x % 8) * nb8 + blockIdx.x / 8;
    if (tile >= a.ntiles) return;
    int ti, tj, tk;
    tile_coords(a, tile, ti, tj, tk);
    const int t = threadIdx.x;
    for (int k = t; k < NW; k += NT) wsh[k / VW][k % VW] = wcompact[STAGE * NW + k];
    const int lx = t % TX, ly = (t / TX) % TY, lz = t / (TX * TY);
    const int i = ti * TX + lx, j = tj * TY + ly, k = tk * TZ + lz;
    const bool ok = i < a.nx && j < a.ny && k < a.nz;
    const long long n = a.n;
    const int ci = min(i, a.nx - 1), cj = min(j, a.ny - 1), ck = min(k, a.nz - 1);
    const long long c = ((long long)ck * a.ny + cj) * a.nx + ci;

    long long gidx[SPT];
    int lidx[SPT];
#pragma unroll
    for (int r = 0; r < SPT; r++) {
        const int s = t + r * NT;
        gidx[r] = 0;
        lidx[r] = 0;
        if (s < NSLOT) {
            const int sx = s % LX, sy = (s / LX) % LY, sz = s / (LX * LY);
            const int gx = wrap1(ti * TX + sx - HALO, a.nx), gy = wrap1(tj * TY + sy - HALO, a.ny),
                      gz = wrap1(tk * TZ + sz - HALO, a.nz);
            gidx[r] = ((long long)gz * a.ny + gy) * a.nx + gx;
            lidx[r] = (sz * LY + sy) * LXP + sx;
        }
    }
    S nxt[SPT];
    auto load = [&](int q) {
#pragma unroll
        for (int r = 0; r < SPT; r++)
            if (r * NT + NT <= NSLOT || t + r * NT < NSLOT) nxt[r] = Bin[(long long)q * n + gidx[r]];
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < SPT; r++)
            if (r * NT + NT <= NSLOT || t + r * NT < NSLOT) lds[buf][lidx[r]] = nxt[r];
    };

    const double tau_c = a.tau[c];
    const double h = a.h[STAGE];
    // alpha of each face; beta = 1 - alpha is formed after the loop (fewer
    // registers held through it)
    T al[3][2];
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
#pragma unroll
        for (int sd = 0; sd < 2; sd++) {
            const int o = sd ? 1 : -1;
            const int ni = ax == 0 ? wrap1(ci + o, a.nx) : ci, nj = ax == 1 ? wrap1(cj + o, a.ny) : cj,
                      nk = ax == 2 ? wrap1(ck + o, a.nz) : ck;
            const double tb = 0.5 * (tau_c + a.tau[((long long)nk * a.ny + nj) * a.nx + ni]);
            al[ax][sd] = (T)(2.0 * tb / (2.0 * tb + h));
        }
    }
    // base of the cell's window: every offset below is then non-negative
    constexpr int PITCH[3] = {1, LXP, LXP * LY};
    constexpr int BIAS = 2 * PITCH[2] + 2 * PITCH[1] + 2 * PITCH[0];
    const int own = ((lz + HALO) * LY + (ly + HALO)) * LXP + (lx + HALO);
    double mf[3][2][4];
#pragma unroll
    for (int ax = 0; ax < 3; ax++)
#pragma unroll
        for (int sd = 0; sd < 2; sd++)
#pragma unroll
            for (int m = 0; m < 4; m++) mf[ax][sd][m] = 0.0;
    const double dt = a.dt;
    T r1t = 0, dr1 = 0, cv1[3] = {0, 0, 0}, uu1 = 0, kw = 0;
    if (STAGE == 1) {
        const double r1 = M1[c], u1d[3] = {M1[n + c], M1[2 * n + c], M1[3 * n + c]};
        r1t = (T)r1;
        dr1 = (T)(r1 - (DELTA ? a.rho0 : 0.0));
        for (int d = 0; d < 3; d++) cv1[d] = (T)(a.cs * u1d[d] * a.iRT);
        uu1 = (T)(0.5 * (u1d[0] * u1d[0] + u1d[1] * u1d[1] + u1d[2] * u1d[2]) * a.iRT);
        kw = (T)(6.0 * dt / (6.0 * tau_c + dt));
    }
    const T wl = (T)(STAGE == 0 ? dt / 3.0 : 4.0 * dt / 7.0);
    T X[Q];

    load(0);
    store(0);
    __syncthreads();
    static_for<Q>([&](auto QC) {
        constexpr int q = decltype(QC)::value;
        if (q + 1 < Q) load(q + 1);
        const T f = fh[(long long)q * n + c];
        T b = 0, g = 0;
        if (STAGE == 1) {
            b = Ba[(long long)q * n + c];
            g = G[(long long)q * n + c];
        }
        const S *B = lds[q & 1] + own - BIAS;
        constexpr E3 e = lat_e<LAT>(q);
        constexpr double om = DELTA ? lat_w<LAT>(q) : 1.0;
        T acc = 0;
        static_for<3>([&](auto AXC) {
            constexpr int ax = decltype(AXC)::value;
            T vlo = 0, vhi = 0;
            static_for<36>([&](auto MC) {
                constexpr int m = decltype(MC)::value;
                constexpr int wi = kWin<LAT>.idx[ax][q][m];
                if constexpr (wi >= 0) {
                    constexpr int off = [] {
                        int o[3] = {0, 0, 0};
                        win_offset(ax, m, o);
                        return o[0] * PITCH[0] + o[1] * PITCH[1] + o[2] * PITCH[2] + BIAS;
                    }();
                    const T wv = wsh[wi / VW][wi % VW];
                    vlo = fmat(wv, B[off], vlo);
                    vhi = fmat(wv, B[off + PITCH[ax]], vhi);
                }
            });
            const double dlo = om * (double)vlo, dhi = om * (double)vhi;
            mf[ax][0][0] += dlo;
            mf[ax][1][0] += dhi;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                if (e.c[d] > 0) {
                    mf[ax][0][d + 1] += dlo;
                    mf[ax][1][d + 1] += dhi;
                } else if (e.c[d] < 0) {
                    mf[ax][0][d + 1] -= dlo;
                    mf[ax][1][d + 1] -= dhi;
                }
            }
            if constexpr (e.c[ax] != 0)
                acc += (T)(e.c[ax] * a.cs * a.inv_d[ax]) * (al[ax][1] * vhi - al[ax][0] * vlo);
        });
        T own_part;
        if (STAGE == 0) {
            own_part = (T)1.25 * B[BIAS] - (T)0.25 * f;
        } else {
            const T W = -kw * (g - eq_lat<T, DELTA, LAT, q>(cv1, r1t, dr1, uu1));
            // 4/7 f - 6/7 B_A + 9/7 G as f + 9/7 (G - f) - 6/7 (B_A - f): the
            // rounded coefficients then act on differences only, so the
            // constant (rho0) part of the stored deviations is kept exactly
            own_part = f + (T)(9.0 / 7.0) * (g - f) - (T)(6.0 / 7.0) * (b - f) + (T)0.75 * W;
        }
        X[q] = own_part - wl * acc;
        // The unrolled kernel is one basic block, in which nothing ties the
        // arithmetic to the barriers: keep this velocity's sums ahead of the
        // barrier (else they sink past every later one and all the window
        // values stay live until the end).
        asm volatile("" : "+v"(X[q]));
#pragma unroll
        for (int ax = 0; ax < 3; ax++)
#pragma unroll
            for (int sd = 0; sd < 2; sd++)
#pragma unroll
                for (int m = 0; m < 4; m++) asm volatile("" : "+v"(mf[ax][sd][m]));
        if (q + 1 < Q) store((q + 1) & 1);
        __syncthreads();
    });

    // face equilibria: the beta E part of the micro-flux, along the axes where
    // the velocity has a component.  Each face's weight in the output,
    // K = wl (cs / width) beta, is folded into its density terms: the face
    // adds K (D + R P) with D = rho - rho0 (DELTA) or rho, R = rho, and P as
    // in p_lat (times w for the f-form)
    T fcv[3][2][3], fuu[3][2], fkr[3][2], fkd[3];
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        double kd[2];
#pragma unroll
        for (int sd = 0; sd < 2; sd++) {
            double rho, u[3];
            moments_of(a, DELTA, mf[ax][sd], rho, u);
            // the sums held the momenta over cs: u here is the velocity over cs
            const double c2 = a.cs * a.cs;
            const double K = (double)wl * a.cs * a.inv_d[ax] * (1.0 - (double)al[ax][sd]);
            fkr[ax][sd] = (T)(K * rho);
            kd[sd] = K * (rho - (DELTA ? a.rho0 : 0.0));
            for (int d = 0; d < 3; d++) fcv[ax][sd][d] = (T)(c2 * u[d] * a.iRT);
            fuu[ax][sd] = (T)(0.5 * c2 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * a.iRT);
        }
        fkd[ax] = (T)(kd[1] - kd[0]);
    }
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    static_for<Q>([&](auto QC) {
        constexpr int q = decltype(QC)::value;
        constexpr E3 e = lat_e<LAT>(q);
        T lb = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            if (e.c[ax] == 0) continue;
            const T phi = p_lat<T, LAT, q>(fcv[ax][1], fuu[ax][1]);
            const T plo = p_lat<T, LAT, q>(fcv[ax][0], fuu[ax][0]);
            T d = fkd[ax] + fkr[ax][1] * phi - fkr[ax][0] * plo;
            if (!DELTA) d *= (T)lat_w<LAT>(q);
            lb += e.c[ax] > 0 ? d : -d;
        }
        X[q] -= lb;
        const double v = (DELTA ? lat_w<LAT>(q) : 1.0) * (double)X[q];
        s4[0] += v;
        for (int d = 0; d < 3; d++) {
            if (e.c[d] > 0) s4[d + 1] += v;
            if (e.c[d] < 0) s4[d + 1] -= v;
        }
    });
    double rho, u[3];
    moments_of(a, DELTA, s4, rho, u);
    for (int d = 0; d < 3; d++) u[d] *= a.cs;   // s4 held the momenta over cs
    if (!ok) return;
    const double cc = STAGE == 0 ? (24.0 * tau_c - 5.0 * dt) / (24.0 * tau_c + 4.0 * dt)
                                 : (12.0 * tau_c - dt) / (12.0 * tau_c + 3.0 * dt);
    // B = c X + (1 - c) E as X + (1 - c) (E - X), exact for X = E
    const T cet = (T)(1.0 - cc);
    const T rt = (T)rho, drt = (T)(rho - (DELTA ? a.rho0 : 0.0));
    const T cvo[3] = {(T)(a.cs * u[0] * a.iRT), (T)(a.cs * u[1] * a.iRT), (T)(a.cs * u[2] * a.iRT)};
    const T uu = (T)(0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * a.iRT);
    static_for<Q>([&](auto QC) {
        constexpr int q = decltype(QC)::value;
        out1[(long long)q * n + c] = X[q];
        out2[(long long)q * n + c] = X[q] + cet * (eq_lat<T, DELTA, LAT, q>(cvo, rt, drt, uu) - X[q]);
    });
    Mout[c] = rho;
    Mout[n + c] = u[0];
    Mout[2 * n + c] = u[1];
    Mout[3 * n + c] = u[2];
}

// ---------------------------------------------------------------------------
// Per-cell kernels: state conversions and the first B_A.
// ---------------------------------------------------------------------------
// fhat from the physical f (FP64 [q][cell]): fhat = f - dt/4 (E - f) / tau;
// then B_A and the moments, as the stage C epilogue leaves them.
template <class S, bool DELTA, int Q>
__global__ void k3_from_f(const Args a, const double *__restrict__ f, S *__restrict__ fh, S *__restrict__ Ba,
                          double *__restrict__ M0)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    const long long n = a.n;
    double r = 0, m[3] = {0, 0, 0};
    for (int q = 0; q < Q; q++) {
        const double v = f[q * n + c];
        r += v;
        for (int d = 0; d < 3; d++) m[d] += a.xi[d * Q + q] * v;
    }
    const double u[3] = {m[0] / r, m[1] / r, m[2] / r};
    const double uu2 = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * a.iRT;
    const double tau = a.tau[c], dt = a.dt;
    const double c1 = (12.0 * tau - dt) / (12.0 * tau + 3.0 * dt);
    double s4[4] = {0, 0, 0, 0};
    S g[Q];
    for (int q = 0; q < Q; q++) {
        const double E = eq_tab<double, false>(a, q, Q, r, 0.0, u, uu2);
        const double v = f[q * n + c];
        const double fhat = v - 0.25 * dt * (E - v) / tau;
        g[q] = DELTA ? (S)(fhat / a.w[q] - a.rho0) : (S)fhat;
        const double om = DELTA ? a.w[q] : 1.0;
        s4[0] += om * (double)g[q];
        for (int d = 0; d < 3; d++) s4[d + 1] = __builtin_fma(om * a.xi[d * Q + q], (double)g[q], s4[d + 1]);
    }
    double rho, uf[3];
    moments_of(a, DELTA, s4, rho, uf);
    const S rt = (S)rho, drt = (S)(rho - (DELTA ? a.rho0 : 0.0));
    const S ut[3] = {(S)uf[0], (S)uf[1], (S)uf[2]};
    const S uu = (S)(0.5 * (uf[0] * uf[0] + uf[1] * uf[1] + uf[2] * uf[2]) * a.iRT);
    for (int q = 0; q < Q; q++) {
        fh[q * n + c] = g[q];
        Ba[q * n + c] = g[q] + (S)(1.0 - c1) * (eq_tab<S, DELTA>(a, q, Q, rt, drt, ut, uu) - g[q]);
    }
    M0[c] = rho;
    for (int d = 0; d < 3; d++) M0[(d + 1) * n + c] = uf[d];
}

// equilibrium f = E(rho, u) from FP64 cell fields (rho [cell], u [3][cell])
template <int Q>
__global__ void k3_equilibrium(const Args a, const double *__restrict__ rho, const double *__restrict__ u3,
                               double *__restrict__ f)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    const long long n = a.n;
    const double u[3] = {u3[c], u3[n + c], u3[2 * n + c]};
    const double uu2 = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * a.iRT;
    for (int q = 0; q < Q; q++) f[q * n + c] = eq_tab<double, false>(a, q, Q, rho[c], 0.0, u, uu2);
}

// fhat (want_f = 0) or f = (4 tau fhat + dt E) / (4 tau + dt) in FP64
template <class S, bool DELTA, int Q>
__global__ void k3_to_f(const Args a, const S *__restrict__ fh, const double *__restrict__ M0, double *__restrict__ f,
                        int want_f)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n) return;
    const long long n = a.n;
    const double rho = M0[c], u[3] = {M0[n + c], M0[2 * n + c], M0[3 * n + c]};
    const double uu2 = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * a.iRT;
    const double tau = a.tau[c], dt = a.dt;
    for (int q = 0; q < Q; q++) {
        const double v = DELTA ? a.w[q] * ((double)fh[q * n + c] + a.rho0) : (double)fh[q * n + c];
        f[q * n + c] = want_f ? (4.0 * tau * v + dt * eq_tab<double, false>(a, q, Q, rho, 0.0, u, uu2)) /
                                    (4.0 * tau + dt)
                              : v;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// Window weights of the low face of a cell along axis ax for velocity q:
// the quadratic expansion (coefficient kq on the second-order terms) about
// the upwind cell U, evaluated at the foot point x_b - xi h, as weights on the
// cells around U (central 3-point derivatives, mixed ones from the four edge
// neighbours); a velocity parallel to the face takes the mean of the
// expansions about both cells.  Keys: offsets from the face's high cell.
static void window(const double xi[3], int ax, double h, const double d_[3], double kq,
                   std::map<std::array<int, 3>, double> &wmap)
{
    auto expand = [&](int Uax, const double dd[3], double scale) {
        std::array<int, 3> U = {0, 0, 0};
        U[ax] = Uax;
        auto add = [&](std::array<int, 3> o, double v) {
            for (int e = 0; e < 3; e++) o[e] += U[e];
            wmap[o] += scale * v;
        };
        double centre = 1.0;
        for (int e = 0; e < 3; e++) {
            const double r = dd[e] / d_[e];
            std::array<int, 3> p = {0, 0, 0}, m = {0, 0, 0};
            p[e] = 1;
            m[e] = -1;
            add(p, 0.5 * r + kq * r * r);
            add(m, -0.5 * r + kq * r * r);
            centre -= 2.0 * kq * r * r;
        }
        add({0, 0, 0}, centre);
        for (int e = 0; e < 3; e++)
            for (int f = e + 1; f < 3; f++) {
                const double v = kq * 2.0 * (dd[e] / d_[e]) * (dd[f] / d_[f]) / 4.0;
                for (int se = -1; se <= 1; se += 2)
                    for (int sf = -1; sf <= 1; sf += 2) {
                        std::array<int, 3> o = {0, 0, 0};
                        o[e] = se;
                        o[f] = sf;
                        add(o, se * sf * v);
                    }
            }
    };
    double dd[3];
    for (int e = 0; e < 3; e++) dd[e] = -xi[e] * h;
    const double en = xi[ax];
    if (en > 0.0) {
        dd[ax] = 0.5 * d_[ax] - en * h;
        expand(-1, dd, 1.0);
    } else if (en < 0.0) {
        dd[ax] = -0.5 * d_[ax] - en * h;
        expand(0, dd, 1.0);
    } else {
        dd[ax] = 0.5 * d_[ax];
        expand(-1, dd, 0.5);
        dd[ax] = -0.5 * d_[ax];
        expand(0, dd, 0.5);
    }
}

}  // namespace dk3

struct dugks3d {
    int nx, ny, nz, nq;
    long long n;
    bool delta;
    hipStream_t s;
    dk3::Args a;
    void *fh = nullptr, *Ba = nullptr, *G = nullptr, *Bc = nullptr;
    double *M0 = nullptr, *M1 = nullptr, *tau = nullptr;
    double *xi = nullptr, *w = nullptr, *wd = nullptr;
    int *wcnt = nullptr, *woff = nullptr;
    float *wf = nullptr;
    int lat = 0;              // 19 or 27: the velocity set is the library's lattice (k3_stage_lat)
    void *wcomp = nullptr;    // that kernel's weights: [stage][non-empty window entries]
    std::vector<void *> allocs;
};

namespace {

int err3(int code, const std::string &m) { return dk::set_error(code, m.c_str()); }

#define HIP3(expr)                                                                      \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return err3(DUGKS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int alloc3(dugks3d *h, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 8);
    if (e != hipSuccess) return err3(DUGKS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    h->allocs.push_back(*p);
    return DUGKS_OK;
}

template <class T>
int upload3(dugks3d *h, T **p, const T *src, size_t count)
{
    int rc = alloc3(h, (void **)p, sizeof(T) * count);
    if (rc) return rc;
    HIP3(hipMemcpy(*p, src, sizeof(T) * count, hipMemcpyHostToDevice));
    return DUGKS_OK;
}

dim3 grid1(long long n) { return dim3((unsigned)((n + 255) / 256)); }

size_t ssize(const dugks3d *h) { return h->delta ? sizeof(float) : sizeof(double); }

// device copy of a caller array (host or device) of count doubles
int stage_in(dugks3d *h, const double *src, size_t count, int mem, double **dev, bool &owned)
{
    if (mem == DUGKS_MEM_DEVICE) {
        *dev = const_cast<double *>(src);
        owned = false;
        return DUGKS_OK;
    }
    HIP3(hipMalloc((void **)dev, sizeof(double) * count));
    owned = true;
    hipError_t e = hipMemcpyAsync(*dev, src, sizeof(double) * count, hipMemcpyHostToDevice, h->s);
    if (e != hipSuccess) {
        (void)hipFree(*dev);
        return err3(DUGKS_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    }
    return DUGKS_OK;
}

template <class S, bool DELTA, int Q>
void launch_stage(dugks3d *h, int stage)
{
    const dim3 g((unsigned)(((h->a.ntiles + 7) / 8) * 8)), b(dk3::NT);
    S *fh = (S *)h->fh, *Ba = (S *)h->Ba, *G = (S *)h->G, *Bc = (S *)h->Bc;
    const S *wc = (const S *)h->wcomp;
    if (h->lat) {
        if (stage == 0)
            hipLaunchKernelGGL((dk3::k3_stage_lat<S, DELTA, Q, 0>), g, b, 0, h->s, h->a, Ba, fh, nullptr, nullptr,
                               nullptr, G, Bc, h->M1, wc);
        else
            hipLaunchKernelGGL((dk3::k3_stage_lat<S, DELTA, Q, 1>), g, b, 0, h->s, h->a, Bc, fh, Ba, G, h->M1, fh, Ba,
                               h->M0, wc);
        return;
    }
    if (stage == 0)
        hipLaunchKernelGGL((dk3::k3_stage<S, DELTA, Q, 0>), g, b, 0, h->s, h->a, Ba, fh, nullptr, nullptr, nullptr, G,
                           Bc, h->M1);
    else
        hipLaunchKernelGGL((dk3::k3_stage<S, DELTA, Q, 1>), g, b, 0, h->s, h->a, Bc, fh, Ba, G, h->M1, fh, Ba, h->M0);
}

void launch_stage_any(dugks3d *h, int stage)
{
    if (h->delta) {
        if (h->nq == 19) launch_stage<float, true, 19>(h, stage);
        else launch_stage<float, true, 27>(h, stage);
    } else {
        if (h->nq == 19) launch_stage<double, false, 19>(h, stage);
        else launch_stage<double, false, 27>(h, stage);
    }
}

template <int Q>
void launch_from_f(dugks3d *h, const double *f)
{
    if (h->delta)
        hipLaunchKernelGGL((dk3::k3_from_f<float, true, Q>), grid1(h->n), dim3(256), 0, h->s, h->a, f, (float *)h->fh,
                           (float *)h->Ba, h->M0);
    else
        hipLaunchKernelGGL((dk3::k3_from_f<double, false, Q>), grid1(h->n), dim3(256), 0, h->s, h->a, f,
                           (double *)h->fh, (double *)h->Ba, h->M0);
}

template <int Q>
void launch_to_f(dugks3d *h, double *f, int want_f)
{
    if (h->delta)
        hipLaunchKernelGGL((dk3::k3_to_f<float, true, Q>), grid1(h->n), dim3(256), 0, h->s, h->a, (const float *)h->fh,
                           h->M0, f, want_f);
    else
        hipLaunchKernelGGL((dk3::k3_to_f<double, false, Q>), grid1(h->n), dim3(256), 0, h->s, h->a,
                           (const double *)h->fh, h->M0, f, want_f);
}

int state_from_f(dugks3d *h, const double *fdev)
{
    if (h->nq == 19) launch_from_f<19>(h, fdev);
    else launch_from_f<27>(h, fdev);
    HIP3(hipGetLastError());
    return DUGKS_OK;
}

int read_f(dugks3d *h, double *out, int mem, int want_f)
{
    if (!h || !out || (mem != DUGKS_MEM_HOST && mem != DUGKS_MEM_DEVICE)) return err3(DUGKS_EINVAL, "bad argument");
    const size_t count = (size_t)h->nq * h->n;
    double *dst = out;
    if (mem == DUGKS_MEM_HOST) HIP3(hipMalloc((void **)&dst, sizeof(double) * count));
    if (h->nq == 19) launch_to_f<19>(h, dst, want_f);
    else launch_to_f<27>(h, dst, want_f);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && mem == DUGKS_MEM_HOST) {
        e = hipMemcpyAsync(out, dst, sizeof(double) * count, hipMemcpyDeviceToHost, h->s);
        if (e == hipSuccess) e = hipStreamSynchronize(h->s);
    }
    if (mem == DUGKS_MEM_HOST) (void)hipFree(dst);
    if (e != hipSuccess) return err3(DUGKS_EDEVICE, hipGetErrorString(e));
    return DUGKS_OK;
}

}  // namespace

extern "C" {

int dugks3d_create(const dugks3d_desc *d, dugks3d_t **out)
{
    if (!d || !out) return err3(DUGKS_EINVAL, "null descriptor or output");
    *out = nullptr;
    if (d->nx < 3 || d->ny < 3 || d->nz < 3) return err3(DUGKS_EINVAL, "nx, ny and nz must be >= 3");
    if (!(d->lx > 0) || !(d->ly > 0) || !(d->lz > 0)) return err3(DUGKS_EINVAL, "box lengths must be > 0");
    if (!d->xi || !d->w) return err3(DUGKS_EINVAL, "null velocity array");
    if (d->nq != 19 && d->nq != 27) return err3(DUGKS_ENOTSUP, "three-dimensional sets of 19 or 27 velocities only");
    if (!(d->dt > 0) || !(d->RT > 0)) return err3(DUGKS_EINVAL, "dt and RT must be > 0");
    if (d->precision != DUGKS_FP64 && d->precision != DUGKS_FP32_DELTA) return err3(DUGKS_EINVAL, "unknown precision");
    if (d->precision == DUGKS_FP32_DELTA && !(d->rho0 > 0)) return err3(DUGKS_EINVAL, "FP32-delta storage needs rho0 > 0");
    const int Q = d->nq;
    // CFL: per axis, the characteristic foot point stays within the upwind cell's stencil
    {
        const double wd3[3] = {d->lx / d->nx, d->ly / d->ny, d->lz / d->nz};
        for (int a = 0; a < 3; a++) {
            double cm = 0.0;
            for (int q = 0; q < Q; q++) cm = std::max(cm, std::fabs(d->xi[a * Q + q]));
            if (cm * d->dt > wd3[a] * (1.0 + 1e-12)) return err3(DUGKS_EINVAL, "CFL number above 1");
        }
    }
    const long long n = (long long)d->nx * d->ny * d->nz;
    // weight moments: sum w = 1, sum w xi = 0, sum w xi xi = RT I
    double s0 = 0, s1[3] = {0, 0, 0}, s2[3][3] = {{0}};
    for (int q = 0; q < Q; q++) {
        s0 += d->w[q];
        for (int a = 0; a < 3; a++) {
            s1[a] += d->w[q] * d->xi[a * Q + q];
            for (int b = 0; b < 3; b++) s2[a][b] += d->w[q] * d->xi[a * Q + q] * d->xi[b * Q + q];
        }
    }
    bool bad = std::fabs(s0 - 1.0) > 1e-10;
    for (int a = 0; a < 3; a++) {
        bad = bad || std::fabs(s1[a]) > 1e-10 * std::sqrt(d->RT);
        for (int b = 0; b < 3; b++) bad = bad || std::fabs(s2[a][b] - (a == b ? d->RT : 0.0)) > 1e-10 * d->RT;
    }
    if (bad) return err3(DUGKS_EMOMENT, "weights miss sum w = 1, sum w xi = 0 or sum w xi xi = RT I");
    std::vector<double> tau((size_t)n);
    for (long long c = 0; c < n; c++) {
        tau[c] = d->tau ? d->tau[c] : d->tau0;
        if (!(tau[c] > 0)) return err3(DUGKS_EINVAL, "tau must be > 0");
        if (d->dt / tau[c] > 12.0) return err3(DUGKS_EUNSTABLE, "dt/tau above 12");
    }

    dugks3d *h = new dugks3d();
    h->nx = d->nx;
    h->ny = d->ny;
    h->nz = d->nz;
    h->nq = Q;
    h->n = n;
    h->delta = d->precision == DUGKS_FP32_DELTA;
    h->s = (hipStream_t)d->stream;
    const double dw[3] = {d->lx / d->nx, d->ly / d->ny, d->lz / d->nz};
    const double kq = d->taylor_quad == 0.0 ? 1.0 : d->taylor_quad;
    // window tables of both stages
    std::vector<int> wcnt(2 * 3 * Q), woff(2 * 3 * Q * dk3::MAXW, 0);
    std::vector<double> wd(2 * 3 * Q * dk3::MAXW, 0.0);
    std::vector<float> wf(2 * 3 * Q * dk3::MAXW, 0.0f);
    const double hs[2] = {d->dt / 6.0, 5.0 * d->dt / 12.0};
    for (int st = 0; st < 2; st++)
        for (int ax = 0; ax < 3; ax++)
            for (int q = 0; q < Q; q++) {
                std::map<std::array<int, 3>, double> wm;
                const double x[3] = {d->xi[q], d->xi[Q + q], d->xi[2 * Q + q]};
                dk3::window(x, ax, hs[st], dw, kq, wm);
                const int tb = (st * 3 + ax) * Q + q;
                int m = 0;
                for (auto &kv : wm) {
                    if (kv.second == 0.0) continue;
                    if (m >= dk3::MAXW) {
                        dugks3d_destroy(h);
                        return err3(DUGKS_EINVAL, "window larger than its table");
                    }
                    const auto &o = kv.first;
                    woff[tb * dk3::MAXW + m] = (o[2] * dk3::LY + o[1]) * dk3::LX + o[0];
                    wd[tb * dk3::MAXW + m] = kv.second;
                    wf[tb * dk3::MAXW + m] = (float)kv.second;
                    m++;
                }
                wcnt[tb] = m;
            }
    // the library's lattice order (xi = c e_q, c the largest component)?
    {
        double cm = 0.0;
        for (int k = 0; k < 3 * Q; k++) cm = std::max(cm, std::fabs(d->xi[k]));
        bool same = cm > 0;
        for (int q = 0; q < Q && same; q++) {
            const dk3::E3 e = Q == 27 ? dk3::lat_e<27>(q) : dk3::lat_e<19>(q);
            const double wl = Q == 27 ? dk3::lat_w<27>(q) : dk3::lat_w<19>(q);
            for (int ax = 0; ax < 3; ax++)
                if (std::fabs(d->xi[ax * Q + q] - cm * e.c[ax]) > 1e-12 * cm) same = false;
            if (std::fabs(d->w[q] - wl) > 1e-14 * wl) same = false;
        }
        h->lat = same ? Q : 0;
        h->a.cs = cm;
    }
    std::vector<double> wcd;
    if (h->lat) {
        const int NW = Q == 27 ? dk3::kWin<27>.total : dk3::kWin<19>.total;
        wcd.assign(2 * (size_t)NW, 0.0);
        for (int st = 0; st < 2; st++)
            for (int ax = 0; ax < 3; ax++)
                for (int q = 0; q < Q; q++) {
                    std::map<std::array<int, 3>, double> wm;
                    const double x[3] = {d->xi[q], d->xi[Q + q], d->xi[2 * Q + q]};
                    dk3::window(x, ax, hs[st], dw, kq, wm);
                    for (int m = 0; m < 36; m++) {
                        const int wi = Q == 27 ? dk3::kWin<27>.idx[ax][q][m] : dk3::kWin<19>.idx[ax][q][m];
                        std::array<int, 3> o;
                        dk3::win_offset(ax, m, o.data());
                        auto it = wm.find(o);
                        const double v = it == wm.end() ? 0.0 : it->second;
                        if (wi >= 0) wcd[(size_t)st * NW + wi] = v;
                        else if (v != 0.0) {   // a weight outside the compile-time window
                            dugks3d_destroy(h);
                            return err3(DUGKS_EINVAL, "interface expansion outside its window");
                        }
                    }
                }
    }
    std::vector<float> wcf(wcd.begin(), wcd.end());
    std::vector<double> xi(d->xi, d->xi + 3 * Q), w(d->w, d->w + Q);
    int rc;
    if (h->lat) {
        rc = h->delta ? upload3(h, (float **)&h->wcomp, wcf.data(), wcf.size())
                      : upload3(h, (double **)&h->wcomp, wcd.data(), wcd.size());
        if (rc) {
            dugks3d_destroy(h);
            return rc;
        }
    }
    if ((rc = upload3(h, &h->xi, xi.data(), xi.size())) || (rc = upload3(h, &h->w, w.data(), w.size())) ||
        (rc = upload3(h, &h->tau, tau.data(), tau.size())) || (rc = upload3(h, &h->wcnt, wcnt.data(), wcnt.size())) ||
        (rc = upload3(h, &h->woff, woff.data(), woff.size())) || (rc = upload3(h, &h->wd, wd.data(), wd.size())) ||
        (rc = upload3(h, &h->wf, wf.data(), wf.size())) ||
        (rc = alloc3(h, &h->fh, ssize(h) * Q * n)) || (rc = alloc3(h, &h->Ba, ssize(h) * Q * n)) ||
        (rc = alloc3(h, &h->G, ssize(h) * Q * n)) || (rc = alloc3(h, &h->Bc, ssize(h) * Q * n)) ||
        (rc = alloc3(h, (void **)&h->M0, sizeof(double) * 4 * n)) ||
        (rc = alloc3(h, (void **)&h->M1, sizeof(double) * 4 * n))) {
        dugks3d_destroy(h);
        return rc;
    }
    dk3::Args &a = h->a;
    a.nx = d->nx;
    a.ny = d->ny;
    a.nz = d->nz;
    a.ntx = (d->nx + dk3::TX - 1) / dk3::TX;
    a.nty = (d->ny + dk3::TY - 1) / dk3::TY;
    a.ntiles = a.ntx * a.nty * ((d->nz + dk3::TZ - 1) / dk3::TZ);
    a.n = n;
    a.dt = d->dt;
    a.rho0 = h->delta ? d->rho0 : 0.0;
    a.iRT = 1.0 / d->RT;
    for (int e = 0; e < 3; e++) a.inv_d[e] = 1.0 / dw[e];
    a.h[0] = hs[0];
    a.h[1] = hs[1];
    a.xi = h->xi;
    a.w = h->w;
    a.tau = h->tau;
    a.wcnt = h->wcnt;
    a.woff = h->woff;
    a.wd = h->wd;
    a.wf = h->wf;
    *out = h;
    return DUGKS_OK;
}

int dugks3d_destroy(dugks3d_t *h)
{
    if (!h) return DUGKS_OK;
    for (void *p : h->allocs) (void)hipFree(p);
    delete h;
    return DUGKS_OK;
}

int dugks3d_set_state(dugks3d_t *h, const double *f, int mem)
{
    if (!h || !f || (mem != DUGKS_MEM_HOST && mem != DUGKS_MEM_DEVICE)) return err3(DUGKS_EINVAL, "bad argument");
    double *fd;
    bool owned;
    int rc = stage_in(h, f, (size_t)h->nq * h->n, mem, &fd, owned);
    if (rc) return rc;
    rc = state_from_f(h, fd);
    if (owned) {
        (void)hipStreamSynchronize(h->s);
        (void)hipFree(fd);
    }
    return rc;
}

int dugks3d_init_equilibrium(dugks3d_t *h, const double *rho, const double *u, int mem)
{
    if (!h || !rho || !u || (mem != DUGKS_MEM_HOST && mem != DUGKS_MEM_DEVICE))
        return err3(DUGKS_EINVAL, "bad argument");
    double *rd, *ud, *fd;
    bool ro, uo;
    int rc = stage_in(h, rho, (size_t)h->n, mem, &rd, ro);
    if (rc) return rc;
    if ((rc = stage_in(h, u, (size_t)3 * h->n, mem, &ud, uo))) {
        if (ro) (void)hipFree(rd);
        return rc;
    }
    hipError_t e = hipMalloc((void **)&fd, sizeof(double) * h->nq * h->n);
    if (e == hipSuccess) {
        if (h->nq == 19)
            hipLaunchKernelGGL((dk3::k3_equilibrium<19>), grid1(h->n), dim3(256), 0, h->s, h->a, rd, ud, fd);
        else
            hipLaunchKernelGGL((dk3::k3_equilibrium<27>), grid1(h->n), dim3(256), 0, h->s, h->a, rd, ud, fd);
        rc = state_from_f(h, fd);
        (void)hipStreamSynchronize(h->s);
        (void)hipFree(fd);
    } else {
        rc = err3(DUGKS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    if (ro) (void)hipFree(rd);
    if (uo) (void)hipFree(ud);
    return rc;
}

int dugks3d_step(dugks3d_t *h, int nsteps)
{
    if (!h || nsteps < 0) return err3(DUGKS_EINVAL, "bad argument");
    for (int s = 0; s < nsteps; s++) {
        launch_stage_any(h, 0);
        launch_stage_any(h, 1);
    }
    HIP3(hipGetLastError());
    return DUGKS_OK;
}

int dugks3d_step_timed(dugks3d_t *h, int nsteps, double *ms_a, double *ms_c)
{
    if (!h || nsteps < 1) return err3(DUGKS_EINVAL, "bad argument");
    std::vector<hipEvent_t> ev(4 * (size_t)nsteps);
    for (auto &e : ev) HIP3(hipEventCreate(&e));
    for (int s = 0; s < nsteps; s++) {
        HIP3(hipEventRecord(ev[4 * s], h->s));
        launch_stage_any(h, 0);
        HIP3(hipEventRecord(ev[4 * s + 1], h->s));
        HIP3(hipEventRecord(ev[4 * s + 2], h->s));
        launch_stage_any(h, 1);
        HIP3(hipEventRecord(ev[4 * s + 3], h->s));
    }
    HIP3(hipGetLastError());
    HIP3(hipStreamSynchronize(h->s));
    double ta = 0, tc = 0;
    for (int s = 0; s < nsteps; s++) {
        float x, y;
        HIP3(hipEventElapsedTime(&x, ev[4 * s], ev[4 * s + 1]));
        HIP3(hipEventElapsedTime(&y, ev[4 * s + 2], ev[4 * s + 3]));
        ta += x;
        tc += y;
    }
    for (auto &e : ev) hipEventDestroy(e);
    if (ms_a) *ms_a = ta / nsteps;
    if (ms_c) *ms_c = tc / nsteps;
    return DUGKS_OK;
}

int dugks3d_moments(dugks3d_t *h, double *rho, double *u, int mem)
{
    if (!h || (mem != DUGKS_MEM_HOST && mem != DUGKS_MEM_DEVICE)) return err3(DUGKS_EINVAL, "bad argument");
    const hipMemcpyKind k = mem == DUGKS_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (rho) HIP3(hipMemcpyAsync(rho, h->M0, sizeof(double) * h->n, k, h->s));
    if (u) HIP3(hipMemcpyAsync(u, h->M0 + h->n, sizeof(double) * 3 * h->n, k, h->s));
    if (mem == DUGKS_MEM_HOST) HIP3(hipStreamSynchronize(h->s));
    return DUGKS_OK;
}

int dugks3d_get_fhat(dugks3d_t *h, double *fhat, int mem) { return read_f(h, fhat, mem, 0); }

int dugks3d_get_state(dugks3d_t *h, double *f, int mem) { return read_f(h, f, mem, 1); }

}  // extern "C"
