// Per-cell kernels around the sweep: conversions between the physical
// distribution f and the stored variable fhat = f - (dt/4) Omega(f) (paper,
// definitions under eq. feqIntD3rdHat2), equilibrium initialisation and cell
// moments rho = sum f, rho u = sum xi f ("Discrete particle velocities").
// One thread per cell, all velocities in a loop (any nq).
#include "dugks_internal.h"

namespace dk {

__device__ __forceinline__ double eq_poly(const SweepParams &p, int q, double ux, double uy)
{
    const double eu = p.xi[q] * ux + p.eta[q] * uy;
    const double uu = ux * ux + uy * uy;
    return 1.0 + eu / p.RT + eu * eu / (2.0 * p.RT * p.RT) - uu / (2.0 * p.RT);
}

// physical value of storage element x of velocity q
template <bool DELTA>
__device__ __forceinline__ double to_phys(const SweepParams &p, int q, double x)
{
    return DELTA ? p.w[q] * (x + p.rho0) : x;
}

template <bool DELTA>
__device__ __forceinline__ double to_store(const SweepParams &p, int q, double f)
{
    return DELTA ? f / p.w[q] - p.rho0 : f;
}

template <class S, bool DELTA>
__device__ void cell_moments(const SweepParams &p, const S *x, long long cell, double &rho,
                             double &ux, double &uy)
{
    const long long n = p.ncell;
    double a0 = 0, ax = 0, ay = 0;
    for (int q = 0; q < p.nq; q++) {
        const double v = (double)x[q * n + cell];
        const double d = DELTA ? p.w[q] * v : v;
        a0 += d;
        ax += p.xi[q] * d;
        ay += p.eta[q] * d;
    }
    if (DELTA) {
        rho = p.rho0 + (p.rho0 * p.M0m1 + a0);
        ux = (p.rho0 * p.M1x + ax) / rho;
        uy = (p.rho0 * p.M1y + ay) / rho;
    } else {
        rho = a0;
        ux = ax / rho;
        uy = ay / rho;
    }
}

// The stored state is f - (dt/m) Omega(f) = f + dt/(m tau) (f - E): m = 4 for
// T3S3 (fhat, eq. feqIntD3rdHat2 definitions), 2 for the T2 step (ftilde,
// Remark I), 1/P_{n+1} for the member a of the family (eq. EEWithP).
__device__ __forceinline__ double state_m(const SweepParams &p) { return p.state_m; }

template <class S, bool DELTA>
__global__ void k_set_state(const SweepParams p, const double *__restrict__ f, S *__restrict__ x)
{
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= p.ncell) return;
    const long long n = p.ncell;
    double rho = 0, mx = 0, my = 0;
    for (int q = 0; q < p.nq; q++) {
        const double v = f[q * n + cell];
        rho += v;
        mx += p.xi[q] * v;
        my += p.eta[q] * v;
    }
    const double ux = mx / rho, uy = my / rho;
    const double tau = p.tau_field ? p.tau[cell] : p.tau0;
    const double k = p.dt / (state_m(p) * tau);
    for (int q = 0; q < p.nq; q++) {
        const double v = f[q * n + cell];
        const double e = p.w[q] * rho * eq_poly(p, q, ux, uy);
        x[q * n + cell] = (S)to_store<DELTA>(p, q, v + k * (v - e));
    }
}

template <class S, bool DELTA>
__global__ void k_get_state(const SweepParams p, const S *__restrict__ x, double *__restrict__ f,
                            int physical)
{
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= p.ncell) return;
    const long long n = p.ncell;
    double rho, ux, uy;
    cell_moments<S, DELTA>(p, x, cell, rho, ux, uy);
    const double tau = p.tau_field ? p.tau[cell] : p.tau0;
    for (int q = 0; q < p.nq; q++) {
        const double fh = to_phys<DELTA>(p, q, (double)x[q * n + cell]);
        if (physical) {
            const double e = p.w[q] * rho * eq_poly(p, q, ux, uy);
            const double mt = state_m(p) * tau;
            f[q * n + cell] = (mt * fh + p.dt * e) / (mt + p.dt);
        } else {
            f[q * n + cell] = fh;
        }
    }
}

// f = E(rho, u), stored as fhat = f + dt/(4 tau) (f - E(moments of f)); the
// second term vanishes for moment-exact weights but not for, e.g., Newton-Cotes
// weights with a quadrature defect.
template <class S, bool DELTA>
__global__ void k_init_eq(const SweepParams p, const double *__restrict__ rho,
                          const double *__restrict__ ux, const double *__restrict__ uy,
                          S *__restrict__ x)
{
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= p.ncell) return;
    const long long n = p.ncell;
    const double r = rho[cell], u = ux[cell], v = uy[cell];
    double rf = 0, mfx = 0, mfy = 0;
    for (int q = 0; q < p.nq; q++) {
        const double f = p.w[q] * r * eq_poly(p, q, u, v);
        rf += f;
        mfx += p.xi[q] * f;
        mfy += p.eta[q] * f;
    }
    const double uf = mfx / rf, vf = mfy / rf;
    const double tau = p.tau_field ? p.tau[cell] : p.tau0;
    const double k = p.dt / (state_m(p) * tau);
    for (int q = 0; q < p.nq; q++) {
        const double P = eq_poly(p, q, u, v);
        const double Pf = eq_poly(p, q, uf, vf);
        if (DELTA) {
            // fhat / w_q - rho0 without forming rho - rho0 by cancellation
            const double dev = (r - p.rho0) + r * (P - 1.0);
            x[q * n + cell] = (S)(dev + k * (r * P - rf * Pf));
        } else {
            const double f = p.w[q] * r * P;
            x[q * n + cell] = (S)(f + k * (f - p.w[q] * rf * Pf));
        }
    }
}

template <class S, bool DELTA>
__global__ void k_moments(const SweepParams p, const S *__restrict__ x, double *__restrict__ rho,
                          double *__restrict__ ux, double *__restrict__ uy, int *__restrict__ bad)
{
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= p.ncell) return;
    double r, u, v;
    cell_moments<S, DELTA>(p, x, cell, r, u, v);
    if (rho) rho[cell] = r;
    if (ux) ux[cell] = u;
    if (uy) uy[cell] = v;
    if (bad && !(r == r && r < 1e300 && r > -1e300)) atomicOr(bad, 1);
}

static inline dim3 cells_grid(const SweepParams &p) { return dim3((unsigned)((p.ncell + 255) / 256)); }

hipError_t launch_set_state(const SweepParams &p, bool delta, const double *f, void *state,
                            hipStream_t s)
{
    if (delta)
        hipLaunchKernelGGL((k_set_state<float, true>), cells_grid(p), dim3(256), 0, s, p, f, (float *)state);
    else
        hipLaunchKernelGGL((k_set_state<double, false>), cells_grid(p), dim3(256), 0, s, p, f, (double *)state);
    return hipGetLastError();
}

hipError_t launch_get_state(const SweepParams &p, bool delta, const void *state, double *f,
                            int physical, hipStream_t s)
{
    if (delta)
        hipLaunchKernelGGL((k_get_state<float, true>), cells_grid(p), dim3(256), 0, s, p,
                           (const float *)state, f, physical);
    else
        hipLaunchKernelGGL((k_get_state<double, false>), cells_grid(p), dim3(256), 0, s, p,
                           (const double *)state, f, physical);
    return hipGetLastError();
}

hipError_t launch_init_eq(const SweepParams &p, bool delta, const double *rho, const double *ux,
                          const double *uy, void *state, hipStream_t s)
{
    if (delta)
        hipLaunchKernelGGL((k_init_eq<float, true>), cells_grid(p), dim3(256), 0, s, p, rho, ux, uy,
                           (float *)state);
    else
        hipLaunchKernelGGL((k_init_eq<double, false>), cells_grid(p), dim3(256), 0, s, p, rho, ux, uy,
                           (double *)state);
    return hipGetLastError();
}

hipError_t launch_moments(const SweepParams &p, bool delta, const void *state, double *rho,
                          double *ux, double *uy, int *bad, hipStream_t s)
{
    if (delta)
        hipLaunchKernelGGL((k_moments<float, true>), cells_grid(p), dim3(256), 0, s, p,
                           (const float *)state, rho, ux, uy, bad);
    else
        hipLaunchKernelGGL((k_moments<double, false>), cells_grid(p), dim3(256), 0, s, p,
                           (const double *)state, rho, ux, uy, bad);
    return hipGetLastError();
}

}  // namespace dk
