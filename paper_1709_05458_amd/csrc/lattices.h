// Integer lattices whose velocities are xi_q = clat * (ex(q), ey(q)): the
// paper's D2Q9 set (section "Discrete particle velocities") and a D2Q37 set
// of eight velocity shells.  Kernels take the lattice as a template argument
// so that every per-velocity integer is a compile-time constant.
#pragma once

namespace dk {

// shell(q): index of the velocity's shell |e|^2 (equal weights within a shell)
struct LatD2Q9 {
    static constexpr int Q = 9;
    static constexpr int NSHELL = 3;
    static constexpr __host__ __device__ int ex(int q) { return q / 3 - 1; }
    static constexpr __host__ __device__ int ey(int q) { return q % 3 - 1; }
    static constexpr __host__ __device__ int opp(int q) { return 8 - q; }
    static constexpr __host__ __device__ int shell(int q) { return ex(q) * ex(q) + ey(q) * ey(q); }
};

struct LatD2Q37 {
    static constexpr int Q = 37;
    static constexpr int NSHELL = 8;
    static constexpr __host__ __device__ int ex(int q)
    {
        constexpr int t[37] = {0, -1, 0, 0, 1, -1, -1, 1, 1, -2, 0, 0, 2, -2, -2, -1, -1, 1, 1,
                               2, 2, -2, -2, 2, 2, -3, 0, 0, 3, -3, -3, -1, -1, 1, 1, 3, 3};
        return t[q];
    }
    static constexpr __host__ __device__ int ey(int q)
    {
        constexpr int t[37] = {0, 0, -1, 1, 0, -1, 1, -1, 1, 0, -2, 2, 0, -1, 1, -2, 2, -2, 2,
                               -1, 1, -2, 2, -2, 2, 0, -3, 3, 0, -1, 1, -3, 3, -3, 3, -1, 1};
        return t[q];
    }
    static constexpr __host__ __device__ int opp(int q)
    {
        constexpr int t[37] = {0, 4, 3, 2, 1, 8, 7, 6, 5, 12, 11, 10, 9, 20, 19, 18, 17, 16, 15,
                               14, 13, 24, 23, 22, 21, 28, 27, 26, 25, 36, 35, 34, 33, 32, 31, 30, 29};
        return t[q];
    }
    static constexpr __host__ __device__ int shell(int q)
    {
        // |e|^2 = 0, 1, 2, 4, 5, 8, 9, 10
        constexpr int t[11] = {0, 1, 2, -1, 3, 4, -1, -1, 5, 6, 7};
        return t[ex(q) * ex(q) + ey(q) * ey(q)];
    }
};

}  // namespace dk
