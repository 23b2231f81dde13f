// Selection by value (lattice 9 / 37, FP32-delta or FP64) of the lattice
// sweep launchers, which are instantiated per lattice and precision in their
// own object files.  Host code only.
#include "launchers.h"

namespace dk {

#define DUGKS_BY_LAT(lat, delta, CALL)                                     \
    do {                                                                   \
        if ((lat) == 9) {                                                  \
            if (delta) return CALL(LatD2Q9, float, true);                  \
            return CALL(LatD2Q9, double, false);                           \
        }                                                                  \
        if ((lat) == 37) {                                                 \
            if (delta) return CALL(LatD2Q37, float, true);                 \
            return CALL(LatD2Q37, double, false);                          \
        }                                                                  \
        return hipErrorInvalidValue;                                       \
    } while (0)

hipError_t launch_stage(int stage, int lat, bool delta, const SweepParams &p, double h, const void *X,
                        const void *F, void *out, const void *coef, hipStream_t s, int parts)
{
#define C_(L, S, D) small_stage<L, S, D>(stage, p, h, X, F, out, coef, s, parts)
    DUGKS_BY_LAT(lat, delta, C_);
#undef C_
}

hipError_t launch_stage_batched(int stage, int lat, bool delta, const SweepParams *P, const StageIO *io,
                                const int4 *work_fast, int nfast, const int4 *work_gen, int ngen,
                                int nthreads, size_t smem, hipStream_t s)
{
#define C_(L, S, D) small_stage_batched<L, S, D>(stage, P, io, work_fast, nfast, work_gen, ngen, nthreads, smem, s)
    DUGKS_BY_LAT(lat, delta, C_);
#undef C_
}

hipError_t set_stage_smem(int lat, bool delta, size_t bytes)
{
#define C_(L, S, D) small_smem<L, S, D>(bytes)
    DUGKS_BY_LAT(lat, delta, C_);
#undef C_
}

int fast_tile_index(int tx, int ty)
{
    int k = 0;
#define DUGKS_FS(A, B) if (tx == A && ty == B) return k; k++;
    DUGKS_FAST_SHAPES(DUGKS_FS)
#undef DUGKS_FS
    return -1;
}

hipError_t set_fast_smem(int lat, bool delta, int tx, int ty, size_t bytes)
{
#define C_(L, S, D) fast_smem<L, S, D>(tx, ty, bytes)
    DUGKS_BY_LAT(lat, delta, C_);
#undef C_
}

hipError_t launch_stage_fast(int stage, int lat, bool delta, const SweepParams &p, double h, const void *X,
                             const void *F, void *out, const void *coef, hipStream_t s)
{
#define C_(L, S, D) fast_stage<L, S, D>(stage, p, h, X, F, out, coef, s)
    DUGKS_BY_LAT(lat, delta, C_);
#undef C_
}

hipError_t launch_stage_fast_batched(int stage, int lat, bool delta, int tx, int ty, bool tau_field,
                                     const SweepParams *P, const StageIO *io, const int4 *work, int nwork,
                                     size_t smem, hipStream_t s)
{
#define C_(L, S, D) fast_stage_batched<L, S, D>(stage, tx, ty, tau_field, P, io, work, nwork, smem, s)
    DUGKS_BY_LAT(lat, delta, C_);
#undef C_
}

}  // namespace dk
