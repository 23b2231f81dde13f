// Launchers of one lattice and precision.  sweep.hip and sweep_fast.hip each
// define them and are compiled once per (lattice, precision) pair with
// explicit instantiations; dispatch.hip selects one by value.
#pragma once
#include "dugks_internal.h"
#include "lattices.h"

namespace dk {

// The tile shapes of the compile-time-shape kernels: the ones the library and
// the tile tuner choose from.
#define DUGKS_FAST_SHAPES(X) X(32, 8) X(16, 16) X(64, 4) X(8, 32)

template <class Lat, class S, bool DELTA>
hipError_t small_stage(int stage, const SweepParams &p, double h, const void *X, const void *F, void *out,
                       const void *coef, hipStream_t s, int parts);
template <class Lat, class S, bool DELTA>
hipError_t small_stage_batched(int stage, const SweepParams *P, const StageIO *io, const int4 *work_fast,
                               int nfast, const int4 *work_gen, int ngen, int nthreads, size_t smem,
                               hipStream_t s);
template <class Lat, class S, bool DELTA>
hipError_t small_smem(size_t bytes);

template <class Lat, class S, bool DELTA>
hipError_t fast_smem(int tx, int ty, size_t bytes);
template <class Lat, class S, bool DELTA>
hipError_t fast_stage(int stage, const SweepParams &p, double h, const void *X, const void *F, void *out,
                      const void *coef, hipStream_t s);
template <class Lat, class S, bool DELTA>
hipError_t fast_stage_batched(int stage, int tx, int ty, bool tf, const SweepParams *P, const StageIO *io,
                              const int4 *work, int nwork, size_t smem, hipStream_t s);

}  // namespace dk
