// Deterministic compensated sums on the device (FP64).  A partial sum is a
// (sum, compensation) pair combined with Knuth's error-free two-sum, so the
// rounding error of every addition is carried along; sums of squares use
// plain addition.  All trees have a fixed shape, so results do not depend on
// scheduling.
#pragma once
#include <hip/hip_runtime.h>

namespace heget {

struct CSum {
    double s, c;
};

__device__ __forceinline__ CSum csum_add(CSum a, CSum b)
{
    const double t = a.s + b.s;
    const double bb = t - a.s;
    const double err = (a.s - (t - bb)) + (b.s - bb);
    return {t, a.c + b.c + err};
}

// Butterfly over the 64 lanes of a wave: every lane ends with the total of
// (sum, compensation) and of the squares.
__device__ __forceinline__ void wave_reduce(CSum &cs, double &sq)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const CSum o{__shfl_xor(cs.s, m, 64), __shfl_xor(cs.c, m, 64)};
        const double osq = __shfl_xor(sq, m, 64);
        cs = csum_add(cs, o);
        sq += osq;
    }
}

// Weighted epilogue of the amplitude pass: lane value w (0 on lanes without a
// point) -> one (sum, compensation, sum of squares) triple per 64-point tile.
__device__ __forceinline__ void tile_partial(double w, int lane, double *__restrict__ partials,
                                             int64_t tile)
{
    CSum cs{w, 0.0};
    double sq = w * w;
    wave_reduce(cs, sq);
    if (lane == 0) {
        partials[3 * tile + 0] = cs.s;
        partials[3 * tile + 1] = cs.c;
        partials[3 * tile + 2] = sq;
    }
}

}  // namespace heget
