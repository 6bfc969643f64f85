// Deterministic compensated sums on the device (FP64).  A partial sum is a
// (sum, compensation) pair combined with Knuth's error-free two-sum, so the
// rounding error of every addition is carried along; sums of squares use
// plain addition.  All trees have a fixed shape, so results do not depend on
// scheduling.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Cross-lane moves of an FP64 value without the LDS unit: a DPP permutation
// inside rows of 16 lanes (quad_perm, half-row and row mirrors), and the
// gfx950 row swaps, which exchange rows 1, 3 with rows 0, 2 (16) or lanes
// 32-63 with lanes 0-31 (32).  For a swap called with the same value twice,
// `lo` receives the even row (lower half) and `hi` the odd row (upper half)
// of each pair, on both rows of the pair.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, static_cast<uint32_t>(b), CTRL, 0xF, 0xF, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, static_cast<uint32_t>(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

template <int ROWS>
__device__ __forceinline__ void swap_f64(double v, double &lo, double &hi)
{
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
    const uint32_t b0 = static_cast<uint32_t>(b), b1 = static_cast<uint32_t>(b >> 32);
    uint32_t l0, l1, h0, h1;
    if constexpr (ROWS == 16) {
        const auto r0 = __builtin_amdgcn_permlane16_swap(b0, b0, false, false);
        const auto r1 = __builtin_amdgcn_permlane16_swap(b1, b1, false, false);
        l0 = r0[0], h0 = r0[1], l1 = r1[0], h1 = r1[1];
    } else {
        const auto r0 = __builtin_amdgcn_permlane32_swap(b0, b0, false, false);
        const auto r1 = __builtin_amdgcn_permlane32_swap(b1, b1, false, false);
        l0 = r0[0], h0 = r0[1], l1 = r1[0], h1 = r1[1];
    }
    lo = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(l1) << 32) | l0));
    hi = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(h1) << 32) | h0));
}

// One level of the wave tree: combine each lane's triple with its partner's.
// csum_add(a, b) and csum_add(b, a) give the same bits (the two-sum's error
// term is the exact rounding error of a.s + b.s), so both partners hold the
// same value after every level.
template <int CTRL>
__device__ __forceinline__ void dpp_level(CSum &cs, double &sq)
{
    const CSum o{dpp_f64<CTRL>(cs.s), dpp_f64<CTRL>(cs.c)};
    const double osq = dpp_f64<CTRL>(sq);
    cs = csum_add(cs, o);
    sq += osq;
}

template <int ROWS>
__device__ __forceinline__ void swap_level(CSum &cs, double &sq)
{
    CSum a, b;
    double qa, qb;
    swap_f64<ROWS>(cs.s, a.s, b.s);
    swap_f64<ROWS>(cs.c, a.c, b.c);
    swap_f64<ROWS>(sq, qa, qb);
    cs = csum_add(a, b);
    sq = qa + qb;
}

// Tree over the 64 lanes of a wave (all lanes active): pairs of lanes, of
// pairs, of quads (half-row mirror), of half rows (row mirror), of rows, of
// half waves.  Every lane ends with the total of (sum, compensation) and of
// the squares.  All moves are VALU operations, so the tree costs no LDS
// round trips.
__device__ __forceinline__ void wave_reduce(CSum &cs, double &sq)
{
    dpp_level<0xB1>(cs, sq);   // quad_perm [1,0,3,2]: lane ^ 1
    dpp_level<0x4E>(cs, sq);   // quad_perm [2,3,0,1]: lane ^ 2
    dpp_level<0x141>(cs, sq);  // row_half_mirror: lane i <-> 7 - i within 8
    dpp_level<0x140>(cs, sq);  // row_mirror: lane i <-> 15 - i within 16
    swap_level<16>(cs, sq);    // rows 0+1, 2+3
    swap_level<32>(cs, sq);    // lanes 0-31 + 32-63
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
