// Amplitude work item and kernel template: one point per lane, one work item
// (64 points x one chunk of helicity walks) per wave.  See me2_tree.hpp for
// the algorithm.  Instantiated by the me2_shapes_*.hip tables.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "kernels.hpp"
#include "me2_tree.hpp"
#include "reduce.hpp"

namespace heget {

// Inputs of one point of a work item, loaded ahead of the walk that uses them.
template <int N>
struct PointLoad {
    double x[8 + 4 * N];  // momenta p1, p2, k1..kN
    double wf;            // weight factor (0 without one)
    uint32_t hel;         // sampled helicity configuration (0 without one)
};

// Column of mom holding lane `lane` of `tile`: past the last point the tile
// repeats the last point (its result is not stored).  Columns are below 2^31;
// kept unsigned so that widening one needs no wait for the load that gave it.
__device__ __forceinline__ uint32_t point_column(const int32_t *__restrict__ index, int64_t npts,
                                                 int64_t tile, int lane)
{
    const int64_t i = tile * 64 + lane;
    const int64_t ic = i < npts ? i : npts - 1;
    return index ? static_cast<uint32_t>(index[ic]) : static_cast<uint32_t>(ic);
}

template <int N>
__device__ __forceinline__ PointLoad<N> load_point(const double *__restrict__ mom, int64_t ld,
                                                   uint32_t src, const double *__restrict__ wfac,
                                                   const uint16_t *__restrict__ hel)
{
    PointLoad<N> q;
#pragma unroll
    for (int r = 0; r < 8 + 4 * N; ++r) q.x[r] = mom[r * ld + src];
    q.wf = wfac ? wfac[src] : 0.0;
    q.hel = hel ? static_cast<uint32_t>(hel[src]) : 0u;
    return q;
}

// The walk and epilogue of one work item: 64 points (one per lane) x one
// chunk of helicity walks, from inputs already loaded.  `tab` is this wave's
// LDS photon table (kPhotonFields * N * 64 values of R).  H = 0 selects
// helicity sampling: one walk per lane with the configuration q.hel (bit j
// set = photon j has helicity +1) instead of the sum.
// Output: with kWeighted, `partials` set and one chunk, the tile's (sum,
// compensation, sum of squares) of |M|^2 * wf (the Monte-Carlo weights of
// eq. (1)-(2)), and the weight itself at wout[i] when wout is set; otherwise
// |M|^2 of the chunk at out[chunk * ld_out + i].
template <typename R, int N, int MB, int H, int CL, bool kWeighted = true, int PS = 0>
__device__ __forceinline__ void me2_compute(const PointLoad<N> &q, int64_t npts, int64_t tile,
                                            int chunk, int nchunks, double coef,
                                            double *__restrict__ out, int64_t ld_out,
                                            double *__restrict__ partials, double *__restrict__ wout,
                                            unsigned *__restrict__ flags, R *tab, int lane)
{
    constexpr bool kTopInLds = N > MB;
    const int64_t i = tile * 64 + lane;
    const bool valid = i < npts;

    // ---- FP64 set-up: preconditions, power-of-two scale, light-cone photons
    const double E1 = q.x[0], p1x = q.x[1], p1y = q.x[2], p1z = q.x[3];
    const double E2 = q.x[4], p2x = q.x[5], p2y = q.x[6], p2z = q.x[7];
    bool ok = p1x == 0.0 && p1y == 0.0 && p1z > 0.0 && p2x == 0.0 && p2y == 0.0 && p2z < 0.0;
    int m = 0;
    frexp(E1 + E2, &m);
    const double sc = ldexp(1.0, -m);
    // |u|^2 |vbar|^2 = (E1 + p1z) * 2 E2 (ixxxx1, oxxxx2), scaled
    double norm = ((E1 + p1z) * sc) * (2.0 * E2 * sc);

    PointIn<R, N> in;
    in.q0 = {static_cast<R>(-(E2 + p2z) * sc), static_cast<R>(-(E2 - p2z) * sc), R(0), R(0), R(0), R(0)};
    in.p1 = {static_cast<R>((E1 + p1z) * sc), static_cast<R>((E1 - p1z) * sc), R(0), R(0), R(0), R(0)};
    double norm_den = 1.0;  // product of the photons' 2 E^2 / pT^2, divided out once
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int r = 8 + 4 * j;
        const double E = q.x[r] * sc, kx = q.x[r + 1] * sc, ky = q.x[r + 2] * sc, kz = q.x[r + 3] * sc;
        const double pt2 = kx * kx + ky * ky;
        ok = ok && E > 0.0 && pt2 > 0.0;
        // k+ k- = pT^2 for a massless photon: the light-cone component free of
        // cancellation is E + |kz|, the other one pT^2 / (E + |kz|) (for FP32
        // amplitudes through the hardware reciprocal: within an FP32 ulp or so)
        const double big = E + fabs(kz);
        R small;
        if constexpr (std::is_same<R, float>::value)
            small = static_cast<float>(pt2) * __builtin_amdgcn_rcpf(static_cast<float>(big));
        else
            small = pt2 / big;
        const R kp = kz >= 0.0 ? static_cast<R>(big) : small;
        const R km = kz >= 0.0 ? small : static_cast<R>(big);
        // 1/k+ and 1/k- for the normalised vertex block (hardware reciprocal
        // in FP32, correctly rounded in FP64); the block's factor
        // pT / (sqrt(2) E) per photon enters |M|^2 here, in FP64
        R ip, im;
        if constexpr (std::is_same<R, float>::value) {
            ip = __builtin_amdgcn_rcpf(kp);
            im = __builtin_amdgcn_rcpf(km);
        } else {
            ip = 1.0 / kp;
            im = 1.0 / km;
        }
        norm_den *= 2.0 * E * E / pt2;
        in.k[j] = {kp, km, static_cast<R>(kx), static_cast<R>(ky), ip, im};
        if constexpr (kTopInLds) {
            tab[0 * N * 64 + j * 64 + lane] = in.k[j].p;
            tab[1 * N * 64 + j * 64 + lane] = in.k[j].m;
            tab[2 * N * 64 + j * 64 + lane] = in.k[j].x;
            tab[3 * N * 64 + j * 64 + lane] = in.k[j].y;
            tab[4 * N * 64 + j * 64 + lane] = in.k[j].ip;
            tab[5 * N * 64 + j * 64 + lane] = in.k[j].im;
        }
    }

    double s;
    if constexpr (H == 0) {
        s = tree_one<R, N, MB, CL, PS>(in, tab, lane, q.hel);
    } else {
        constexpr int kPasses = (1 << N) / H;
        const int ppc = kPasses / nchunks;
        s = tree_sum<R, N, MB, H, CL, PS>(in, tab, lane, chunk * ppc, (chunk + 1) * ppc);
    }
    double me2 = ldexp(coef * (norm / norm_den) * s, 2 * m * (2 - N));
    if (!ok) me2 = __builtin_nan("");
    if (kWeighted && partials && nchunks == 1) {
        const double w = valid ? me2 * q.wf : 0.0;
        if (!isfinite(w)) atomicOr(flags, 1u);
        if (wout && valid) wout[i] = w;
        tile_partial(w, lane, partials, tile);
    } else if (valid) {
        if (!isfinite(me2)) atomicOr(flags, 1u);
        out[static_cast<int64_t>(chunk) * ld_out + i] = me2;
    }
}

// Load and compute one work item (used by the mixed-n batch kernel).
template <typename R, int N, int MB, int H, int CL, bool kWeighted = true, int PS = 0>
__device__ __forceinline__ void me2_item(const double *__restrict__ mom, int64_t ld,
                                         const int32_t *__restrict__ index,
                                         const uint16_t *__restrict__ hel, int64_t npts,
                                         int64_t tile, int chunk, int nchunks, double coef,
                                         double *__restrict__ out, int64_t ld_out,
                                         const double *__restrict__ wfac,
                                         double *__restrict__ partials, double *__restrict__ wout,
                                         unsigned *__restrict__ flags, R *tab, int lane)
{
    const uint32_t src = point_column(index, npts, tile, lane);
    const double *wf = kWeighted && partials && nchunks == 1 ? wfac : nullptr;
    const PointLoad<N> q = load_point<N>(mom, ld, src, wf, H == 0 ? hel : nullptr);
    me2_compute<R, N, MB, H, CL, kWeighted, PS>(q, npts, tile, chunk, nchunks, coef, out, ld_out,
                                            partials, wout, flags, tab, lane);
}

// The amplitude kernel.  Work item k (64 points x one helicity chunk) goes to
// wave k mod (number of waves); with PF = 0 the grid has one wave per item,
// with PF = 1 it holds only the waves resident on the device and each wave
// walks its items in turn, loading the next item's inputs (and the survivor
// index of the one after) before the walk of the current one, so the walk
// hides the memory latency even at one wave per SIMD.  Item numbers are
// wave-uniform (scalar registers), so the loop and its bounds are scalar.
// WPE > 0 asks the compiler for at least WPE waves per SIMD (registers capped
// at 512 / WPE): the SIMD issues FP32 instructions of two waves side by side,
// which one wave alone cannot use.  PPL = 2 (with PF = 0) gives each lane two
// points: a work item is two consecutive 64-point tiles whose walks are
// independent instruction streams in one loop body (each with its own LDS
// photon table), for more instruction-level parallelism per wave; the
// weighted partial-sum buffer needs one spare tile slot after the last tile.
// PS = 1 walks the top levels by prefix sets (prefix_sets in me2_tree.hpp).
template <typename R, int N, int MB, int H, int CL, int WPB, int PF, int WPE, int PPL, int PS>
__global__ void __launch_bounds__(WPB * 64) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
me2_kernel(const double *__restrict__ mom, int64_t ld, const int32_t *__restrict__ index,
           const uint16_t *__restrict__ hel, const int64_t *__restrict__ d_count, int64_t count,
           int nchunks, double coef, double *__restrict__ out, int64_t ld_out,
           const double *__restrict__ wfac, double *__restrict__ partials,
           double *__restrict__ wout, unsigned *__restrict__ flags)
{
    static_assert(PPL == 1 || PF == 0, "several points per lane only without prefetch");
    // LDS of one walk: the photon table of the top levels, or the held
    // currents of the meeting in the middle with LDS staging (PS = 4)
    constexpr int kTab = N > MB ? kPhotonFields * N * 64 : PS == 4 ? meet_lds_values<N, (H > 0 ? H : 1)>() * 64 : 0;
    __shared__ R tab_all[kTab > 0 ? WPB * PPL * kTab : 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t npts = d_count ? *d_count : count;
    const int64_t ntiles = (npts + 63) >> 6;
    const int64_t nitems = ((ntiles + PPL - 1) / PPL) * nchunks;
    int64_t stride = static_cast<int64_t>(gridDim.x) * WPB;
    int64_t item = static_cast<int64_t>(blockIdx.x) * WPB + wave;
    int64_t end = nitems;
    // Blocks go round-robin to the eight XCDs, each with its own L2.  With a
    // grid of whole rounds, XCD x walks the contiguous items [x per,
    // (x + 1) per) of the items that exist (the device-side count), so
    // neighbouring tiles, which share cache lines of the gathered momenta,
    // are read through one L2, and every XCD gets an equal share.
    constexpr unsigned kXcds = 8;
    if (gridDim.x % kXcds == 0) {
        const int64_t x = blockIdx.x % kXcds;
        const int64_t per = (nitems + kXcds - 1) / kXcds;
        stride = static_cast<int64_t>(gridDim.x / kXcds) * WPB;
        item = x * per + static_cast<int64_t>(blockIdx.x / kXcds) * WPB + wave;
        end = (x + 1) * per < nitems ? (x + 1) * per : nitems;
    }
    if (item >= end) return;  // whole wave
    R *tab = tab_all + wave * PPL * kTab;
    const double *wf = partials && nchunks == 1 ? wfac : nullptr;
    const uint16_t *hl = H == 0 ? hel : nullptr;
    auto tile_of = [nchunks](int64_t it) -> int64_t { return nchunks == 1 ? it : it / nchunks; };
    if constexpr (PF == 0 && PPL == 1) {
        for (; item < end; item += stride) {
            const int64_t tile = tile_of(item);
            const int chunk = static_cast<int>(item - tile * nchunks);
            const PointLoad<N> q = load_point<N>(mom, ld, point_column(index, npts, tile, lane), wf, hl);
            me2_compute<R, N, MB, H, CL, true, PS>(q, npts, tile, chunk, nchunks, coef, out, ld_out,
                                                   partials, wout, flags, tab, lane);
        }
    } else if constexpr (PF == 0) {
        for (; item < end; item += stride) {
            const int64_t group = tile_of(item);
            const int chunk = static_cast<int>(item - group * nchunks);
            PointLoad<N> q[PPL];
#pragma unroll
            for (int p = 0; p < PPL; ++p)
                q[p] = load_point<N>(mom, ld, point_column(index, npts, group * PPL + p, lane), wf, hl);
            // unconditional, so that the walks can share one basic block: a
            // tile past the last one (only in the last group) holds no valid
            // point, stores nothing and writes a zero tile sum into the
            // spare slot the partial-sum buffer keeps after the last tile
#pragma unroll
            for (int p = 0; p < PPL; ++p)
                me2_compute<R, N, MB, H, CL, true, PS>(q[p], npts, group * PPL + p, chunk, nchunks, coef,
                                                       out, ld_out, partials, wout, flags, tab + p * kTab,
                                                       lane);
        }
    } else {
        // Loads for items past the last one read the last tile again (their
        // values are never used): every load is unconditional, so none has to
        // complete at a branch join before the walk it was issued ahead of.
        const int64_t last_tile = (npts - 1) >> 6;
        auto ahead = [&](int64_t it) -> int64_t {
            const int64_t t = tile_of(it);
            return t < last_tile ? t : last_tile;
        };
        PointLoad<N> cur = load_point<N>(mom, ld, point_column(index, npts, tile_of(item), lane), wf, hl);
        uint32_t src_next = point_column(index, npts, ahead(item + stride), lane);
        for (;;) {
            const PointLoad<N> nxt = load_point<N>(mom, ld, src_next, wf, hl);
            const uint32_t src_after = point_column(index, npts, ahead(item + 2 * stride), lane);
            const int64_t tile = tile_of(item);
            const int chunk = static_cast<int>(item - tile * nchunks);
            me2_compute<R, N, MB, H, CL, true, PS>(cur, npts, tile, chunk, nchunks, coef, out, ld_out,
                                                   partials, wout, flags, tab, lane);
            item += stride;
            if (item >= end) break;
            cur = nxt;
            src_next = src_after;
        }
    }
}

template <typename R, int N, int MB, int H, int CL, int WPB, int PF = 0, int WPE = 0, int PPL = 1,
          int PS = 0>
constexpr Me2Variant variant()
{
    return Me2Variant{std::is_same<R, float>::value ? 1 : 0, N, MB, H, CL, WPB, PF, WPE, PPL, PS,
                      reinterpret_cast<const void *>(&me2_kernel<R, N, MB, H, CL, WPB, PF, WPE, PPL, PS>)};
}

}  // namespace heget
