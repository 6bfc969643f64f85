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

// One work item: 64 points (one per lane) x one chunk of helicity walks.
// `tab` is this wave's LDS photon table (kPhotonFields * N * 64 values of R).
// Point i of the item is column index[i] of mom (column i without an index).
// H = 0 selects helicity sampling: one walk per lane with the configuration
// hel[column] (bit j set = photon j has helicity +1) instead of the sum.
// Output: with kWeighted, `partials` set and one chunk, the tile's (sum,
// compensation, sum of squares) of |M|^2 * wfac[column] (the Monte-Carlo
// weights of eq. (1)-(2)), and the weight itself at wout[i] when wout is set;
// otherwise |M|^2 of the chunk at out[chunk * ld_out + i].
template <typename R, int N, int MB, int H, int CL, bool kWeighted = true>
__device__ __forceinline__ void me2_item(const double *__restrict__ mom, int64_t ld,
                                         const int32_t *__restrict__ index,
                                         const uint16_t *__restrict__ hel, int64_t npts,
                                         int64_t tile, int chunk, int nchunks, double coef,
                                         double *__restrict__ out, int64_t ld_out,
                                         const double *__restrict__ wfac,
                                         double *__restrict__ partials, double *__restrict__ wout,
                                         unsigned *__restrict__ flags, R *tab, int lane)
{
    constexpr bool kTopInLds = N > MB;
    const int64_t i = tile * 64 + lane;
    const bool valid = i < npts;
    const int64_t ic = valid ? i : npts - 1;  // ragged tail: repeat the last point
    const int64_t src = index ? static_cast<int64_t>(index[ic]) : ic;

    // ---- FP64 set-up: preconditions, power-of-two scale, light-cone photons
    const double E1 = mom[0 * ld + src], p1x = mom[1 * ld + src], p1y = mom[2 * ld + src],
                 p1z = mom[3 * ld + src];
    const double E2 = mom[4 * ld + src], p2x = mom[5 * ld + src], p2y = mom[6 * ld + src],
                 p2z = mom[7 * ld + src];
    bool ok = p1x == 0.0 && p1y == 0.0 && p1z > 0.0 && p2x == 0.0 && p2y == 0.0 && p2z < 0.0;
    int m = 0;
    frexp(E1 + E2, &m);
    const double sc = ldexp(1.0, -m);
    // |u|^2 |vbar|^2 = (E1 + p1z) * 2 E2 (ixxxx1, oxxxx2), scaled
    double norm = ((E1 + p1z) * sc) * (2.0 * E2 * sc);

    PointIn<R, N> in;
    in.q0 = {static_cast<R>(-(E2 + p2z) * sc), static_cast<R>(-(E2 - p2z) * sc), R(0), R(0), R(0)};
    in.p1 = {static_cast<R>((E1 + p1z) * sc), static_cast<R>((E1 - p1z) * sc), R(0), R(0), R(0)};
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int r = 8 + 4 * j;
        const double E = mom[(r + 0) * ld + src] * sc, kx = mom[(r + 1) * ld + src] * sc,
                     ky = mom[(r + 2) * ld + src] * sc, kz = mom[(r + 3) * ld + src] * sc;
        const double pt2 = kx * kx + ky * ky;
        ok = ok && E > 0.0 && pt2 > 0.0;
        // k+ k- = pT^2 for a massless photon; take the cancellation-free one directly
        const double kp = kz >= 0.0 ? E + kz : pt2 / (E - kz);
        const double km = kz >= 0.0 ? pt2 / (E + kz) : E - kz;
        // vertex normalisation t ~ 1/(sqrt(2) E pT) in R; the exact remainder
        // (1/(sqrt(2) E pT t))^2 goes into the FP64 normalisation
        const R t = static_cast<R>(1.0 / sqrt(2.0 * E * E * pt2));
        const double td = static_cast<double>(t);
        norm *= 1.0 / (2.0 * E * E * pt2 * td * td);
        in.k[j] = {static_cast<R>(kp), static_cast<R>(km), static_cast<R>(kx), static_cast<R>(ky), t};
        if constexpr (kTopInLds) {
            tab[0 * N * 64 + j * 64 + lane] = in.k[j].p;
            tab[1 * N * 64 + j * 64 + lane] = in.k[j].m;
            tab[2 * N * 64 + j * 64 + lane] = in.k[j].x;
            tab[3 * N * 64 + j * 64 + lane] = in.k[j].y;
            tab[4 * N * 64 + j * 64 + lane] = in.k[j].t;
        }
    }

    double s;
    if constexpr (H == 0) {
        s = tree_one<R, N, MB, CL>(in, tab, lane, static_cast<uint32_t>(hel[src]));
    } else {
        constexpr int kPasses = (1 << N) / H;
        const int ppc = kPasses / nchunks;
        s = tree_sum<R, N, MB, H, CL>(in, tab, lane, chunk * ppc, (chunk + 1) * ppc);
    }
    double me2 = ldexp(coef * norm * s, 2 * m * (2 - N));
    if (!ok) me2 = __builtin_nan("");
    if (kWeighted && partials && nchunks == 1) {
        const double w = valid ? me2 * wfac[src] : 0.0;
        if (!isfinite(w)) atomicOr(flags, 1u);
        if (wout && valid) wout[i] = w;
        tile_partial(w, lane, partials, tile);
    } else if (valid) {
        if (!isfinite(me2)) atomicOr(flags, 1u);
        out[static_cast<int64_t>(chunk) * ld_out + i] = me2;
    }
}

template <typename R, int N, int MB, int H, int CL, int WPB>
__global__ void __launch_bounds__(WPB * 64)
me2_kernel(const double *__restrict__ mom, int64_t ld, const int32_t *__restrict__ index,
           const uint16_t *__restrict__ hel, const int64_t *__restrict__ d_count, int64_t count, int nchunks, double coef, double *__restrict__ out, int64_t ld_out,
           const double *__restrict__ wfac, double *__restrict__ partials,
           double *__restrict__ wout, unsigned *__restrict__ flags)
{
    __shared__ R tab_all[N > MB ? WPB * kPhotonFields * N * 64 : 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t npts = d_count ? *d_count : count;
    const int64_t ntiles = (npts + 63) >> 6;
    const int64_t item = static_cast<int64_t>(blockIdx.x) * WPB + wave;
    if (item >= ntiles * nchunks) return;  // whole wave
    const int64_t tile = item / nchunks;
    const int chunk = static_cast<int>(item - tile * nchunks);
    R *tab = tab_all + (N > MB ? wave * kPhotonFields * N * 64 : 0);
    me2_item<R, N, MB, H, CL>(mom, ld, index, hel, npts, tile, chunk, nchunks, coef, out, ld_out, wfac,
                              partials, wout, flags, tab, lane);
}

template <typename R, int N, int MB, int H, int CL, int WPB>
constexpr Me2Variant variant()
{
    return Me2Variant{std::is_same<R, float>::value ? 1 : 0, N, MB, H, CL, WPB,
                      reinterpret_cast<const void *>(&me2_kernel<R, N, MB, H, CL, WPB>)};
}

}  // namespace heget
