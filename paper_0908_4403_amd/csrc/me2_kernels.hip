// Amplitude kernel: one point per lane, one work item (64 points x one chunk
// of helicity passes) per wave.  See me2_tree.hpp for the algorithm.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.hpp"
#include "me2_tree.hpp"

namespace heget {

// One work item: 64 points (one per lane) x one chunk of helicity walks.
// `tab` is this wave's LDS photon table (kPhotonFields * N * 64 values of R).
template <typename R, int N, int MB, int H>
__device__ __forceinline__ void me2_item(const double *__restrict__ mom, int64_t ld,
                                         const int32_t *__restrict__ index, int64_t npts,
                                         int64_t tile, int chunk, int nchunks, double coef,
                                         double *__restrict__ out, int64_t ld_out,
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

    constexpr int kPasses = (1 << N) / H;
    const int ppc = kPasses / nchunks;
    const double s = tree_sum<R, N, MB, H>(in, tab, lane, chunk * ppc, (chunk + 1) * ppc);
    double me2 = ldexp(coef * norm * s, 2 * m * (2 - N));
    if (!ok) me2 = __builtin_nan("");
    if (valid) {
        if (!isfinite(me2)) atomicOr(flags, 1u);
        out[static_cast<int64_t>(chunk) * ld_out + i] = me2;
    }
}

template <typename R, int N, int MB, int H, int WPB>
__global__ void __launch_bounds__(WPB * 64)
me2_kernel(const double *__restrict__ mom, int64_t ld, const int32_t *__restrict__ index,
           const int64_t *__restrict__ d_count, int64_t count, int nchunks, double coef,
           double *__restrict__ out, int64_t ld_out, unsigned *__restrict__ flags)
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
    me2_item<R, N, MB, H>(mom, ld, index, npts, tile, chunk, nchunks, coef, out, ld_out, flags,
                          tab, lane);
}

// ---------------------------------------------------------------- mixed-n batch

// Shapes inside the mixed kernel: its register allocation is the largest of
// its branches, so n = 4 takes the 3-level unroll there (the 4-level one alone
// would halve the occupancy of every other n).
template <typename R>
struct BatchShape {
    static constexpr int mb(int n) { return n < 4 ? n : (n == 4 ? 3 : 4); }
    static constexpr int h = std::is_same<R, float>::value ? 2 : 1;
};

__device__ __forceinline__ int64_t wave_broadcast(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(v & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(v >> 32));
    return (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo);
}

__global__ void batch_plan_kernel(BatchDesc b)
{
    int64_t acc = 0;
    b.item_start[0] = 0;
    for (int s = 0; s < b.nslices; ++s) {
        const int64_t cnt = *b.s[s].d_count;
        acc += ((cnt + 63) / 64) * b.s[s].nchunks;
        b.item_start[s + 1] = acc;
    }
}

template <typename R, int N>
__device__ __forceinline__ void batch_item(const SliceDesc &d, int64_t npts, int64_t tile, int chunk,
                                           unsigned *flags, R *tab, int lane)
{
    me2_item<R, N, BatchShape<R>::mb(N), BatchShape<R>::h>(d.mom, d.ld, d.index, npts, tile, chunk,
                                                           d.nchunks, d.coef, d.out, d.ld_out,
                                                           flags, tab, lane);
}

template <typename R>
__global__ void __launch_bounds__(256) me2_batch_kernel(BatchDesc b)
{
    __shared__ R tab_all[4 * kPhotonFields * 8 * 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    R *tab = tab_all + wave * kPhotonFields * 8 * 64;
    const int64_t total = b.item_start[b.nslices];
    for (;;) {
        int64_t item = 0;
        if (lane == 0) item = static_cast<int64_t>(atomicAdd(b.queue, 1ull));
        item = wave_broadcast(item);
        if (item >= total) break;
        int s = 0;
        while (s + 1 < b.nslices && item >= b.item_start[s + 1]) ++s;
        const SliceDesc &d = b.s[s];
        const int64_t local = item - b.item_start[s];
        const int64_t tile = local / d.nchunks;
        const int chunk = static_cast<int>(local - tile * d.nchunks);
        const int64_t npts = *d.d_count;
        switch (d.n) {
        case 2: batch_item<R, 2>(d, npts, tile, chunk, b.flags, tab, lane); break;
        case 3: batch_item<R, 3>(d, npts, tile, chunk, b.flags, tab, lane); break;
        case 4: batch_item<R, 4>(d, npts, tile, chunk, b.flags, tab, lane); break;
        case 5: batch_item<R, 5>(d, npts, tile, chunk, b.flags, tab, lane); break;
        case 6: batch_item<R, 6>(d, npts, tile, chunk, b.flags, tab, lane); break;
        case 7: batch_item<R, 7>(d, npts, tile, chunk, b.flags, tab, lane); break;
        default: batch_item<R, 8>(d, npts, tile, chunk, b.flags, tab, lane); break;
        }
    }
}

hipError_t launch_batch_plan(const BatchDesc &b, hipStream_t stream)
{
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(1), 0, stream, b);
    return hipGetLastError();
}

hipError_t launch_me2_batch(int prec, const BatchDesc &b, int grid, hipStream_t stream)
{
    if (prec == 1)
        hipLaunchKernelGGL(me2_batch_kernel<float>, dim3(grid), dim3(256), 0, stream, b);
    else
        hipLaunchKernelGGL(me2_batch_kernel<double>, dim3(grid), dim3(256), 0, stream, b);
    return hipGetLastError();
}

int me2_batch_blocks_per_cu(int prec)
{
    int blocks = 1;
    const void *f = prec == 1 ? reinterpret_cast<const void *>(&me2_batch_kernel<float>)
                              : reinterpret_cast<const void *>(&me2_batch_kernel<double>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, 256, 0) != hipSuccess || blocks < 1)
        blocks = 1;
    return blocks;
}

void me2_batch_shape(int prec, int n, int *mb, int *h)
{
    if (prec == 1) {
        *mb = BatchShape<float>::mb(n);
        *h = BatchShape<float>::h;
    } else {
        *mb = BatchShape<double>::mb(n);
        *h = BatchShape<double>::h;
    }
}

template <typename R, int N, int MB, int H, int WPB>
constexpr Me2Variant variant()
{
    return Me2Variant{std::is_same<R, float>::value ? 1 : 0, N, MB, H, WPB,
                      reinterpret_cast<const void *>(&me2_kernel<R, N, MB, H, WPB>)};
}

// Compiled shapes (the autotuner chooses among them per (prec, n)); the first
// entry for each (prec, n) is the untuned default.  MB = unrolled depth, H =
// helicities per walk, WPB = waves per block.
#define HG_V(R, N, MB, H, WPB) variant<R, N, MB, H, WPB>()
static const Me2Variant kVariants[] = {
    // FP32
    HG_V(float, 2, 2, 2, 4), HG_V(float, 2, 2, 4, 4), HG_V(float, 2, 2, 1, 4), HG_V(float, 2, 2, 2, 1),
    HG_V(float, 3, 3, 2, 4), HG_V(float, 3, 3, 4, 4), HG_V(float, 3, 3, 1, 4), HG_V(float, 3, 3, 2, 1),
    HG_V(float, 4, 4, 2, 4), HG_V(float, 4, 3, 2, 4), HG_V(float, 4, 3, 4, 4), HG_V(float, 4, 4, 1, 4),
    HG_V(float, 4, 4, 2, 1),
    HG_V(float, 5, 4, 2, 4), HG_V(float, 5, 3, 2, 4), HG_V(float, 5, 3, 4, 4), HG_V(float, 5, 4, 1, 4),
    HG_V(float, 5, 4, 2, 1),
    HG_V(float, 6, 4, 2, 4), HG_V(float, 6, 3, 2, 4), HG_V(float, 6, 3, 4, 4), HG_V(float, 6, 4, 1, 4),
    HG_V(float, 6, 4, 2, 1),
    HG_V(float, 7, 4, 2, 4), HG_V(float, 7, 3, 2, 4), HG_V(float, 7, 3, 4, 4), HG_V(float, 7, 4, 1, 4),
    HG_V(float, 8, 4, 2, 4), HG_V(float, 8, 3, 2, 4), HG_V(float, 8, 3, 4, 4), HG_V(float, 8, 4, 1, 4),
    // FP64
    HG_V(double, 2, 2, 1, 4), HG_V(double, 2, 2, 2, 4), HG_V(double, 2, 2, 1, 1),
    HG_V(double, 3, 3, 1, 4), HG_V(double, 3, 3, 2, 4), HG_V(double, 3, 3, 1, 1),
    HG_V(double, 4, 4, 1, 4), HG_V(double, 4, 3, 1, 4), HG_V(double, 4, 3, 2, 4), HG_V(double, 4, 4, 1, 1),
    HG_V(double, 5, 4, 1, 4), HG_V(double, 5, 3, 1, 4), HG_V(double, 5, 3, 2, 4), HG_V(double, 5, 4, 1, 1),
    HG_V(double, 6, 4, 1, 4), HG_V(double, 6, 3, 1, 4), HG_V(double, 6, 3, 2, 4), HG_V(double, 6, 4, 1, 1),
    HG_V(double, 7, 4, 1, 4), HG_V(double, 7, 3, 1, 4), HG_V(double, 7, 3, 2, 4), HG_V(double, 7, 4, 1, 1),
    HG_V(double, 8, 4, 1, 4), HG_V(double, 8, 3, 1, 4), HG_V(double, 8, 3, 2, 4), HG_V(double, 8, 4, 1, 1),
};
#undef HG_V

const Me2Variant *me2_variants(int *count)
{
    *count = static_cast<int>(sizeof(kVariants) / sizeof(kVariants[0]));
    return kVariants;
}

const Me2Variant *me2_default(int prec, int n)
{
    for (const Me2Variant &v : kVariants)
        if (v.prec == prec && v.n == n) return &v;
    return nullptr;
}

hipError_t launch_me2(const Me2Variant &v, const Me2Args &a, hipStream_t stream)
{
    const int64_t ntiles = (a.count + 63) / 64;
    const int64_t items = ntiles * a.nchunks;
    if (items == 0) return hipSuccess;
    const int64_t blocks = (items + v.wpb - 1) / v.wpb;
    void *args[] = {const_cast<double **>(&a.mom), const_cast<int64_t *>(&a.ld),
                    const_cast<int32_t **>(&a.index), const_cast<int64_t **>(&a.d_count),
                    const_cast<int64_t *>(&a.count), const_cast<int *>(&a.nchunks),
                    const_cast<double *>(&a.coef), const_cast<double **>(&a.out),
                    const_cast<int64_t *>(&a.ld_out), const_cast<unsigned **>(&a.flags)};
    return hipLaunchKernel(v.func, dim3(static_cast<unsigned>(blocks)), dim3(v.wpb * 64), args, 0,
                           stream);
}

}  // namespace heget
