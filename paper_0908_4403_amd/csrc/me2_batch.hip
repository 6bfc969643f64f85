// Mixed-n batch: one persistent amplitude kernel fed by an atomic work queue.
#include <hip/hip_runtime.h>

#include "me2_item.hpp"

namespace heget {

// ---------------------------------------------------------------- mixed-n batch

// Shapes inside the mixed kernel: 4-level unrolled subtrees whose last four
// photons close with pair sums at both ends.  Its register allocation is the
// largest of its branches: one wave per SIMD in both precisions, no spills.
template <typename R>
struct BatchShape {
    static constexpr bool fp32 = std::is_same<R, float>::value;
    static constexpr int mb(int n) { return n < 4 ? n : 4; }
    static constexpr int h = fp32 ? 2 : 1;
    static constexpr int cl = 3;
    static constexpr int ps(int n) { return n >= 6 ? 1 : 0; }  // prefix sets above the subtree
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
    // |M|^2 only: the weighted sums follow in a separate pass
    me2_item<R, N, BatchShape<R>::mb(N), BatchShape<R>::h, BatchShape<R>::cl, false, BatchShape<R>::ps(N)>(
        d.mom, d.ld, d.index, nullptr, npts, tile, chunk, d.nchunks, d.coef, d.out, d.ld_out, d.wfac,
        d.partials, nullptr, flags, tab, lane);
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
        // the first active lane takes the next item, so the queue advances on
        // every pass whichever lanes the compiled loop keeps active
        int64_t item = 0;
        if (lane == __builtin_amdgcn_readfirstlane(lane))
            item = static_cast<int64_t>(atomicAdd(b.queue, 1ull));
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

void me2_batch_shape(int prec, int n, int *mb, int *h, int *cl, int *ps)
{
    if (prec == 1) {
        *mb = BatchShape<float>::mb(n);
        *h = BatchShape<float>::h;
        *cl = BatchShape<float>::cl;
        *ps = BatchShape<float>::ps(n);
    } else {
        *mb = BatchShape<double>::mb(n);
        *h = BatchShape<double>::h;
        *cl = BatchShape<double>::cl;
        *ps = BatchShape<double>::ps(n);
    }
}

}  // namespace heget
