// Vector-ALU FMA issue rate of the device: independent FMA chains per lane,
// no memory traffic inside the loop.  Built like every other kernel of the
// library (packed FP32 disabled), so it measures the ceiling the amplitude
// kernels can reach on this device and clock.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace heget {

constexpr int kPeakChains = 8;
constexpr int kPeakUnroll = 16;

template <typename R>
__global__ void __launch_bounds__(256) fma_peak_kernel(R *__restrict__ out, R a, R b, int iters)
{
    R x[kPeakChains];
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) x[c] = R(threadIdx.x) * R(1e-3) + R(c);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kPeakUnroll; ++u)
#pragma unroll
            for (int c = 0; c < kPeakChains; ++c) x[c] = fma(x[c], a, b);
    }
    R s = R(0);
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) s += x[c];
    out[static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x] = s;
}

hipError_t launch_fma_peak(int prec, void *out, int blocks, int iters, hipStream_t stream)
{
    if (prec == 1)
        hipLaunchKernelGGL(fma_peak_kernel<float>, dim3(blocks), dim3(256), 0, stream,
                           static_cast<float *>(out), 0.999f, 1e-3f, iters);
    else
        hipLaunchKernelGGL(fma_peak_kernel<double>, dim3(blocks), dim3(256), 0, stream,
                           static_cast<double *>(out), 0.999, 1e-3, iters);
    return hipGetLastError();
}

double fma_peak_flops(int blocks, int iters)
{
    return 2.0 * kPeakChains * kPeakUnroll * double(iters) * double(blocks) * 256.0;
}

}  // namespace heget
