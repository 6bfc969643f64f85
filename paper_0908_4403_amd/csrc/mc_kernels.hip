// Monte-Carlo side of the path: phase-space generation with cuts, stream
// compaction of the surviving points, per-point weights of eq. (1)-(2) and a
// deterministic compensated reduction.  All FP64.
//
// Determinism: compaction keeps point order (block counts -> exclusive scan
// -> in-block ballot ranks), and every sum is a fixed tree (lanes by xor
// shuffles, waves through LDS, blocks in index order), so a configuration
// gives bitwise the same sigma on every run.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.hpp"

namespace heget {

template <int N>
__global__ void __launch_bounds__(256)
gen_kernel(GenParams g, double *__restrict__ mom, int64_t ld, double *__restrict__ wout,
           uint8_t *__restrict__ flag, int32_t *__restrict__ block_count)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    bool acc = false;
    if (i < g.npoints) {
        const uint64_t point = static_cast<uint64_t>(g.first + i);
        const PointKin pk = point_kinematics(g, point);
        Vec4 k[N];
        rambo<N>(pk.sqrt_shat, g.seed, point, k);
        acc = pk.above && pass_cuts<N>(k, pk.y, g.pt_min, g.eta_max, g.dr_min);
        const double e = 0.5 * pk.sqrt_shat;
        mom[0 * ld + i] = e;
        mom[1 * ld + i] = 0.0;
        mom[2 * ld + i] = 0.0;
        mom[3 * ld + i] = e;
        mom[4 * ld + i] = e;
        mom[5 * ld + i] = 0.0;
        mom[6 * ld + i] = 0.0;
        mom[7 * ld + i] = -e;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            mom[(8 + 4 * j) * ld + i] = k[j].e;
            mom[(9 + 4 * j) * ld + i] = k[j].x;
            mom[(10 + 4 * j) * ld + i] = k[j].y;
            mom[(11 + 4 * j) * ld + i] = k[j].z;
        }
        const double shat = pk.sqrt_shat * pk.sqrt_shat;
        double w;
        if (g.weight_kind == 0)
            w = g.phase_volume_coef * ipow(shat, N - 2);
        else
            w = g.partonic_coef * ipow(shat, N - 3) * pk.fpdf;
        wout[i] = acc ? w : 0.0;
        if (flag) flag[i] = acc ? 1 : 0;
    }
    if (block_count) {
        const int c = __syncthreads_count(acc ? 1 : 0);
        if (threadIdx.x == 0) block_count[blockIdx.x] = c;
    }
}

// Exclusive scan of nb counts by one block of 1024 threads.
__global__ void __launch_bounds__(1024)
scan_kernel(const int32_t *__restrict__ counts, int nb, int32_t *__restrict__ offsets,
            int64_t *__restrict__ total)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int beg = min(t * per, nb), end = min(beg + per, nb);
    int64_t s = 0;
    for (int j = beg; j < end; ++j) s += counts[j];
    part[t] = s;
    __syncthreads();
    // inclusive Hillis-Steele scan over the 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int j = beg; j < end; ++j) {
        offsets[j] = static_cast<int32_t>(run);
        run += counts[j];
    }
    if (t == 1023) *total = part[1023];
}

__global__ void __launch_bounds__(256)
compact_kernel(const uint8_t *__restrict__ flag, int64_t np, const int32_t *__restrict__ offsets,
               int32_t *__restrict__ index)
{
    __shared__ int wave_count[4];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const bool f = i < np && flag[i] != 0;
    const uint64_t b = __ballot(f);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rank = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) wave_count[w] = __popcll(b);
    __syncthreads();
    int base = offsets[blockIdx.x];
    for (int k = 0; k < w; ++k) base += wave_count[k];
    if (f) index[base + rank] = static_cast<int32_t>(i);
}

__global__ void __launch_bounds__(256)
sum_chunks_kernel(const double *__restrict__ part, int nchunks, int64_t ld,
                  const int64_t *__restrict__ d_count, int64_t count, double *__restrict__ out,
                  unsigned *__restrict__ flags)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t n = d_count ? *d_count : count;
    if (k >= n) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[c * ld + k];
    if (!isfinite(s)) atomicOr(flags, 1u);
    out[k] = s;
}

// (sum, compensation) pairs combined with an error-free two-sum.
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

__device__ __forceinline__ double shfl_xor_d(double v, int m)
{
    return __shfl_xor(v, m, 64);
}

// Block (256 threads) reduction of (sum, compensation, sum of squares) into thread 0.
__device__ __forceinline__ void block_reduce(CSum &cs, double &sq)
{
    __shared__ double sh[3][4];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const CSum o{shfl_xor_d(cs.s, m), shfl_xor_d(cs.c, m)};
        const double osq = shfl_xor_d(sq, m);
        cs = csum_add(cs, o);
        sq += osq;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][w] = cs.s;
        sh[1][w] = cs.c;
        sh[2][w] = sq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cs = {sh[0][0], sh[1][0]};
        sq = sh[2][0];
        for (int k = 1; k < 4; ++k) {
            cs = csum_add(cs, CSum{sh[0][k], sh[1][k]});
            sq += sh[2][k];
        }
    }
}

__global__ void __launch_bounds__(256)
weights_kernel(const double *__restrict__ me2, const int32_t *__restrict__ index,
               const double *__restrict__ wfac, const int64_t *__restrict__ d_count,
               double *__restrict__ partials, unsigned *__restrict__ flags)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t n = *d_count;
    double w = 0.0;
    if (k < n) {
        w = me2[k] * wfac[index[k]];
        if (!isfinite(w)) atomicOr(flags, 1u);
    }
    CSum cs{w, 0.0};
    double sq = w * w;
    block_reduce(cs, sq);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = cs.s;
        partials[3 * blockIdx.x + 1] = cs.c;
        partials[3 * blockIdx.x + 2] = sq;
    }
}

__global__ void __launch_bounds__(256)
final_kernel(const double *__restrict__ partials, int nb, const int64_t *__restrict__ d_count,
             double *__restrict__ res)
{
    // each thread folds a contiguous range in order, then a fixed tree
    const int t = threadIdx.x;
    const int per = (nb + 255) / 256;
    const int beg = min(t * per, nb), end = min(beg + per, nb);
    CSum cs{0.0, 0.0};
    double sq = 0.0;
    for (int j = beg; j < end; ++j) {
        cs = csum_add(cs, CSum{partials[3 * j], partials[3 * j + 1]});
        sq += partials[3 * j + 2];
    }
    block_reduce(cs, sq);
    if (t == 0) {
        res[0] = cs.s + cs.c;
        res[1] = cs.c;
        res[2] = sq;
        res[3] = static_cast<double>(*d_count);
    }
}

// sigma = sum/N and its MC error written as the heget_result layout
// {sigma, err, sum, comp, sum2, n_gen, n_acc} (five doubles, two int64).
__global__ void result_kernel(const double *__restrict__ res, int64_t n_gen, void *out)
{
    double *d = static_cast<double *>(out);
    int64_t *q = static_cast<int64_t *>(out);
    const double sum = res[0], sum2 = res[2];
    const double N = static_cast<double>(n_gen);
    const double sigma = n_gen > 0 ? sum / N : 0.0;
    const double var = n_gen > 1 ? (sum2 / N - sigma * sigma) / (N - 1.0) : 0.0;
    d[0] = sigma;
    d[1] = sqrt(var > 0.0 ? var : 0.0);
    d[2] = sum;
    d[3] = res[1];
    d[4] = sum2;
    q[5] = n_gen;
    q[6] = static_cast<int64_t>(res[3]);
}

__global__ void zero_u32_kernel(unsigned *p, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// ---------------------------------------------------------------- launchers

template <int N>
static hipError_t gen_n(const GenParams &g, double *mom, int64_t ld, double *w, uint8_t *flag,
                        int32_t *block_count, hipStream_t stream)
{
    const int64_t blocks = (g.npoints + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(gen_kernel<N>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, g,
                       mom, ld, w, flag, block_count);
    return hipGetLastError();
}

hipError_t launch_gen(int n, const GenParams &g, double *mom, int64_t ld, double *w,
                      uint8_t *flag, int32_t *block_count, hipStream_t stream)
{
    switch (n) {
    case 2: return gen_n<2>(g, mom, ld, w, flag, block_count, stream);
    case 3: return gen_n<3>(g, mom, ld, w, flag, block_count, stream);
    case 4: return gen_n<4>(g, mom, ld, w, flag, block_count, stream);
    case 5: return gen_n<5>(g, mom, ld, w, flag, block_count, stream);
    case 6: return gen_n<6>(g, mom, ld, w, flag, block_count, stream);
    case 7: return gen_n<7>(g, mom, ld, w, flag, block_count, stream);
    case 8: return gen_n<8>(g, mom, ld, w, flag, block_count, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_scan(const int32_t *counts, int nb, int32_t *offsets, int64_t *d_count,
                       hipStream_t stream)
{
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, stream, counts, nb, offsets, d_count);
    return hipGetLastError();
}

hipError_t launch_compact(const uint8_t *flag, int64_t np, const int32_t *offsets, int32_t *index,
                          hipStream_t stream)
{
    const int64_t blocks = (np + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(compact_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       flag, np, offsets, index);
    return hipGetLastError();
}

hipError_t launch_sum_chunks(const double *part, int nchunks, int64_t ld, const int64_t *d_count,
                             int64_t count, double *out, unsigned *flags, hipStream_t stream)
{
    const int64_t blocks = (count + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       part, nchunks, ld, d_count, count, out, flags);
    return hipGetLastError();
}

hipError_t launch_weights(const double *me2, const int32_t *index, const double *wfac,
                          const int64_t *d_count, int64_t max_count, double *partials,
                          unsigned *flags, hipStream_t stream)
{
    const int64_t blocks = (max_count + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(weights_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       me2, index, wfac, d_count, partials, flags);
    return hipGetLastError();
}

hipError_t launch_final(const double *partials, int nb, const int64_t *d_count, double *res,
                        hipStream_t stream)
{
    hipLaunchKernelGGL(final_kernel, dim3(1), dim3(256), 0, stream, partials, nb, d_count, res);
    return hipGetLastError();
}

hipError_t launch_result(const double *res, int64_t n_gen, void *out, hipStream_t stream)
{
    hipLaunchKernelGGL(result_kernel, dim3(1), dim3(1), 0, stream, res, n_gen, out);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned *p, int count, hipStream_t stream)
{
    hipLaunchKernelGGL(zero_u32_kernel, dim3((count + 255) / 256), dim3(256), 0, stream, p, count);
    return hipGetLastError();
}

}  // namespace heget
