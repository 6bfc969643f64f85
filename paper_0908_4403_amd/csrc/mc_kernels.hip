// Monte-Carlo side of the path: phase-space generation with cuts, stream
// compaction of the surviving points into an index list; per-point weights of
// eq. (1)-(2) are applied in the amplitude pass; a deterministic compensated
// reduction gives sigma and its error.  All FP64.
//
// Determinism: compaction keeps point order (block counts -> each block's
// offset, the sum of its predecessors' counts -> in-block ballot ranks), and
// every sum is a fixed tree (64-point tiles by a fixed tree of cross-lane
// moves, tiles in index order), so a configuration gives bitwise the same
// sigma on every run.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.hpp"
#include "reduce.hpp"

namespace heget {

// Kinematics and weight of one point in mode MODE, with the cut decision
// split: the FP32 screen only, giving 1 (pass),
// 0 (fail) or -1 (undecided: a cut variable within the screen band of its
// bound), and the frame rapidity for the FP64 decision of undecided points.
template <int N, int MODE>
__device__ __forceinline__ int point_setup_screened(const GenParams &g, uint64_t point, Vec4 (&k)[N],
                                                    double &e_beam, double &w, double &y)
{
    const PointKin pk = point_kinematics<MODE>(g, point);
    rambo<N>(pk.sqrt_shat, g.seed, point, k);
    const int s = pk.above ? screen_cuts<N>(k, pk.y, g.pt_min, g.eta_max, g.dr_min) : 0;
    y = pk.y;
    e_beam = 0.5 * pk.sqrt_shat;
    const double shat = pk.sqrt_shat * pk.sqrt_shat;
    if (g.weight_kind == 0)
        w = g.phase_volume_coef * ipow(shat, N - 2);
    else
        w = g.partonic_coef * ipow(shat, N - 3) * pk.fpdf;
    return s;
}

// SoA rows of one point: quark momenta (E, 0, 0, +-E), then the photons.
template <int N>
__device__ __forceinline__ void store_point(double *__restrict__ mom, int64_t ld, int64_t col,
                                            double e, const Vec4 (&k)[N])
{
    mom[0 * ld + col] = e;
    mom[1 * ld + col] = 0.0;
    mom[2 * ld + col] = 0.0;
    mom[3 * ld + col] = e;
    mom[4 * ld + col] = e;
    mom[5 * ld + col] = 0.0;
    mom[6 * ld + col] = 0.0;
    mom[7 * ld + col] = -e;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        mom[(8 + 4 * j) * ld + col] = k[j].e;
        mom[(9 + 4 * j) * ld + col] = k[j].x;
        mom[(10 + 4 * j) * ld + col] = k[j].y;
        mom[(11 + 4 * j) * ld + col] = k[j].z;
    }
}

// Every point, in point order; rejected points keep their momenta, weight 0.
// Optionally the accept flag per point and the accept count per block of 256.
template <int N, int MODE>
__global__ void __launch_bounds__(256)
gen_kernel(GenParams g, double *__restrict__ mom, int64_t ld, double *__restrict__ wout,
           uint8_t *__restrict__ flag, int32_t *__restrict__ block_count)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (g.clear_word && i == 0) *g.clear_word = 0u;
    bool acc = false;
    if (i < g.npoints) {
        double w, y;
        int s;
        {
            Vec4 k[N];
            double e;
            s = point_setup_screened<N, MODE>(g, static_cast<uint64_t>(g.first + i), k, e, w, y);
            store_point<N>(mom, ld, i, e, k);
        }
        if (s < 0) {
            // Rare: decide in FP64 from the momenta just stored.  The row
            // pointer is passed through an empty asm statement so that the
            // compiler reloads them instead of keeping every momentum live
            // through the whole kernel (which costs two waves per SIMD).
            __threadfence_block();  // this thread's stores above are visible to its loads
            const double *m = mom + i;
            asm volatile("" : "+v"(m));
            Vec4 k[N];
#pragma unroll
            for (int j = 0; j < N; ++j)
                k[j] = {m[(8 + 4 * j) * ld], m[(9 + 4 * j) * ld], m[(10 + 4 * j) * ld], m[(11 + 4 * j) * ld]};
            s = pass_cuts_fp64<N>(k, y, g.pt_min, g.eta_max, g.dr_min) ? 1 : 0;
        }
        acc = s == 1;
        wout[i] = acc ? w : 0.0;
        if (flag) flag[i] = acc ? 1 : 0;
        if (g.hel_out) g.hel_out[i] = draw_helicity<N>(g.seed, static_cast<uint64_t>(g.first + i));
    }
    if (block_count) {
        const int c = __syncthreads_count(acc ? 1 : 0);
        if (threadIdx.x == 0) block_count[blockIdx.x] = c;
    }
}

// Exclusive prefix sums of the nb per-block counts, in place, and their total
// into *d_count: one workgroup of 1024 threads walks the counts in chunks of
// 4096 (four consecutive counts per thread), carrying the running total.
// Used for large point counts, where the blocks of compact_kernel would
// otherwise each sum all their predecessors' counts (work growing as nb^2).
constexpr int kScanThreads = 1024;

__global__ void __launch_bounds__(kScanThreads)
block_scan_kernel(int32_t *__restrict__ counts, int nb, int64_t *__restrict__ d_count)
{
    __shared__ int wave_tot[kScanThreads / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int64_t carry = 0;
    for (int base = 0; base < nb; base += 4 * kScanThreads) {
        int v[4], own = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int idx = base + 4 * t + j;
            v[j] = idx < nb ? counts[idx] : 0;
            own += v[j];
        }
        // inclusive scan of `own` over the wave, then over the waves
        int inc = own;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            const int up = __shfl_up(inc, m, 64);
            if (lane >= m) inc += up;
        }
        if (lane == 63) wave_tot[w] = inc;
        __syncthreads();
        int before = 0, chunk = 0;
        for (int k = 0; k < kScanThreads / 64; ++k) {
            if (k < w) before += wave_tot[k];
            chunk += wave_tot[k];
        }
        int run = static_cast<int>(carry) + before + inc - own;  // offsets stay below 2^31
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int idx = base + 4 * t + j;
            if (idx < nb) counts[idx] = run;
            run += v[j];
        }
        carry += chunk;
        __syncthreads();  // wave_tot is rewritten by the next chunk
    }
    if (t == 0) *d_count = carry;
}

// Survivor list: index[offset_b + rank] = point, in point order, where block b
// (256 points) takes offset_b, the survivors of blocks 0..b-1, from `counts`
// already scanned into offsets (scanned = 1, block_scan_kernel wrote
// *d_count), or sums its predecessors' counts itself (a few KiB of
// L2-resident reads per block at the sizes this is used for, so no separate
// scan pass; the last block writes the total to *d_count).
__global__ void __launch_bounds__(256)
compact_kernel(const uint8_t *__restrict__ flag, int64_t np, const int32_t *__restrict__ counts,
               int nb, int scanned, int32_t *__restrict__ index, int64_t *__restrict__ d_count)
{
    __shared__ int part[4];
    __shared__ int wave_count[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int b = static_cast<int>(blockIdx.x);
    int s = 0;
    if (scanned) {
        s = t == 0 ? counts[b] : 0;
    } else {
        // the counts of blocks 0..b-1, four per 16-byte load (the count
        // buffer is 256-byte aligned), loads batched so their latencies overlap
        const int4 *c4 = reinterpret_cast<const int4 *>(counts);
        const int nfull = b >> 2;
#pragma unroll 4
        for (int j = t; j < nfull; j += 256) {
            const int4 v = c4[j];
            s += (v.x + v.y) + (v.z + v.w);
        }
        if (t < b - (nfull << 2)) s += counts[(nfull << 2) + t];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + t;
    const bool f = i < np && flag[i] != 0;
    const uint64_t bal = __ballot(f);
    const int rank = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) {
        part[w] = s;
        wave_count[w] = __popcll(bal);
    }
    __syncthreads();
    const int offset = part[0] + part[1] + part[2] + part[3];
    int base = offset;
    for (int k = 0; k < w; ++k) base += wave_count[k];
    if (f) index[base + rank] = static_cast<int32_t>(i);
    if (!scanned && t == 0 && b == nb - 1)
        *d_count = offset + wave_count[0] + wave_count[1] + wave_count[2] + wave_count[3];
}

// ---------------------------------------------------------------- event records

// Per generated point of an events call: weight 0 (the survivors' weights
// are scattered in afterwards), the rapidity of the partonic frame in the lab,
// the helicity configuration drawn in sampling mode (bit layout of
// draw_helicity_raw).
template <int MODE>
__global__ void __launch_bounds__(256)
event_fill_kernel(GenParams g, int n, double *__restrict__ w_all, double *__restrict__ y_out,
                  uint16_t *__restrict__ hel_out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= g.npoints) return;
    const uint64_t point = static_cast<uint64_t>(g.first + i);
    w_all[i] = 0.0;
    if (y_out) y_out[i] = point_kinematics<MODE>(g, point).y;
    if (hel_out) hel_out[i] = static_cast<uint16_t>(draw_helicity_raw(g.seed, point, n));
}

// Survivor weights back to point order: w_all[index[k]] = w[k], k < *d_count.
__global__ void __launch_bounds__(256)
event_scatter_kernel(const int32_t *__restrict__ index, const double *__restrict__ w,
                     const int64_t *__restrict__ d_count, int64_t max_count,
                     double *__restrict__ w_all)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t count = *d_count;
    if (k >= count || k >= max_count) return;
    w_all[index[k]] = w[k];
}

// ---------------------------------------------------------------- sums

__global__ void __launch_bounds__(256)
sum_chunks_kernel(const double *__restrict__ part, int nchunks, int64_t ld,
                  const int64_t *__restrict__ d_count, int64_t count, double *__restrict__ out,
                  const int32_t *__restrict__ index, const double *__restrict__ wfac,
                  double *__restrict__ partials, double *__restrict__ wout,
                  unsigned *__restrict__ flags)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t n = d_count ? *d_count : count;
    if (partials) {
        // whole waves stay for the tile reduction
        if ((k & ~int64_t(63)) >= n) return;
        double w = 0.0;
        if (k < n) {
            double s = 0.0;
            for (int c = 0; c < nchunks; ++c) s += part[c * ld + k];
            w = s * wfac[index ? static_cast<int64_t>(index[k]) : k];
            if (!isfinite(w)) atomicOr(flags, 1u);
            if (wout) wout[k] = w;
        }
        tile_partial(w, threadIdx.x & 63, partials, k >> 6);
        return;
    }
    if (k >= n) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[c * ld + k];
    if (!isfinite(s)) atomicOr(flags, 1u);
    out[k] = s;
}

constexpr int kFinalThreads = 1024;
constexpr int kFinalBatch = 8;

// Block reduction of (sum, compensation, sum of squares) into thread 0.
__device__ __forceinline__ void block_reduce(CSum &cs, double &sq)
{
    constexpr int kWaves = kFinalThreads / 64;
    __shared__ double sh[3][kWaves];
    wave_reduce(cs, sq);
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
        for (int q = 1; q < kWaves; ++q) {
            cs = csum_add(cs, CSum{sh[0][q], sh[1][q]});
            sq += sh[2][q];
        }
    }
}

// One block: thread t folds tiles t, t + T, t + 2T, ... in that order (loads
// issued kFinalBatch at a time), then a fixed tree.  The record is {sigma,
// err, sum, comp, sum2 (double), n_gen, n_acc (int64)}, sigma = sum / n_gen
// and err^2 = (sum2/N - sigma^2)/(N - 1).
__global__ void __launch_bounds__(kFinalThreads)
final_kernel(const double *__restrict__ partials, const int64_t *__restrict__ d_count,
             int64_t n_gen, double *__restrict__ res, void *record)
{
    const int64_t nacc = *d_count;
    const int64_t nt = (nacc + 63) / 64;
    const int t = threadIdx.x;
    CSum cs{0.0, 0.0};
    double sq = 0.0;
    for (int64_t j0 = t; j0 < nt; j0 += int64_t(kFinalThreads) * kFinalBatch) {
        double v[kFinalBatch][3];
#pragma unroll
        for (int u = 0; u < kFinalBatch; ++u) {
            const int64_t j = j0 + int64_t(u) * kFinalThreads;
            const bool in = j < nt;
            v[u][0] = in ? partials[3 * j + 0] : 0.0;
            v[u][1] = in ? partials[3 * j + 1] : 0.0;
            v[u][2] = in ? partials[3 * j + 2] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kFinalBatch; ++u) {
            cs = csum_add(cs, CSum{v[u][0], v[u][1]});
            sq += v[u][2];
        }
    }
    block_reduce(cs, sq);
    if (t != 0) return;
    const double sum = cs.s + cs.c;
    res[0] = sum;
    res[1] = cs.c;
    res[2] = sq;
    res[3] = static_cast<double>(nacc);
    if (record) {
        double *d = static_cast<double *>(record);
        int64_t *q = static_cast<int64_t *>(record);
        const double N = static_cast<double>(n_gen);
        const double sigma = n_gen > 0 ? sum / N : 0.0;
        const double var = n_gen > 1 ? (sq / N - sigma * sigma) / (N - 1.0) : 0.0;
        d[0] = sigma;
        d[1] = sqrt(var > 0.0 ? var : 0.0);
        d[2] = sum;
        d[3] = cs.c;
        d[4] = sq;
        q[5] = n_gen;
        q[6] = nacc;
    }
}

// ---------------------------------------------------------------- histograms

// Largest photon pT, or smallest photon-pair Delta R (pseudorapidity and
// azimuth as in the cuts; both invariant under the longitudinal boost).
template <int N>
__device__ __forceinline__ double observable_value(const double *__restrict__ mom, int64_t ld,
                                                   int64_t col, int which)
{
    double pt[N], eta[N], phi[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double x = mom[(9 + 4 * j) * ld + col], y = mom[(10 + 4 * j) * ld + col],
                     z = mom[(11 + 4 * j) * ld + col];
        const double pt2 = x * x + y * y;
        pt[j] = sqrt(pt2);
        eta[j] = copysign(fm::log((sqrt(pt2 + z * z) + fabs(z)) / pt[j]), z);
        phi[j] = fm::atan2(y, x);
    }
    if (which == 0) {
        double m = pt[0];
#pragma unroll
        for (int j = 1; j < N; ++j) m = fmax(m, pt[j]);
        return m;
    }
    double m = INFINITY;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = i + 1; j < N; ++j) {
            double dp = fabs(phi[i] - phi[j]);
            dp = dp > M_PI ? 2.0 * M_PI - dp : dp;
            const double de = eta[i] - eta[j];
            m = fmin(m, sqrt(de * de + dp * dp));
        }
    return m;
}

// Fixed-point exponent: every weight and every partial sum stays below 2^62.
__device__ __forceinline__ int hist_shift(const double *res)
{
    int e = 0;
    frexp(res[0], &e);  // sum of weights < 2^e
    return 62 - e;
}

template <int N>
__global__ void __launch_bounds__(256)
hist_kernel(const double *__restrict__ mom, int64_t ld, const int32_t *__restrict__ index,
            const double *__restrict__ w, const int64_t *__restrict__ d_count,
            const double *__restrict__ res, int which, int nbins, double lo, double hi,
            unsigned long long *__restrict__ bins)
{
    __shared__ unsigned long long lb[kHistMaxBins + 2];
    for (int b = threadIdx.x; b < nbins + 2; b += 256) lb[b] = 0ull;
    __syncthreads();
    const int64_t count = *d_count;
    const int shift = hist_shift(res);
    const double scale = static_cast<double>(nbins) / (hi - lo);
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; k < count;
         k += static_cast<int64_t>(gridDim.x) * 256) {
        const double wk = w[k];
        if (!(wk > 0.0) || !isfinite(wk)) continue;
        const double x = observable_value<N>(mom, ld, index[k], which);
        int b;
        if (x < lo) {
            b = 0;
        } else if (!(x < hi)) {
            b = nbins + 1;
        } else {
            b = 1 + static_cast<int>((x - lo) * scale);
            b = b > nbins ? nbins : b;
        }
        atomicAdd(&lb[b], static_cast<unsigned long long>(llrint(ldexp(wk, shift))));
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins + 2; b += 256)
        if (lb[b]) atomicAdd(&bins[b], lb[b]);
}

__global__ void hist_finish_kernel(const unsigned long long *__restrict__ bins, int nbins,
                                   const double *__restrict__ res, int64_t n_gen,
                                   double *__restrict__ hist)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins + 2) return;
    const int shift = hist_shift(res);
    hist[b] = n_gen > 0 ? ldexp(static_cast<double>(bins[b]), -shift) / static_cast<double>(n_gen)
                        : 0.0;
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
    // one kernel per partonic mode: the fixed-energy one needs far fewer registers
    const auto kern = g.mode == 1 ? gen_kernel<N, 1> : g.mode == 2 ? gen_kernel<N, 2> : gen_kernel<N, 0>;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, g, mom, ld,
                       w, flag, block_count);
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

hipError_t launch_events(int n, const GenParams &g, double *w_all, double *y, uint16_t *hel,
                         hipStream_t stream)
{
    const int64_t blocks = (g.npoints + 255) / 256;
    if (blocks == 0) return hipSuccess;
    const auto kern = g.mode == 1 ? event_fill_kernel<1> : g.mode == 2 ? event_fill_kernel<2>
                                                                         : event_fill_kernel<0>;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, g, n, w_all,
                       y, hel);
    return hipGetLastError();
}

hipError_t launch_event_scatter(const int32_t *index, const double *w, const int64_t *d_count,
                                int64_t max_count, double *w_all, hipStream_t stream)
{
    const int64_t blocks = (max_count + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(event_scatter_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                       stream, index, w, d_count, max_count, w_all);
    return hipGetLastError();
}

// Above this many 256-point blocks (2^20 points) the block counts are scanned
// by one workgroup first instead of each block summing its predecessors'.
constexpr int64_t kScanAboveBlocks = 4096;

hipError_t launch_compact(int32_t *counts, const uint8_t *flag, int64_t np, int32_t *index,
                          int64_t *d_count, hipStream_t stream)
{
    const int64_t blocks = (np + 255) / 256;
    if (blocks == 0) return hipSuccess;
    const int scanned = blocks > kScanAboveBlocks ? 1 : 0;
    if (scanned)
        hipLaunchKernelGGL(block_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, counts,
                           static_cast<int>(blocks), d_count);
    hipLaunchKernelGGL(compact_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       flag, np, counts, static_cast<int>(blocks), scanned, index, d_count);
    return hipGetLastError();
}

hipError_t launch_sum_chunks(const double *part, int nchunks, int64_t ld, const int64_t *d_count,
                             int64_t count, double *out, const int32_t *index, const double *wfac,
                             double *partials, double *wout, unsigned *flags, hipStream_t stream)
{
    const int64_t blocks = (count + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       part, nchunks, ld, d_count, count, out, index, wfac, partials, wout, flags);
    return hipGetLastError();
}

hipError_t launch_final(const double *partials, const int64_t *d_count, int64_t n_gen, double *res,
                        void *record, hipStream_t stream)
{
    hipLaunchKernelGGL(final_kernel, dim3(1), dim3(kFinalThreads), 0, stream, partials, d_count,
                       n_gen, res, record);
    return hipGetLastError();
}

template <int N>
static hipError_t hist_n(const double *mom, int64_t ld, const int32_t *index, const double *w,
                        const int64_t *d_count, int64_t max_count, const double *res, int which,
                        int nbins, double lo, double hi, unsigned long long *bins,
                        hipStream_t stream)
{
    int64_t blocks = (max_count + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
    hipLaunchKernelGGL(hist_kernel<N>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       mom, ld, index, w, d_count, res, which, nbins, lo, hi, bins);
    return hipGetLastError();
}

hipError_t launch_hist(int n, const double *mom, int64_t ld, const int32_t *index, const double *w,
                       const int64_t *d_count, int64_t max_count, const double *res,
                       int observable, int nbins, double lo, double hi, unsigned long long *bins,
                       hipStream_t stream)
{
    switch (n) {
    case 2: return hist_n<2>(mom, ld, index, w, d_count, max_count, res, observable, nbins, lo, hi, bins, stream);
    case 3: return hist_n<3>(mom, ld, index, w, d_count, max_count, res, observable, nbins, lo, hi, bins, stream);
    case 4: return hist_n<4>(mom, ld, index, w, d_count, max_count, res, observable, nbins, lo, hi, bins, stream);
    case 5: return hist_n<5>(mom, ld, index, w, d_count, max_count, res, observable, nbins, lo, hi, bins, stream);
    case 6: return hist_n<6>(mom, ld, index, w, d_count, max_count, res, observable, nbins, lo, hi, bins, stream);
    case 7: return hist_n<7>(mom, ld, index, w, d_count, max_count, res, observable, nbins, lo, hi, bins, stream);
    case 8: return hist_n<8>(mom, ld, index, w, d_count, max_count, res, observable, nbins, lo, hi, bins, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hist_finish(const unsigned long long *bins, int nbins, const double *res,
                              int64_t n_gen, double *hist, hipStream_t stream)
{
    hipLaunchKernelGGL(hist_finish_kernel, dim3((nbins + 2 + 255) / 256), dim3(256), 0, stream, bins,
                       nbins, res, n_gen, hist);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned *p, int count, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((count + 255) / 256), dim3(256), 0, stream, p, count);
    return hipGetLastError();
}

}  // namespace heget
