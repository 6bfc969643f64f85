// Launch interfaces of the device kernels (host side).  Every launcher only
// enqueues work on `stream`; shapes are checked by the caller (heget_api.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kinematics.hpp"

namespace heget {

// One compiled shape of the amplitude kernel.
struct Me2Variant {
    int prec;   // 0 = FP64, 1 = FP32
    int n;      // photons
    int mb;     // unrolled bottom levels (photons held in registers)
    int h;      // helicity configurations per tree walk
    int cl;     // closing: 1 = photon by photon, 2 = last pair by pair vectors, 3 = last
                // four by pair sums at both ends (FP64 products for h >= 8), 4 = as 3
                // with the products in the working precision, 5 = as 4 with the
                // products of complementary splits summed before the FP64 sum
    int wpb;    // waves per block
    int pf;     // 1: resident waves loop over the items, loading the next one ahead
    int wpe;    // minimum waves per SIMD the kernel is compiled for (0: no bound)
    int ppl;    // points per lane: 64-point tiles per work item (1 unless pf = 0)
    int ps;     // 1: top levels walked by prefix sets (currents summed over their orderings);
                // 2-4: meet in the middle (2: momenta once per point, 3: per walk,
                // 4: per walk with the held v-bar-end currents in LDS)
    const void *func;  // kernel symbol
};

// All compiled variants (static table) and the default choice per (prec, n).
const Me2Variant *me2_variants(int *count);
const Me2Variant *me2_default(int prec, int n);
// The helicity-sampling kernel (h = 0) for (prec, n).
const Me2Variant *me2_sampled(int prec, int n);

// Arguments of one amplitude launch.
struct Me2Args {
    const double *mom;       // SoA [(n+2)*4][ld]
    int64_t ld;
    const int32_t *index;    // survivor -> column of mom (and of wfac), or nullptr (identity)
    const uint16_t *hel;     // sampled helicity configuration per column (H = 0 shapes only)
    const int64_t *d_count;  // number of points on the device, or nullptr
    int64_t count;           // number of points when d_count is null; else an upper bound
    int nchunks;             // helicity chunks (each a separate work item)
    double coef;             // 2 (e Q)^(2n)
    double *out;             // [nchunks][ld_out]: |M|^2 of each chunk (summed over chunks)
    int64_t ld_out;
    const double *wfac;      // per-point weight factor (with partials), else nullptr
    double *partials;        // one chunk: per-tile weighted triples instead of out
    double *wout;            // with partials: also each point's weight, or nullptr
    unsigned *flags;         // bit 0 set if a result is not finite
};

hipError_t launch_me2(const Me2Variant &v, const Me2Args &a, hipStream_t stream);

// Mixed-n batch: one persistent launch whose waves take (slice, tile, chunk)
// work items from an atomic queue, slices in the given order (most expensive
// per item first).  Each slice runs the batch shape for its n and writes
// |M|^2 per chunk to `out` (its `wfac` and `partials` are not used).
constexpr int kMaxSlices = 8;
struct SliceDesc {
    const double *mom;
    int64_t ld;
    const int32_t *index;
    const int64_t *d_count;
    double *out;
    int64_t ld_out;
    const double *wfac;
    double *partials;
    double coef;
    int n;
    int nchunks;
};
struct BatchDesc {
    SliceDesc s[kMaxSlices];
    int nslices;
    int64_t *item_start;           // [nslices + 1], written by launch_batch_plan
    unsigned long long *queue;     // zeroed before the launch
    unsigned *flags;
};
// item_start[s+1] = item_start[s] + ceil(count_s / 64) * nchunks_s (one thread).
hipError_t launch_batch_plan(const BatchDesc &b, hipStream_t stream);
// prec 0 = FP64, 1 = FP32; grid = number of persistent blocks of 256 threads.
hipError_t launch_me2_batch(int prec, const BatchDesc &b, int grid, hipStream_t stream);
int me2_batch_blocks_per_cu(int prec);
// (unrolled depth, helicities per walk, closing depth, prefix sets) of the mixed kernel for n
void me2_batch_shape(int prec, int n, int *mb, int *h, int *cl, int *ps);

// Phase-space generation (FP64): momenta of every point in SoA and its
// weight (kind 0: Phi_n or 0 if cut; kind 1: full eq. (1)-(2) factor without
// |M|^2, or 0 if cut); optionally the accept flag per point and the accept
// count per block of 256 points.
hipError_t launch_gen(int n, const GenParams &g, double *mom, int64_t ld, double *w,
                      uint8_t *flag, int32_t *block_count, hipStream_t stream);
// Survivor list: index[offset_b + rank] = point, in point order, with the
// offsets summed from the per-block counts; the survivor total -> *d_count.
// For more than 2^20 points the counts are first scanned into offsets in
// place (so `counts` is overwritten).
hipError_t launch_compact(int32_t *counts, const uint8_t *flag, int64_t np, int32_t *index,
                          int64_t *d_count, hipStream_t stream);

// Event records of a cross-section call, per generated point of g: w_all = 0,
// y = rapidity of the partonic frame, hel = the raw helicity draw (each
// optional but w_all); then w_all[index[k]] = w[k] for the survivors.
hipError_t launch_events(int n, const GenParams &g, double *w_all, double *y, uint16_t *hel,
                         hipStream_t stream);
hipError_t launch_event_scatter(const int32_t *index, const double *w, const int64_t *d_count,
                                int64_t max_count, double *w_all, hipStream_t stream);

// Sum of helicity chunks: out[k] = sum_c part[c*ld + k]; with `partials`, the
// per-tile weighted triples of sum_c part * wfac[index[k]] instead (as the
// amplitude kernel's one-chunk epilogue).
hipError_t launch_sum_chunks(const double *part, int nchunks, int64_t ld, const int64_t *d_count,
                             int64_t count, double *out, const int32_t *index, const double *wfac,
                             double *partials, double *wout, unsigned *flags, hipStream_t stream);

// Weighted histograms of an event observable (0: largest photon pT, 1:
// smallest photon-pair Delta R) over the survivors: w[k] of survivor k (point
// index[k] of mom) goes to bins[0] below lo, bins[1 + b] for bin b of nbins on
// [lo, hi), bins[nbins + 1] above.  Bins are 64-bit fixed-point integers
// scaled by 2^(62 - e) where 2^e > res[0] (the sum of all weights), so the sums
// are exact and independent of the order of the atomic adds; `bins` must be
// zero at launch.  hist_finish converts them to sum(w) / n_gen per bin.
constexpr int kHistMaxBins = 4096;
hipError_t launch_hist(int n, const double *mom, int64_t ld, const int32_t *index, const double *w,
                       const int64_t *d_count, int64_t max_count, const double *res,
                       int observable, int nbins, double lo, double hi, unsigned long long *bins,
                       hipStream_t stream);
hipError_t launch_hist_finish(const unsigned long long *bins, int nbins, const double *res,
                              int64_t n_gen, double *hist, hipStream_t stream);
// Fixed-order compensated reduction of the ceil(*d_count / 64) tile triples
// into res[0..3] = (sum + compensation, compensation, sum of squares, *d_count)
// and, if `record` is set, the heget_result record for n_gen generated points.
hipError_t launch_final(const double *partials, const int64_t *d_count, int64_t n_gen, double *res,
                        void *record, hipStream_t stream);
// FMA issue-rate probe: blocks x 256 threads, iters x 128 FMAs per thread into
// out[blocks * 256] (float for prec 1, double for prec 0); its flop count.
hipError_t launch_fma_peak(int prec, void *out, int blocks, int iters, hipStream_t stream);
double fma_peak_flops(int blocks, int iters);

// HELAS device library over independent FP64 records (helas_kernels.hip).
// func numbers the functions as heget_helas_fn does; a record holds
// helas_in_size(func) doubles in and helas_out_size(func) doubles out.
enum {
    kHelasIxxxx0 = 0, kHelasIxxxx1, kHelasIxxxx2, kHelasOxxxx0, kHelasOxxxx1, kHelasOxxxx2,
    kHelasVxxxx0, kHelasVxxxx1, kHelasVxxxx2, kHelasIovxxx, kHelasFvixx0, kHelasFvoxx0,
    kHelasJioxx0, kHelasFuncs
};
__host__ __device__ constexpr int helas_in_size(int func)
{
    return func <= kHelasVxxxx2 ? 6 : func == kHelasIovxxx ? 38 : 26;
}
__host__ __device__ constexpr int helas_out_size(int func) { return func == kHelasIovxxx ? 2 : 12; }
hipError_t launch_helas(int func, int prec, int64_t count, const double *in, double *out,
                        hipStream_t stream);
// |M|^2 of u ubar -> n photons (2 <= n <= kFrameMaxN) for momenta in any
// frame, SoA [(n+2)*4][ld]; coef = (e Q)^(2n); bit 0 of *flags set if a
// result is not finite.
constexpr int kFrameMaxN = 5;
hipError_t launch_me2_frame(int n, int prec, int64_t np, const double *mom, int64_t ld, double coef,
                            double *out, unsigned *flags, hipStream_t stream);

// Zero a small device buffer with a kernel (usable under stream capture).
hipError_t launch_zero_u32(unsigned *p, int count, hipStream_t stream);

// Fixed-size device workspace of static_scratch.hip: its size in bytes, and
// its device address on the current device (looked up once per device).
size_t static_scratch_bytes();
hipError_t static_scratch_ptr(void **ptr);

}  // namespace heget
