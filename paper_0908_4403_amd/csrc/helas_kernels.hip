// Batch kernels over the HELAS device library (helas.hpp):
//  * helas_eval_kernel: one library function on independent records, one
//    lane per record (FP64 records in and out; the arithmetic in FP32 or FP64);
//  * me2_frame_kernel: helicity-summed |M|^2 of u(p1) ubar(p2) -> n photons for
//    momenta in any frame, composed from the direction-general functions
//    (ixxxx0, oxxxx0, vxxxx0, fvoxx0, iovxxx), one lane per point.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "helas.hpp"
#include "kernels.hpp"

namespace heget {
namespace {

using helas::Cx;
using helas::Wave;

// record layouts: a wavefunction is 12 doubles (re, im of four components,
// then the momentum along the flow)
template <typename R>
__device__ inline Wave<R> load_wave(const double *x)
{
    Wave<R> w;
#pragma unroll
    for (int m = 0; m < 4; ++m) w.c[m] = helas::cx(R(x[2 * m]), R(x[2 * m + 1]));
#pragma unroll
    for (int m = 0; m < 4; ++m) w.p[m] = R(x[8 + m]);
    return w;
}

template <typename R>
__device__ inline void store_wave(const Wave<R> &w, double *y)
{
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        y[2 * m] = double(w.c[m].re);
        y[2 * m + 1] = double(w.c[m].im);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) y[8 + m] = double(w.p[m]);
}

template <typename R>
__global__ __launch_bounds__(256) void helas_eval_kernel(int func, int64_t count,
                                                         const double *__restrict__ in,
                                                         double *__restrict__ out)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double *x = in + i * helas_in_size(func);
    double *y = out + i * helas_out_size(func);
    if (func <= kHelasVxxxx2) {
        const R p[4] = {R(x[0]), R(x[1]), R(x[2]), R(x[3])};
        const int nhel = int(x[4]), nsf = int(x[5]);
        Wave<R> w;
        switch (func) {
        case kHelasIxxxx0: w = helas::ixxxx0(p, nhel, nsf); break;
        case kHelasIxxxx1: w = helas::ixxxx1(p, nhel, nsf); break;
        case kHelasIxxxx2: w = helas::ixxxx2(p, nhel, nsf); break;
        case kHelasOxxxx0: w = helas::oxxxx0(p, nhel, nsf); break;
        case kHelasOxxxx1: w = helas::oxxxx1(p, nhel, nsf); break;
        case kHelasOxxxx2: w = helas::oxxxx2(p, nhel, nsf); break;
        case kHelasVxxxx0: w = helas::vxxxx0(p, nhel, nsf); break;
        case kHelasVxxxx1: w = helas::vxxxx1(p, nhel); break;
        default: w = helas::vxxxx2(p, nhel); break;
        }
        store_wave(w, y);
        return;
    }
    if (func == kHelasIovxxx) {
        const Cx<R> v = helas::iovxxx(load_wave<R>(x), load_wave<R>(x + 12), load_wave<R>(x + 24),
                                      R(x[36]), R(x[37]));
        y[0] = double(v.re);
        y[1] = double(v.im);
        return;
    }
    const Wave<R> a = load_wave<R>(x), b = load_wave<R>(x + 12);
    const R g0 = R(x[24]), g1 = R(x[25]);
    Wave<R> w;
    if (func == kHelasFvixx0) w = helas::fvixx0(a, b, g0, g1);
    else if (func == kHelasFvoxx0) w = helas::fvoxx0(a, b, g0, g1);
    else w = helas::jioxx0(a, b, g0, g1);
    store_wave(w, y);
}

// The n! orderings of the photons in lexicographic order, each as the
// photon at every position (4 bits each) and the first position that differs
// from the previous ordering (bits 28-31): chains of consecutive orderings
// share their currents up to that position.  Built at compile time.
constexpr int factorial(int n) { return n <= 1 ? 1 : n * factorial(n - 1); }

template <int N>
struct Orderings {
    uint32_t e[factorial(N)];
    constexpr Orderings() : e()
    {
        int a[8] = {0, 1, 2, 3, 4, 5, 6, 7};
        int prev[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int t = 0; t < factorial(N); ++t) {
            int first = 0;
            if (t > 0)
                while (first < N && a[first] == prev[first]) ++first;
            uint32_t w = uint32_t(first) << 28;
            for (int d = 0; d < N; ++d) w |= uint32_t(a[d]) << (4 * d);
            e[t] = w;
            for (int d = 0; d < N; ++d) prev[d] = a[d];
            // next permutation
            int i = N - 2;
            while (i >= 0 && a[i] >= a[i + 1]) --i;
            if (i < 0) break;
            int j = N - 1;
            while (a[j] <= a[i]) --j;
            int s = a[i]; a[i] = a[j]; a[j] = s;
            for (int l = i + 1, r = N - 1; l < r; ++l, --r) { s = a[l]; a[l] = a[r]; a[r] = s; }
        }
    }
};
template <int N>
__constant__ constexpr Orderings<N> kOrderings{};

constexpr int kFrameBlock = 64;  // one wave per block: the photon table is per lane
constexpr int kEpsFields = 10;   // eps^1..3 (re, im) and the momentum

// Photon j of this lane from the per-lane table (field f at [f][j][lane]).
template <typename R, int N>
__device__ inline Wave<R> table_eps(const R *tab, int j, int lane)
{
    Wave<R> w;
    const R *t = tab + j * kFrameBlock + lane;
    w.c[0] = helas::cx(R(0));
#pragma unroll
    for (int m = 0; m < 3; ++m)
        w.c[m + 1] = helas::cx(t[(2 * m) * N * kFrameBlock], t[(2 * m + 1) * N * kFrameBlock]);
#pragma unroll
    for (int m = 0; m < 4; ++m) w.p[m] = t[(6 + m) * N * kFrameBlock];
    return w;
}

// |M|^2 summed over helicities.  Massless quarks keep their chirality along
// the line, so only (h_u, h_ubar) = (-1, +1) and (+1, -1) contribute (the
// other two vanish identically in every frame); all 2^n photon helicities.
// Each helicity configuration sums the n! orderings of eq. (6)-(8): every
// ordering is one chain of fvoxx0 from the ubar end closed on u with iovxxx,
// and consecutive orderings (lexicographic, the same on every lane) reuse the
// currents of their common prefix.  Photon polarisations sit in LDS so that
// the photon of a position, known only at run time, is one indexed read.
// Unit couplings in the chain; coef = (e Q)^(2n) applied in FP64.  Momenta
// are scaled by 2^-m (m even, 2^m ~ E1 + E2) so the FP32 range is never
// approached: |M(p)|^2 = 2^(2m(2-n)) |M(2^-m p)|^2, exactly.
template <typename R, int N>
__global__ __launch_bounds__(kFrameBlock) void me2_frame_kernel(const double *__restrict__ mom,
                                                                int64_t ld, int64_t np, double coef,
                                                                double *__restrict__ out,
                                                                unsigned *__restrict__ flags)
{
    __shared__ R tab[kEpsFields * N * kFrameBlock];
    const int lane = threadIdx.x;
    const int64_t i = int64_t(blockIdx.x) * kFrameBlock + lane;
    const bool live = i < np;
    const int64_t c = live ? i : 0;  // dead lanes compute on point 0 and store nothing
    int ex = 0;
    frexp(mom[c] + mom[4 * ld + c], &ex);
    ex &= ~1;
    R p[2][4];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int m = 0; m < 4; ++m) p[k][m] = R(ldexp(mom[(4 * k + m) * ld + c], -ex));
    R kph[N][4];
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int m = 0; m < 4; ++m) kph[j][m] = R(ldexp(mom[(4 * (j + 2) + m) * ld + c], -ex));
    double sum = 0.0;
    for (int q = 0; q < 2; ++q) {
        const int h = q ? 1 : -1;
        const Wave<R> u = helas::ixxxx0(p[0], h, 1);
        Wave<R> chain[N];
        chain[0] = helas::oxxxx0(p[1], -h, -1);
        for (int bits = 0; bits < (1 << N); ++bits) {
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const Wave<R> e = helas::vxxxx0(kph[j], ((bits >> j) & 1) ? 1 : -1, 1);
                R *t = tab + j * kFrameBlock + lane;
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    t[(2 * m) * N * kFrameBlock] = e.c[m + 1].re;
                    t[(2 * m + 1) * N * kFrameBlock] = e.c[m + 1].im;
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) t[(6 + m) * N * kFrameBlock] = e.p[m];
            }
            Cx<R> amp = helas::cx(R(0));
            for (int t = 0; t < factorial(N); ++t) {
                const uint32_t w = kOrderings<N>.e[t];
                const int first = int(w >> 28);
#pragma unroll
                for (int d = 0; d < N - 1; ++d)
                    if (d >= first)
                        chain[d + 1] = helas::fvoxx0(chain[d], table_eps<R, N>(tab, (w >> (4 * d)) & 15u, lane),
                                                     R(1), R(1));
                amp = amp + helas::iovxxx(u, chain[N - 1],
                                          table_eps<R, N>(tab, (w >> (4 * (N - 1))) & 15u, lane), R(1), R(1));
            }
            sum += double(amp.re) * double(amp.re) + double(amp.im) * double(amp.im);
        }
    }
    if (!live) return;
    const double r = sum * coef * ldexp(1.0, 2 * ex * (2 - N));
    out[i] = r;
    if (!isfinite(r)) atomicOr(flags, 1u);
}

template <typename R, int N>
hipError_t launch_frame_n(int64_t np, const double *mom, int64_t ld, double coef, double *out,
                          unsigned *flags, hipStream_t s)
{
    const unsigned blocks = unsigned((np + kFrameBlock - 1) / kFrameBlock);
    hipLaunchKernelGGL((me2_frame_kernel<R, N>), dim3(blocks), dim3(kFrameBlock), 0, s, mom, ld, np,
                       coef, out, flags);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_frame(int n, int64_t np, const double *mom, int64_t ld, double coef, double *out,
                        unsigned *flags, hipStream_t s)
{
    switch (n) {
    case 2: return launch_frame_n<R, 2>(np, mom, ld, coef, out, flags, s);
    case 3: return launch_frame_n<R, 3>(np, mom, ld, coef, out, flags, s);
    case 4: return launch_frame_n<R, 4>(np, mom, ld, coef, out, flags, s);
    case 5: return launch_frame_n<R, 5>(np, mom, ld, coef, out, flags, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_helas(int func, int prec, int64_t count, const double *in, double *out,
                        hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const unsigned blocks = unsigned((count + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(helas_eval_kernel<double>, dim3(blocks), dim3(256), 0, s, func, count, in, out);
    else
        hipLaunchKernelGGL(helas_eval_kernel<float>, dim3(blocks), dim3(256), 0, s, func, count, in, out);
    return hipGetLastError();
}

hipError_t launch_me2_frame(int n, int prec, int64_t np, const double *mom, int64_t ld, double coef,
                            double *out, unsigned *flags, hipStream_t s)
{
    if (np <= 0) return hipSuccess;
    return prec == 0 ? launch_frame<double>(n, np, mom, ld, coef, out, flags, s)
                     : launch_frame<float>(n, np, mom, ld, coef, out, flags, s);
}

}  // namespace heget
