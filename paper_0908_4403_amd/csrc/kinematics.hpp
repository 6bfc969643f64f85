// Phase-space generation, cuts and Monte-Carlo weights on the device (FP64).
//
//  - RAMBO for n massless momenta (Kleiss, Stirling, Ellis, CPC 40 (1986) 359):
//    n isotropic momenta with energy density q exp(-q), then the conformal
//    map (boost to their rest frame + rescale) onto total momentum
//    (sqrt_s, 0, 0, 0).  The weight is constant: the massless n-body volume of
//    eq. (4), (2pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!).
//  - Cuts of eq. (9)-(10) in a frame boosted by rapidity y along z.
//  - Partonic kinematics of eq. (1) for the three modes of heget_mode.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fastmath.hpp"
#include "rng.hpp"

namespace heget {

struct Vec4 {
    double e, x, y, z;
};

// sqrt(x) for positive normal x (every square root of the generator: the
// arguments are bounded away from zero, overflow and denormals): the
// hardware estimate of 1/sqrt(x), one Goldschmidt step for the root and its
// half-reciprocal, then two Newton corrections of the root, which leave it
// within an ulp.  Without the range scaling and special cases of the
// general square root, it issues half the instructions.
__device__ __forceinline__ double sqrt_pos(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    double g = x * r, h = 0.5 * r;
    const double e = fma(-h, g, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
}

// RAMBO's conformal transformation in place: boost the N vectors to the rest
// frame of their sum Q and rescale the sum to (sqrt_s, 0, 0, 0).  1/M and
// 1/(1 + gamma) = M/(M + Q0) both come from the one quotient 1/(M (M + Q0)).
template <int N>
__device__ __forceinline__ void conformal_map(double sqrt_s, Vec4 (&k)[N])
{
    double Qe = 0.0, Qx = 0.0, Qy = 0.0, Qz = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        Qe += k[i].e;
        Qx += k[i].x;
        Qy += k[i].y;
        Qz += k[i].z;
    }
    const double M = sqrt_pos(Qe * Qe - Qx * Qx - Qy * Qy - Qz * Qz);
    const double r = 1.0 / (M * (M + Qe));
    const double inv_m = (M + Qe) * r;
    const double bx = -Qx * inv_m, by = -Qy * inv_m, bz = -Qz * inv_m;
    const double x = sqrt_s * inv_m;
    const double gam = Qe * inv_m;
    const double a = M * M * r;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double bq = bx * k[i].x + by * k[i].y + bz * k[i].z;
        const double e = k[i].e;
        k[i].e = x * (gam * e + bq);
        k[i].x = x * (k[i].x + bx * e + a * bq * bx);
        k[i].y = x * (k[i].y + by * e + a * bq * by);
        k[i].z = x * (k[i].z + bz * e + a * bq * bz);
    }
}

// The same map for a sum Q = (sqrt_s + d0, d) within rounding of
// (sqrt_s, 0, 0, 0), to first order in d / sqrt_s: beta = -d / sqrt_s,
// gamma = 1 and x = 1 - d0 / sqrt_s.  The terms left out are of order
// (d / sqrt_s)^2 relative, far below one rounding.
template <int N>
__device__ __forceinline__ void rebalance(double sqrt_s, Vec4 (&k)[N])
{
    double Qe = 0.0, Qx = 0.0, Qy = 0.0, Qz = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        Qe += k[i].e;
        Qx += k[i].x;
        Qy += k[i].y;
        Qz += k[i].z;
    }
    const double inv = 1.0 / sqrt_s;
    const double x = 1.0 - (Qe - sqrt_s) * inv;
    const double bx = -Qx * inv, by = -Qy * inv, bz = -Qz * inv;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double e = k[i].e;
        k[i].e = x * (e + (bx * k[i].x + by * k[i].y + bz * k[i].z));
        k[i].x = x * fma(bx, e, k[i].x);
        k[i].y = x * fma(by, e, k[i].y);
        k[i].z = x * fma(bz, e, k[i].z);
    }
}

// Photon momenta of point `point`: four uniforms from stream 0, block i, for photon i.
template <int N>
__device__ __forceinline__ void rambo(double sqrt_s, uint64_t seed, uint64_t point, Vec4 (&k)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double u[4];
        uniform_quad(seed, point, static_cast<uint32_t>(i), 0u, u);
        const double ucos = u[0], uphi = u[1], ue1 = u[2], ue2 = u[3];
        const double c = 2.0 * ucos - 1.0;
        const double s = sqrt_pos(1.0 - c * c);
        double sf, cf;
        fm::sincospi(2.0 * uphi, &sf, &cf);  // azimuth 2 pi uphi
        const double e = -fm::log(ue1 * ue2);
        k[i] = {e, e * s * cf, e * s * sf, e * c};
    }
    conformal_map<N>(sqrt_s, k);
    // The map scales the rounding-level masses of the isotropic vectors by
    // about the square of its boost factor, which is large when they are
    // nearly collinear.  Put every momentum back on shell and map once more:
    // now a near-identity, so the result is massless and conserves momentum to
    // rounding (exact arithmetic gives the same points).
#pragma unroll
    for (int i = 0; i < N; ++i) k[i].e = sqrt_pos(k[i].x * k[i].x + k[i].y * k[i].y + k[i].z * k[i].z);
    rebalance<N>(sqrt_s, k);
}

// 1 if every photon has pT > pt_min and |eta + y| < eta_max and every pair
// Delta R > dr_min (bounds <= 0 are off).  eta = atanh(pz/|p|), evaluated as
// sign(pz) log((|p| + |pz|)^2 / pT^2) / 2, which has no cancellation near the
// beam; phi = atan2(py, px).  Both with the short functions of fastmath.hpp,
// and pT and Delta R compared through their squares: these only decide cuts,
// and a decision can move only for a point within a few ulp of a bound.
template <int N>
__device__ __forceinline__ bool pass_cuts_fp64(const Vec4 (&k)[N], double y, double pt_min,
                                               double eta_max, double dr_min)
{
    double eta[N], phi[N];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double pt2 = k[i].x * k[i].x + k[i].y * k[i].y;
        const double pabs = sqrt(pt2 + k[i].z * k[i].z);
        const double big = pabs + fabs(k[i].z);
        eta[i] = copysign(0.5 * fm::log(big * big / pt2), k[i].z) + y;
        phi[i] = fm::atan2(k[i].y, k[i].x);
        if (pt_min > 0.0) ok = ok && (pt2 > pt_min * pt_min);
        if (eta_max > 0.0) ok = ok && (fabs(eta[i]) < eta_max);
    }
    if (dr_min > 0.0) {
        const double dr2 = dr_min * dr_min;
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = i + 1; j < N; ++j) {
                const double de = eta[i] - eta[j];
                double dp = fabs(phi[i] - phi[j]);
                dp = dp > M_PI ? 2.0 * M_PI - dp : dp;
                ok = ok && (de * de + dp * dp > dr2);
            }
    }
    return ok;
}

// The eta and Delta R parts of the same decision in FP32: 1 (pass), 0 (fail),
// or -1 when an eta lies within kEtaScreen of +-eta_max or a Delta R^2 within
// kDr2Screen of dr_min^2, where the FP32 values (about 2e-6 from the FP64 ones
// in eta up to |eta| = 5, 5e-5 in Delta R^2) could sit on the other side.
// pT is compared in FP64 (it is cheap).  Outside the bands the two
// evaluations agree, so the screen changes no decision, only its cost.
constexpr float kEtaScreen = 1e-4f;
constexpr float kDr2Screen = 1e-3f;

template <int N>
__device__ __forceinline__ int screen_cuts(const Vec4 (&k)[N], double y, double pt_min,
                                           double eta_max, double dr_min)
{
    float eta[N], phi[N];
    bool ok = true, unsure = false;
    const float ln2_half = 0.34657359f;  // ln(2) / 2
    const float pi = 3.14159265f, half_pi = 1.57079633f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double pt2 = k[i].x * k[i].x + k[i].y * k[i].y;
        if (pt_min > 0.0) ok = ok && (pt2 > pt_min * pt_min);
        const float x = static_cast<float>(k[i].x), yy = static_cast<float>(k[i].y);
        const float z = static_cast<float>(k[i].z);
        const float p2 = x * x + yy * yy;
        const float big = __builtin_sqrtf(p2 + z * z) + fabsf(z);
        // eta = sign(z) ln(big^2 / pT^2) / 2, through the hardware log2
        eta[i] = copysignf(ln2_half * __builtin_amdgcn_logf(big * big * __builtin_amdgcn_rcpf(p2)), z) +
                 static_cast<float>(y);
        // phi by octant reduction and atan on [0, 1]
        const float ax = fabsf(x), ay = fabsf(yy);
        const bool swap = ay > ax;
        const float t = (swap ? ax : ay) * __builtin_amdgcn_rcpf(swap ? ay : ax);
        float a = fm::atan_unit_f(t);
        a = swap ? half_pi - a : a;
        a = x < 0.0f ? pi - a : a;
        phi[i] = copysignf(a, yy);
        if (eta_max > 0.0) {
            const float d = fabsf(eta[i]) - static_cast<float>(eta_max);
            ok = ok && (d < 0.0f);
            unsure = unsure || (fabsf(d) < kEtaScreen);
        }
    }
    if (dr_min > 0.0) {
        const float dr2 = static_cast<float>(dr_min * dr_min);
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = i + 1; j < N; ++j) {
                const float de = eta[i] - eta[j];
                float dp = fabsf(phi[i] - phi[j]);
                dp = dp > pi ? 2.0f * pi - dp : dp;
                const float d = de * de + dp * dp - dr2;
                ok = ok && (d > 0.0f);
                unsure = unsure || (fabsf(d) < kDr2Screen);
            }
    }
    return unsure ? -1 : (ok ? 1 : 0);
}

// The cut decision: the FP32 screen, and the FP64 evaluation only for points
// the screen leaves open.
template <int N>
__device__ __forceinline__ bool pass_cuts(const Vec4 (&k)[N], double y, double pt_min,
                                          double eta_max, double dr_min)
{
    const int s = screen_cuts<N>(k, y, pt_min, eta_max, dr_min);
    if (s >= 0) return s == 1;
    return pass_cuts_fp64<N>(k, y, pt_min, eta_max, dr_min);
}

// Kinematic parameters shared by every point of one generation call.
struct GenParams {
    int mode;            // heget_mode
    uint64_t seed;
    int64_t first;       // index of the first point
    int64_t npoints;
    double sqrt_s;       // FIXED: sqrt(shat); PP: hadronic sqrt(s)
    double lo, hi;       // UNIFORM range / PP: min sqrt(shat)
    double pt_min, eta_max, dr_min;
    // eq. (2) without |M|^2, as c * shat^(n-3): 1/(2 shat) 1/4 1/9 3 1/n! Phi_n (hbar c)^2,
    // with Phi_n = phase_volume_coef * shat^(n-2)
    double partonic_coef;
    double phase_volume_coef;
    int weight_kind;     // 0: write Phi_n (or 0 if cut); 1: write the full non-|M|^2 weight
    unsigned *clear_word;  // if set, zeroed by the generation launch (the call's status flags)
    uint16_t *hel_out;     // if set, the sampled helicity configuration of every point
};

// Helicity configuration drawn for `point` in sampling mode (the paper's
// per-event helicities, Section 3.1): the low n + 1 bits of word 0 of the
// generator at block 0 of stream 2.  Bit 0 picks the quark pair (0: h_u = -1,
// h_ubar = +1, the pair the amplitude kernel evaluates; 1: its parity image),
// bit 1 + j the helicity of photon j (1: +1).
__device__ __forceinline__ uint32_t draw_helicity_raw(uint64_t seed, uint64_t point, int n)
{
    const Words4 r = philox4x32_10(static_cast<uint32_t>(point), static_cast<uint32_t>(point >> 32),
                                   0u, 2u, static_cast<uint32_t>(seed),
                                   static_cast<uint32_t>(seed >> 32));
    return r.w0 & ((2u << n) - 1u);
}

// The same draw in the amplitude kernel's convention: photon bits of the
// evaluated pair, flipped for the parity image (|M(-h, -lam)| = |M(h, lam)|).
template <int N>
__device__ __forceinline__ uint16_t draw_helicity(uint64_t seed, uint64_t point)
{
    const uint32_t raw = draw_helicity_raw(seed, point, N);
    const uint32_t mask = (1u << N) - 1u;
    const uint32_t lam = (raw >> 1) & mask;
    return static_cast<uint16_t>((raw & 1u) ? (~lam & mask) : lam);
}

struct PointKin {
    double sqrt_shat;
    double y;      // rapidity of the partonic CM frame in the lab
    double fpdf;   // parton-density importance weight times beam-assignment factor
    bool above;    // PP: sqrt(shat) >= lo
};

// Partonic kinematics of point `point` (stream 1 of the generator) in mode
// MODE (heget_mode: 0 fixed, 1 uniform, 2 proton-proton).
template <int MODE>
__device__ __forceinline__ PointKin point_kinematics(const GenParams &g, uint64_t point)
{
    PointKin pk{g.sqrt_s, 0.0, 1.0, true};
    if constexpr (MODE == 1) {
        double r0, r1;
        uniform_pair(g.seed, point, 1u, 1u, r0, r1);
        pk.sqrt_shat = g.lo + (g.hi - g.lo) * r0;
    } else if constexpr (MODE == 2) {
        // x = r^(1/a) samples a x^(a-1); the weight D(x) / (a x^(a-1)) keeps
        // only the smooth (1-x)^b factor: a = 0.5 for u, 0.7 for ubar.
        double r0, r1;
        uniform_pair(g.seed, point, 0u, 1u, r0, r1);
        const double xu = r0 * r0;
        const double xub = pow(r1, 1.0 / 0.7);
        const double omu = 1.0 - xu, omub = 1.0 - xub;
        const double f = (omu * omu * omu / 0.5) * ((omub * omub) * (omub * omub) * (omub * omub) / 0.7);
        const double shat = xu * xub * g.sqrt_s * g.sqrt_s;
        pk.sqrt_shat = sqrt(shat);
        pk.above = pk.sqrt_shat >= g.lo;
        if (!pk.above) pk.sqrt_shat = g.lo;  // keep the generator finite; weight is 0
        // both beam assignments of eq. (1): the second is the first rotated by
        // pi about x with y -> -y, which leaves |M|^2 and every cut unchanged
        pk.fpdf = 2.0 * f;
        pk.y = 0.5 * log(xu / xub);
    }
    return pk;
}

__device__ __forceinline__ double ipow(double x, int e)
{
    double r = 1.0;
    if (e >= 0) {
        for (int i = 0; i < e; ++i) r *= x;
    } else {
        for (int i = 0; i < -e; ++i) r /= x;
    }
    return r;
}

}  // namespace heget
