// FP64 elementary functions for phase-space generation.  Each one makes one
// argument reduction and sums one Taylor series whose truncation error on
// the reduced range is below 2^-55 relative, so results are within a few
// units in the last place of the exact value; they are shorter than the
// general-purpose library versions because they need no special-case paths
// beyond the domain used here.  Written for host and device so that a CPU
// test can compare them with the C library on many arguments.
#pragma once
#include <math.h>

namespace heget {
namespace fm {

// ln 2 split so that e * kLn2Hi is exact for |e| < 2^21.
constexpr double kLn2Hi = 0.6931471803691238;
constexpr double kLn2Lo = 1.9082149292705877e-10;
constexpr double kInvSqrt2 = 0.70710678118654752;

// Natural logarithm for x > 0 (0 -> -inf, +inf and NaN pass through).
// x = 2^e m with m in [1/sqrt 2, sqrt 2); log m = 2 atanh(s), s = (m-1)/(m+1),
// |s| <= 0.1716, and atanh(s)/s = sum_k s^(2k)/(2k+1) through k = 10
// (Cody and Waite, Software Manual for the Elementary Functions, 1980).
__host__ __device__ inline double log(double x)
{
    int e = 0;
    double m = frexp(x, &e);  // m in [1/2, 1)
    if (m < kInvSqrt2) {
        m *= 2.0;
        --e;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double lm = fma(2.0 * s * z, p, 2.0 * s);  // 2 s (1 + z p)
    const double ed = static_cast<double>(e);
    const double r = fma(ed, kLn2Hi, fma(ed, kLn2Lo, lm));
    if (x == 0.0) return -INFINITY;
    return x < INFINITY ? r : x;
}

// sin(pi t) and cos(pi t) for finite t.  pi t = k pi/2 + pi r with
// k = rint(2t) and r = t - k/2 in [-1/4, 1/4] (exact); sin(pi r) through
// (pi r)^17 and cos(pi r) through (pi r)^18, then the quadrant k mod 4.
// Coefficients: (-1)^k pi^(2k+1)/(2k+1)! and (-1)^k pi^(2k)/(2k)!, rounded.
__host__ __device__ inline void sincospi(double t, double *sp, double *cp)
{
    const double k = rint(2.0 * t);
    const double r = fma(-0.5, k, t);
    const double z = r * r;
    double ps = 7.952054001475513e-07;
    ps = fma(ps, z, -2.1915353447830217e-05);
    ps = fma(ps, z, 0.00046630280576761255);
    ps = fma(ps, z, -0.0073704309457143504);
    ps = fma(ps, z, 0.08214588661112823);
    ps = fma(ps, z, -0.5992645293207921);
    ps = fma(ps, z, 2.5501640398773455);
    ps = fma(ps, z, -5.16771278004997);
    const double s = fma(r * z, ps, 3.141592653589793 * r);
    double pc = -1.3878952462213771e-07;
    pc = fma(pc, z, 4.303069587032947e-06);
    pc = fma(pc, z, -0.0001046381049248457);
    pc = fma(pc, z, 0.0019295743094039231);
    pc = fma(pc, z, -0.02580689139001406);
    pc = fma(pc, z, 0.2353306303588932);
    pc = fma(pc, z, -1.3352627688545895);
    pc = fma(pc, z, 4.0587121264167685);
    pc = fma(pc, z, -4.934802200544679);
    const double c = fma(z, pc, 1.0);
    const long long q = static_cast<long long>(k) & 3;
    const double sa = (q & 1) ? c : s;  // sin of the quadrant-shifted angle up to sign
    const double ca = (q & 1) ? s : c;
    *sp = (q & 2) ? -sa : sa;
    *cp = (q == 1 || q == 2) ? -ca : ca;
}

// atan2(y, x) for finite (x, y), not both zero.  With a = min(|x|,|y|) and
// b = max(|x|,|y|), t = a/b in [0, 1] lies within 1/8 of c = j/4 (j chosen
// by comparing a with b/8, 3b/8, 5b/8, 7b/8); atan t = atan c + atan t',
// t' = (a - c b)/(b + c a), |t'| <= 1/8, summed through t'^19; then the
// octant and quadrant fix-ups.  atan(j/4) and pi/2, pi as hi + lo pairs.
__host__ __device__ inline double atan2(double y, double x)
{
    const double ax = fabs(x), ay = fabs(y);
    const bool swap = ay > ax;
    const double a = swap ? ax : ay, b = swap ? ay : ax;
    const int j = (a > 0.125 * b) + (a > 0.375 * b) + (a > 0.625 * b) + (a > 0.875 * b);
    const double c = 0.25 * j;
    const double tp = fma(-c, b, a) / fma(c, a, b);
    const double z = tp * tp;
    double p = -1.0 / 19.0;
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, -1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, -1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, -1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, -1.0 / 3.0);
    const double at = fma(tp * z, p, tp);
    const double hi = j == 0 ? 0.0
                    : j == 1 ? 0.24497866312686414
                    : j == 2 ? 0.4636476090008061
                    : j == 3 ? 0.6435011087932844
                             : 0.7853981633974483;
    const double lo = j == 0 ? 0.0
                    : j == 1 ? 1.0698755618734451e-17
                    : j == 2 ? 2.2698777452961687e-17
                    : j == 3 ? 1.5834785051444286e-17
                             : 3.061616997868383e-17;
    double ang = hi + (lo + at);                                          // in [0, pi/4]
    if (swap) ang = 1.5707963267948966 + (6.123233995736766e-17 - ang);  // pi/2 - ang
    if (x < 0.0) ang = 3.141592653589793 + (1.2246467991473532e-16 - ang);  // pi - ang
    return copysign(ang, y);
}

// atan(t) for t in [0, 1] in FP32, for screening cut decisions: the odd
// polynomial of Abramowitz and Stegun, Handbook of Mathematical Functions,
// 4.4.49 (Hastings), absolute error below 2e-8 in exact arithmetic.
__host__ __device__ inline float atan_unit_f(float t)
{
    const float z = t * t;
    float p = 0.0028662257f;
    p = fmaf(p, z, -0.0161657367f);
    p = fmaf(p, z, 0.0429096138f);
    p = fmaf(p, z, -0.0752896400f);
    p = fmaf(p, z, 0.1065626393f);
    p = fmaf(p, z, -0.1420889944f);
    p = fmaf(p, z, 0.1999355085f);
    p = fmaf(p, z, -0.3333314528f);
    return fmaf(t * z, p, t);
}

}  // namespace fm
}  // namespace heget
