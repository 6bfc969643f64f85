"""The FP64 elementary functions of the generation kernels (csrc/fastmath.hpp)
against the C library's long-double versions, on the CPU: the header is
compiled for the host with g++ and evaluated on many arguments from the
ranges generation uses (and wider).  Bound: a few units in the last place."""
from __future__ import annotations

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0908_4403_amd", "csrc")

HARNESS = r"""
#define __host__
#define __device__
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <random>
#include "fastmath.hpp"

static double ulp_err(double got, long double ref) {
    if (ref == 0) return got == 0 ? 0.0 : 1e300;
    int e; std::frexp((double)ref, &e);
    long double ulp = std::ldexp(1.0L, e - 53);
    return (double)(std::fabs((long double)got - ref) / ulp);
}

int main() {
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    double worst_log = 0, worst_sin = 0, worst_cos = 0, worst_atan = 0;
    for (int i = 0; i < 2000000; ++i) {
        // log: products of two uniforms (RAMBO), ratios >= 1, wide exponents
        double x;
        switch (i % 3) {
        case 0: x = (u01(rng) + 0x1p-54) * (u01(rng) + 0x1p-54); break;
        case 1: x = 1.0 + 1e6 * u01(rng); break;
        default: x = std::ldexp(0.5 + u01(rng), (int)(u01(rng) * 240) - 120); break;
        }
        double r = heget::fm::log(x);
        long double ref = std::log((long double)x);
        if (x != 1.0) worst_log = std::fmax(worst_log, ulp_err(r, ref));
        // sincospi on (0, 2) (RAMBO azimuth 2 pi u) and on [-8, 8]
        double t = (i & 1) ? 2.0 * u01(rng) : 16.0 * u01(rng) - 8.0;
        double s, c;
        heget::fm::sincospi(t, &s, &c);
        // reference: reduce t exactly to the nearest multiple of 1/2 (the
        // identities sin(pi(m/2 + r)) = +-sin or +-cos(pi r) are exact), then
        // the long-double sine/cosine of pi r, accurate relative to its value
        const long double pi = 3.141592653589793238462643383279502884L;
        long double tt = (long double)t;
        long double m = std::nearbyint(2.0L * tt);
        long double rr = tt - m / 2.0L;
        long double s0 = std::sin(pi * rr), c0 = std::cos(pi * rr);
        long long mq = ((long long)m % 4 + 4) % 4;
        long double rs = mq == 0 ? s0 : mq == 1 ? c0 : mq == 2 ? -s0 : -c0;
        long double rc = mq == 0 ? c0 : mq == 1 ? -s0 : mq == 2 ? -c0 : s0;
        worst_sin = std::fmax(worst_sin, ulp_err(s, rs));
        worst_cos = std::fmax(worst_cos, ulp_err(c, rc));
        // atan2 over all quadrants and magnitude ratios
        double ax = std::ldexp(u01(rng) + 1e-3, (int)(u01(rng) * 20) - 10);
        double ay = std::ldexp(u01(rng) + 1e-3, (int)(u01(rng) * 20) - 10);
        double xs = (i & 2) ? -ax : ax, ys = (i & 4) ? -ay : ay;
        double a = heget::fm::atan2(ys, xs);
        long double ra = std::atan2((long double)ys, (long double)xs);
        worst_atan = std::fmax(worst_atan, ulp_err(a, ra));
    }
    // special values
    int bad = 0;
    bad += !(std::isinf(heget::fm::log(0.0)) && heget::fm::log(0.0) < 0);
    bad += !std::isinf(heget::fm::log(INFINITY));
    bad += !std::isnan(heget::fm::log(NAN));
    bad += heget::fm::log(1.0) != 0.0;
    double s0, c0;
    heget::fm::sincospi(0.0, &s0, &c0);
    bad += !(s0 == 0.0 && c0 == 1.0);
    heget::fm::sincospi(0.5, &s0, &c0);
    bad += !(s0 == 1.0 && c0 == 0.0);
    bad += heget::fm::atan2(0.0, 1.0) != 0.0;
    bad += std::fabs(heget::fm::atan2(1.0, 0.0) - 1.5707963267948966) > 0;
    bad += std::fabs(heget::fm::atan2(0.0, -1.0) - 3.141592653589793) > 0;
    bad += std::fabs(heget::fm::atan2(-0.0, -1.0) + 3.141592653589793) > 0;
    // FP32 atan on [0, 1] of the cut screen: absolute error in radians
    double worst_atanf = 0;
    for (int i = 0; i <= 1000000; ++i) {
        const float t = (float)(i * 1e-6);
        worst_atanf = std::fmax(worst_atanf, std::fabs((double)heget::fm::atan_unit_f(t) - std::atan((double)t)));
    }
    std::printf("%.3f %.3f %.3f %.3f %d %.3e\n", worst_log, worst_sin, worst_cos, worst_atan, bad, worst_atanf);
    return 0;
}
"""


@pytest.fixture(scope="module")
def errors(tmp_path_factory):
    d = tmp_path_factory.mktemp("fm")
    src = d / "fm.cpp"
    src.write_text(HARNESS)
    exe = d / "fm"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    return [float(v) for v in out[:4]] + [int(out[4]), float(out[5])]


def test_log_within_a_few_ulp(errors):
    assert errors[0] <= 2.0, errors


def test_sincospi_within_a_few_ulp(errors):
    assert errors[1] <= 2.0 and errors[2] <= 2.0, errors


def test_atan2_within_a_few_ulp(errors):
    assert errors[3] <= 2.0, errors


def test_special_values(errors):
    assert errors[4] == 0, errors


def test_fp32_atan_of_the_cut_screen(errors):
    """The screen assumes phi within a few 1e-7 rad: the polynomial (2e-8) plus
    FP32 rounding."""
    assert errors[5] <= 3e-7, errors
