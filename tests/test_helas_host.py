"""The HELAS device header (csrc/helas.hpp) compiled for the host with g++ and
compared with the FP64 oracle on the CPU, for every function in FP64 and
FP32: a check of the library's algebra that needs no GPU (the GPU tests
repeat it on the device).  Bounds as in the GPU tests: FP64 within 1e-12 of
the record's scale; FP32 within 16 times the oracle's own sensitivity to one
FP32 rounding of every input (or one rounding of the scale)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0908_4403_amd", "csrc")
FUNCS = ["ixxxx0", "ixxxx1", "ixxxx2", "oxxxx0", "oxxxx1", "oxxxx2", "vxxxx0", "vxxxx1", "vxxxx2",
         "iovxxx", "fvixx0", "fvoxx0", "jioxx0"]
NI = [6] * 9 + [38, 26, 26, 26]
NO = [12] * 9 + [2, 12, 12, 12]
EPS32 = 2.0 ** -24

HARNESS = r"""
#define __host__
#define __device__
#include <cstdint>
#include "helas.hpp"
using namespace heget::helas;

template <typename R> static Wave<R> load(const double *x)
{
    Wave<R> w;
    for (int m = 0; m < 4; ++m) w.c[m] = cx(R(x[2 * m]), R(x[2 * m + 1]));
    for (int m = 0; m < 4; ++m) w.p[m] = R(x[8 + m]);
    return w;
}
template <typename R> static void store(const Wave<R> &w, double *y)
{
    for (int m = 0; m < 4; ++m) { y[2 * m] = w.c[m].re; y[2 * m + 1] = w.c[m].im; }
    for (int m = 0; m < 4; ++m) y[8 + m] = w.p[m];
}
template <typename R> static void one(int f, const double *x, double *y)
{
    if (f <= 8) {
        const R p[4] = {R(x[0]), R(x[1]), R(x[2]), R(x[3])};
        const int h = int(x[4]), s = int(x[5]);
        Wave<R> w;
        switch (f) {
        case 0: w = ixxxx0(p, h, s); break;
        case 1: w = ixxxx1(p, h, s); break;
        case 2: w = ixxxx2(p, h, s); break;
        case 3: w = oxxxx0(p, h, s); break;
        case 4: w = oxxxx1(p, h, s); break;
        case 5: w = oxxxx2(p, h, s); break;
        case 6: w = vxxxx0(p, h, s); break;
        case 7: w = vxxxx1(p, h); break;
        default: w = vxxxx2(p, h); break;
        }
        store(w, y);
    } else if (f == 9) {
        const Cx<R> v = iovxxx(load<R>(x), load<R>(x + 12), load<R>(x + 24), R(x[36]), R(x[37]));
        y[0] = v.re;
        y[1] = v.im;
    } else {
        const Wave<R> a = load<R>(x), b = load<R>(x + 12);
        const R g0 = R(x[24]), g1 = R(x[25]);
        store(f == 10 ? fvixx0(a, b, g0, g1) : f == 11 ? fvoxx0(a, b, g0, g1) : jioxx0(a, b, g0, g1), y);
    }
}
extern "C" void eval(int f, int fp32, long n, const double *x, double *y, int ni, int no)
{
    for (long i = 0; i < n; ++i) {
        if (fp32) one<float>(f, x + i * ni, y + i * no);
        else one<double>(f, x + i * ni, y + i * no);
    }
}
"""


@pytest.fixture(scope="module")
def host_lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("helas")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    so = d / "h.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC", "-I", CSRC,
                    str(src), "-o", str(so)], check=True)
    return C.CDLL(str(so))


def _eval(lib, f, x, fp32):
    y = np.zeros((len(x), NO[f]))
    dp = C.POINTER(C.c_double)
    x = np.ascontiguousarray(x)
    lib.eval(f, int(fp32), C.c_long(len(x)), x.ctypes.data_as(dp), y.ctypes.data_as(dp), NI[f], NO[f])
    return y


def _records(orc, f, rng, count):
    def massless(direction=None):
        d = rng.normal(size=3) if direction is None else np.asarray(direction, float)
        d = d / np.linalg.norm(d)
        e = rng.uniform(1.0, 2000.0)
        return np.concatenate([[e], e * d])

    special = [(0, 0, 1), (0, 0, -1), (1e-7, 2e-7, -1), (3e-6, -1e-6, 1), (1e-4, 0, -1)]
    out = []
    for k in range(count):
        if f <= 8:
            d = (0, 0, 1) if f in (1, 4, 7) else (0, 0, -1) if f in (2, 5, 8) else \
                (special[(k // 8) % 5] if k % 8 == 0 else None)
            out.append(np.concatenate([massless(d), [rng.choice([-1.0, 1.0]), rng.choice([-1.0, 1.0])]]))
        else:
            w = lambda: np.concatenate([rng.normal(size=8), rng.normal(size=4) * 50])
            parts = [w(), w(), w()] if f == 9 else [w(), w()]
            out.append(np.concatenate(parts + [rng.normal(size=2)]))
    return np.array(out)


@pytest.mark.parametrize("func", FUNCS)
def test_header_matches_oracle_fp64(orc, host_lib, func):
    f = FUNCS.index(func)
    rng = np.random.default_rng(100 + f)
    x = _records(orc, f, rng, 400)
    want = np.array([orc.helas(func, r) for r in x])
    got = _eval(host_lib, f, x, False)
    k = 8 if NO[f] == 12 else 2
    scale = np.abs(want[:, :k]).max(axis=1)
    assert (np.abs(got - want)[:, :k].max(axis=1) / scale).max() <= 1e-12
    if NO[f] == 12:
        assert np.array_equal(got[:, 8:], want[:, 8:])


@pytest.mark.parametrize("func", FUNCS)
def test_header_fp32_within_its_condition(orc, host_lib, func):
    f = FUNCS.index(func)
    rng = np.random.default_rng(200 + f)
    x = _records(orc, f, rng, 400).astype(np.float32).astype(np.float64)
    want = np.array([orc.helas(func, r) for r in x])
    k = 8 if NO[f] == 12 else 2
    real = np.ones(x.shape[1], bool)
    if f <= 8:
        real[4:6] = False
    sens = np.zeros(len(x))
    for _ in range(4):
        xp = x.copy()
        xp[:, real] *= 1 + EPS32 * rng.uniform(-1, 1, size=(len(x), int(real.sum())))
        sens = np.maximum(sens, np.abs(np.array([orc.helas(func, r) for r in xp]) - want)[:, :k].max(axis=1))
    got = _eval(host_lib, f, x, True)
    scale = np.abs(want[:, :k]).max(axis=1)
    ratio = np.abs(got - want)[:, :k].max(axis=1) / np.maximum(sens, EPS32 * scale)
    assert ratio.max() <= 16.0, ratio.max()
