"""The C-ABI library loads, exports every function include/heget.h declares,
and rejects bad arguments on the host before touching a GPU."""
from __future__ import annotations

import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "heget.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(heget_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_three_calls():
    names = declared_functions()
    for f in ("heget_gen_points", "heget_me2", "heget_xsec"):
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_0908_4403_amd as H
    out = subprocess.run(["nm", "-D", "--defined-only", H.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    assert set(H.EXPORTS) == set(declared_functions())


def test_no_cpu_fallback_in_binding():
    """The binding never imports the oracle; every result comes from libheget."""
    src = open(os.path.join(ROOT, "paper_0908_4403_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("no CPU fallback", "")


def test_argument_checks_run_on_the_host():
    import paper_0908_4403_amd as H
    with pytest.raises(H.HegetError) as e:
        H.me2(np.zeros((2, 11, 4)))  # n = 9
    assert e.value.status == H.ERR_RANGE
    with pytest.raises(H.HegetError) as e:
        H.me2(np.zeros((2, 3, 4)))  # n = 1
    assert e.value.status == H.ERR_RANGE
    with pytest.raises(H.HegetError) as e:
        H.me2(np.zeros((2, 6, 4)), prec=7)
    assert e.value.status == H.ERR_ARG
    for bad in (H.Config(npoints=-1), H.Config(npoints=1 << 31)):
        with pytest.raises(H.HegetError) as e:
            H.xsec(4, bad)
        assert e.value.status == H.ERR_RANGE
    for bad in (H.Config(sqrt_s=-1.0), H.Config(mode=7), H.Config(prec=3),
                H.Config(helicity_sampling=2),
                H.Config(mode=H.UNIFORM_SQRTSHAT, sqrt_shat_lo=500.0, sqrt_shat_hi=200.0),
                H.Config(mode=H.PP_TOY, sqrt_s=100.0, sqrt_shat_lo=150.0),
                H.Config(pt_min=float("nan")), H.Config(alpha=0.0)):
        with pytest.raises(H.HegetError) as e:
            H.xsec(4, bad)
        assert e.value.status == H.ERR_ARG, bad
    with pytest.raises(H.HegetError) as e:
        H.xsec_batch([3], [H.Config(helicity_sampling=1)])
    assert e.value.status == H.ERR_ARG
    for args, status in (((7, 10, 0.0, 1.0), H.ERR_ARG), ((H.OBS_PT_MAX, 0, 0.0, 1.0), H.ERR_RANGE),
                         ((H.OBS_PT_MAX, 5000, 0.0, 1.0), H.ERR_RANGE),
                         ((H.OBS_DR_MIN, 10, 1.0, 1.0), H.ERR_ARG)):
        with pytest.raises(H.HegetError) as e:
            H.xsec_hist(4, H.Config(), *args)
        assert e.value.status == status, args
    h, r = H.xsec_hist(4, H.Config(npoints=0), H.OBS_PT_MAX, 8, 0.0, 100.0)
    assert r["n_gen"] == 0 and not h.any()
    with pytest.raises(H.HegetError) as e:  # helicities exist only when they are drawn
        H.xsec_events(4, H.Config(npoints=16), helicity=True)
    assert e.value.status == H.ERR_ARG
    ev = H.xsec_events(4, H.Config(npoints=0), momenta=True, rapidity=True)
    assert ev["result"]["n_gen"] == 0 and ev["momenta"].shape == (0, 6, 4)
    with pytest.raises(H.HegetError):
        H.gen_points(3, float("inf"))
    with pytest.raises(H.HegetError):
        H.set_couplings(-1.0, 2 / 3)
    assert H.me2_flops(4, H.FP32)[0] > 0
    with pytest.raises(H.HegetError):
        H.me2_flops(1, H.FP32)


def test_empty_calls_need_no_device():
    import paper_0908_4403_amd as H
    assert H.me2(np.zeros((0, 6, 4))).shape == (0,)
    assert H.xsec(4, H.Config(npoints=0))["n_gen"] == 0
    assert H.helas("fvoxx0", np.zeros((0, 26))).shape == (0, 12)
    assert H.me2_frame(np.zeros((0, 7, 4))).shape == (0,)


def test_helas_record_sizes_and_host_checks():
    import paper_0908_4403_amd as H
    sizes = [H.helas_sizes(f) for f in H.HELAS_FUNCS]
    assert sizes == [(6, 12)] * 9 + [(38, 2), (26, 12), (26, 12), (26, 12)]
    with pytest.raises(H.HegetError) as e:
        H.helas_sizes(13)
    assert e.value.status == H.ERR_ARG
    with pytest.raises(ValueError):
        H.helas("ixxxx0", np.zeros((3, 5)))
    bad = np.array([[10.0, 0, 0, 10.0, 2.0, 1.0]])  # nHEL = 2
    with pytest.raises(H.HegetError) as e:
        H.helas("ixxxx0", bad)
    assert e.value.status == H.ERR_ARG
    bad[0, 4], bad[0, 5] = 1.0, 0.0                  # nSF = 0
    with pytest.raises(H.HegetError):
        H.helas("ixxxx0", bad)
    with pytest.raises(H.HegetError) as e:
        H.me2_frame(np.zeros((2, 8, 4)))             # n = 6: beyond the frame evaluator
    assert e.value.status == H.ERR_RANGE
    with pytest.raises(H.HegetError) as e:
        H.me2_frame(np.zeros((2, 3, 4)))             # n = 1
    assert e.value.status == H.ERR_RANGE


def _flops_unshared(n, mb, h, cl):
    """Closed form of the algorithmic count when no value is shared between the
    walk's helicities: every node, closing and pair vector h times (vertex
    blocks with a unit diagonal: a node update is 14 + 36 per helicity)."""
    import math
    f = math.factorial
    ns = min(n, mb)
    if cl >= 3 and ns < 4:  # no four-photon subtree: closes as pairs
        cl = 2
    nodes = sum(f(n) // f(n - j) for j in range(1, n - cl + 1))
    subtrees = f(n) // f(ns)
    top = sum(f(n) // f(n - j) for j in range(1, n - ns + 1))
    walk = nodes * (14 + 36 * h) + (ns * subtrees + top) * 4 + 4 * h
    pairs = subtrees * (ns * (12 + 11 * h) + ns * (ns - 1) * 16 * h + ns * (ns - 1) // 2 * 4 * h)
    if cl >= 3 and ns >= 4:
        # the last four photons of every ordering: n!/4! nodes, each with four
        # single-photon updates and six splits (propagator, two vertex halves
        # and their sum, propagator half, pair closing)
        quads = f(n) // f(4)
        nodes = sum(f(n) // f(n - j) for j in range(1, n - 4 + 1))
        walk = nodes * (14 + 36 * h) + (ns * subtrees + top) * 4 + 4 * h
        walk += quads * (4 * (14 + 36 * h) + 6 * (14 + 56 * h + 16 * h))
        walk += pairs
    elif cl == 1:
        walk += f(n) * 10 * h
    else:
        walk += f(n) // 2 * 16 * h
        walk += pairs
    return walk * 2 ** n // h


def _flops_prefix_sets(n, mb, h, cl):
    """Closed form for the prefix-set walk (n > mb, nothing shared): per
    (n - mb)-subset of the photons its vertex blocks, the subset recursion over
    its subsets (momentum 14, per helicity a vertex half 16, 20 per further
    vertex half added, a propagator half 20), and the mb-photon subtree once."""
    import math
    k = n - mb
    subtree = _flops_unshared(mb, mb, h, cl) * h // 2 ** mb - 4 * h
    bg = sum(math.comb(k, m) * (14 + (16 + 20 * (m - 1) + 20) * h) for m in range(1, k + 1))
    walk = math.comb(n, k) * (4 * k + bg + subtree) + 4 * h
    return walk * 2 ** n // h


def _flops_meet(n, h, ps):
    """Closed form for meeting in the middle with nothing shared (h = 1): with
    K = (n + 1) / 2, the v-bar-end subset currents of every set of 1 .. K - 1
    photons, the u-end ones of every set of 1 .. n - K - 1, and per set of K
    photons its current, the row vector of the other n - K photons and one
    contraction.  A node of m photons: momentum 14 (once per point for ps = 2,
    once per walk otherwise); per helicity 11 for one photon, else
    36 + 20 (m - 1).  Row vector: 16 + 20 (n - K - 1) per helicity;
    contraction 16 per helicity; vertex blocks 4 per photon."""
    import math
    K = (n + 1) // 2
    ku = n - K
    walks = 2 ** n // h

    def per(m):
        return (11 if m == 1 else 36 + 20 * (m - 1)) * h

    sizes = list(range(1, K)) + list(range(1, ku)) + [K]
    walk = 4 * n + 4 * h + sum(math.comb(n, m) * per(m) for m in sizes)
    walk += math.comb(n, K) * ((16 + 20 * (ku - 1)) * h + 16 * h)
    momenta = sum(math.comb(n, m) * 14 for m in sizes)
    return walk * walks + momenta * (1 if ps == 2 else walks)


def test_flop_count_of_every_shape():
    """heget_me2_flops equals the closed form where nothing is shared (h = 1, or
    photons in run-time slots), and is below it where helicities share values."""
    import paper_0908_4403_amd as H
    for n in range(2, 9):
        for prec in (H.FP32, H.FP64):
            try:
                for shape in H.kernel_shapes(n, prec):
                    H.set_kernel_shape(n, prec, shape)
                    f, got = H.me2_flops(n, prec)
                    assert got == shape
                    mb, h, cl, wpb, pf, wpe, ppl, ps = shape
                    if ps >= 2:
                        assert mb == n, (n, shape)
                        ref = _flops_meet(n, h, ps)
                        assert (f == ref) if h == 1 else (0.25 * ref < f < ref), (n, shape, f, ref)
                        continue
                    if ps == 1 and n - mb >= 2:
                        assert f == _flops_prefix_sets(n, mb, h, cl), (n, shape, f)
                        continue
                    ref = _flops_unshared(n, mb, h, cl)
                    if h == 1 or n > mb:
                        assert f == ref, (n, shape, f, ref)
                    else:
                        assert 0.25 * ref < f < ref, (n, shape, f, ref)
            finally:
                H.set_kernel_shape(n, prec, None)


class _NoLib:
    """Stands in for the library: any call reaching it fails the test."""

    def __getattr__(self, name):
        raise AssertionError(f"{name} was called although the binding should have refused")


def test_device_calls_check_buffers_before_the_library(monkeypatch):
    """Wrong dtypes, short or host result buffers are refused by the binding,
    before a pointer reaches the library (a float32 buffer would be written
    past its end by the FP64 kernels)."""
    import torch
    import paper_0908_4403_amd as H
    monkeypatch.setattr(H, "_lib", _NoLib())
    n, N = 4, 64
    for mom, w in ((torch.zeros((n + 2) * 4, N, dtype=torch.float32), torch.zeros(N, dtype=torch.float64)),
                   (torch.zeros((n + 2) * 4, N, dtype=torch.float64), torch.zeros(N, dtype=torch.float32))):
        with pytest.raises(TypeError):
            H.gen_points_device(n, 1000.0, mom, w)
        with pytest.raises(TypeError):
            H.me2_device(n, mom, w)
        with pytest.raises(TypeError):
            H.me2_async(n, mom, w)
    f64 = dict(dtype=torch.float64)
    with pytest.raises(ValueError):  # host tensors: not device memory
        H.gen_points_device(n, 1000.0, torch.zeros((n + 2) * 4, N, **f64), torch.zeros(N, **f64))
    with pytest.raises(ValueError):  # shorter than one result record
        H.xsec_device(n, H.Config(), torch.zeros(6, **f64))
    with pytest.raises(ValueError):  # pageable host memory: the device cannot write it
        H.xsec_device(n, H.Config(), torch.zeros(7, **f64))
    with pytest.raises(ValueError):  # not contiguous
        H.xsec_device(n, H.Config(), torch.zeros(14, **f64)[::2])


def test_me2_async_is_the_device_form():
    import paper_0908_4403_amd as H
    names = declared_functions()
    assert "heget_me2_async" in names and "heget_me2_device" in names
    assert H.lib().heget_me2_async(9, 1, None, None, 0, None) == H.ERR_RANGE
    assert H.lib().heget_me2_async(4, 1, None, None, 0, None) == H.ERR_ARG
    assert H.lib().heget_me2_async(4, 0, None, None, 0, None) == H.OK


def test_golden_writer_imports_only_the_oracle():
    """Stored expected values come from oracle/ alone: the writer never imports
    the product package, and the workload table it shares is plain data."""
    src = open(os.path.join(ROOT, "tests", "golden", "make_golden.py")).read()
    assert "paper_0908_4403_amd" not in src
    wl = open(os.path.join(ROOT, "workloads.py")).read()
    assert not re.search(r"^\s*(import|from)\s", wl, flags=re.M)
