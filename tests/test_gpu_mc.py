"""GPU parity of the Monte-Carlo side: phase-space generation (Philox +
RAMBO + cuts) against the oracle's generator on the same counters, and the
cross section against the oracle's on the same sample.

Floating point decides an integer here (the cut decision); both sides take it
in FP64, and a mismatch is only accepted for a point whose cut variables lie
within 1e-9 (relative) of a bound.  sigma: same sample, <= 1e-5 relative
(FP64 amplitudes: <= 1e-10).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0908_4403_amd as H
    return H


def near_cut(k, pt_min, eta_max, dr_min, tol=1e-9):
    pt = np.hypot(k[:, 1], k[:, 2])
    pabs = np.sqrt(pt ** 2 + k[:, 3] ** 2)
    eta = np.arctanh(k[:, 3] / pabs)
    phi = np.arctan2(k[:, 2], k[:, 1])
    if np.any(np.abs(pt / pt_min - 1) < tol) or np.any(np.abs(np.abs(eta) / eta_max - 1) < tol):
        return True
    n = k.shape[0]
    for i in range(n):
        for j in range(i + 1, n):
            dphi = abs(phi[i] - phi[j])
            dphi = 2 * math.pi - dphi if dphi > math.pi else dphi
            if abs(math.hypot(eta[i] - eta[j], dphi) / dr_min - 1) < tol:
                return True
    return False


@pytest.mark.parametrize("n,sqrt_s,seed", [(2, 500.0, 0), (4, 1000.0, 1), (8, 2000.0, 4)])
def test_gen_points_match_oracle(H, orc, n, sqrt_s, seed):
    N = 3000 + 17
    mom, w = H.gen_points(n, sqrt_s, (20.0, 2.5, 0.4), seed, N)
    ref = orc.cm_events(n, sqrt_s, seed, 0, N)
    assert np.allclose(mom, ref, rtol=0, atol=1e-12 * sqrt_s)
    vol = orc.rambo_weight(n, sqrt_s ** 2)
    mismatches = 0
    for i in range(N):
        acc = orc.pass_cuts(ref[i, 2:], 0.0, 20.0, 2.5, 0.4)
        if (w[i] > 0) != acc:
            assert near_cut(ref[i, 2:], 20.0, 2.5, 0.4), i
            mismatches += 1
        elif acc:
            assert w[i] == pytest.approx(vol, rel=1e-13)
    assert mismatches <= 1


@pytest.mark.parametrize("n", [2, 4, 8])
def test_gen_points_massless_and_conserving(H, n):
    """The device generator's photons are massless and balance the beams to
    rounding on many points, nearly collinear seeds included (the oracle's
    own pins bound the same defects)."""
    sqrt_s, N = 1000.0, 1 << 16
    mom, _ = H.gen_points(n, sqrt_s, None, 21, N)
    k = mom[:, 2:, :]
    e = k[..., 0]
    mass = np.abs(e ** 2 - (k[..., 1:] ** 2).sum(axis=-1)) / e ** 2
    tot = k.sum(axis=1) - np.array([sqrt_s, 0.0, 0.0, 0.0])
    print(f"n={n} max mass defect {mass.max():.1e}, max imbalance {np.abs(tot).max() / sqrt_s:.1e}",
          flush=True)
    assert mass.max() <= 4e-15
    assert np.abs(tot).max() <= 4e-15 * sqrt_s * n


def test_gen_points_device_offsets(H, orc):
    import torch
    n, N, first = 3, 1000, 12345
    mom = torch.empty(((n + 2) * 4, N), dtype=torch.float64, device="cuda")
    w = torch.empty(N, dtype=torch.float64, device="cuda")
    H.gen_points_device(n, 800.0, mom, w, (20.0, 2.5, 0.4), 9, first)
    torch.cuda.synchronize()
    got = mom.cpu().numpy().T.reshape(N, n + 2, 4)
    ref = orc.cm_events(n, 800.0, 9, first, N)
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * 800.0)


def _cfgs(H, orc, mode, **kw):
    return H.Config(mode=mode, **kw), orc.Config(mode=mode, **{k: v for k, v in kw.items() if k != "prec"})


@pytest.mark.parametrize("prec", ["FP64", "FP32"])
def test_xsec_config1_matches_oracle_and_closed_form(H, orc, prec):
    import pins
    kw = dict(seed=0, npoints=16384, sqrt_s=500.0, pt_min=20.0, eta_max=2.5, dr_min=0.0)
    hc, oc = _cfgs(H, orc, H.FIXED_SHAT, prec=getattr(H, prec), **kw)
    got = H.xsec(2, hc)
    want = orc.xsec(2, oc)
    assert got["n_gen"] == want["n_gen"] and got["n_acc"] == want["n_acc"]
    tol = 1e-10 if prec == "FP64" else 1e-5
    assert abs(got["sigma_fb"] / want["sigma_fb"] - 1) < tol
    assert abs(got["err_fb"] / want["err_fb"] - 1) < 1e-4
    closed = pins.sigma_hat_n2(500.0 ** 2, 1 / 137, 2 / 3, pins.cos_max_n2(500.0, 0.0, 20.0, 2.5))
    assert abs(got["sigma_fb"] - closed) < 3.5 * got["err_fb"]


@pytest.mark.parametrize("n,mode,extra,npoints", [
    (3, "FIXED_SHAT", dict(sqrt_s=1000.0), 3000),
    (4, "FIXED_SHAT", dict(sqrt_s=1000.0), 1200),
    (3, "UNIFORM_SQRTSHAT", dict(sqrt_shat_lo=200.0, sqrt_shat_hi=2000.0), 3000),
    (3, "PP_TOY", dict(sqrt_s=14000.0, sqrt_shat_lo=150.0), 6000),
    (5, "PP_TOY", dict(sqrt_s=14000.0, sqrt_shat_lo=150.0), 1500),
])
def test_xsec_matches_oracle_same_sample(H, orc, n, mode, extra, npoints):
    kw = dict(seed=3, npoints=npoints, pt_min=20.0, eta_max=2.5, dr_min=0.4, **extra)
    for prec, tol in (("FP64", 1e-10), ("FP32", 1e-5)):
        hc, oc = _cfgs(H, orc, getattr(H, mode), prec=getattr(H, prec), **kw)
        got = H.xsec(n, hc)
        want = orc.xsec(n, oc)
        print(mode, n, prec, got["sigma_fb"], want["sigma_fb"], got["n_acc"], flush=True)
        assert got["n_acc"] == want["n_acc"]
        assert abs(got["sigma_fb"] / want["sigma_fb"] - 1) < tol


@pytest.mark.parametrize("n", [2, 3])
def test_xsec_two_points_per_lane_shapes(H, orc, n):
    """The weighted pass of every two-points-per-lane shape (an odd number of
    64-point tiles, so the last work item holds one real tile and one past the
    end) against the oracle on the same sample."""
    kw = dict(seed=5, npoints=1300, pt_min=20.0, eta_max=2.5, dr_min=0.4, sqrt_s=700.0)  # 21, 19 tiles
    try:
        for prec, tol in (("FP64", 1e-10), ("FP32", 1e-5)):
            P = getattr(H, prec)
            shapes = [s for s in H.kernel_shapes(n, P) if s[6] == 2]
            assert shapes, (n, prec)
            hc, oc = _cfgs(H, orc, H.FIXED_SHAT, prec=P, **kw)
            want = orc.xsec(n, oc)
            for shape in shapes:
                H.set_kernel_shape(n, P, shape)
                got = H.xsec(n, hc)
                print(n, prec, shape, got["sigma_fb"], want["sigma_fb"], got["n_acc"], flush=True)
                assert got["n_acc"] == want["n_acc"] and (got["n_acc"] + 63) // 64 % 2 == 1
                assert abs(got["sigma_fb"] / want["sigma_fb"] - 1) < tol
    finally:
        H.set_kernel_shape(n, H.FP64)
        H.set_kernel_shape(n, H.FP32)


@pytest.mark.parametrize("npoints", [1, 255, 256, 257, 1023, 4097])
def test_compaction_edges_match_oracle(H, orc, npoints):
    """Survivor counts and sigma across block edges (256-point blocks, the
    offsets summed four counts per load plus a remainder), with cuts that
    keep some, none and all of the points."""
    for pt_min, eta_max, dr_min in ((20.0, 2.5, 0.4), (600.0, 2.5, 0.4), (0.0, 0.0, 0.0)):
        kw = dict(seed=21, npoints=npoints, sqrt_s=1000.0, pt_min=pt_min, eta_max=eta_max, dr_min=dr_min)
        hc, oc = _cfgs(H, orc, H.FIXED_SHAT, prec=H.FP64, **kw)
        got = H.xsec(3, hc)
        want = orc.xsec(3, oc)
        assert got["n_gen"] == npoints and got["n_acc"] == want["n_acc"], (pt_min, got, want)
        if want["n_acc"] == 0:
            assert got["sigma_fb"] == 0.0
        else:
            assert abs(got["sigma_fb"] / want["sigma_fb"] - 1) < 1e-10


@pytest.mark.parametrize("npoints", [(1 << 20) + 12345, 3 * 4096 * 256 + 1000])
def test_compaction_with_scanned_offsets_matches_oracle(H, orc, npoints):
    """Above 2^20 points the block counts are scanned by one workgroup in
    chunks of 4096 (here one partial chunk, and three full chunks plus a
    partial one): survivor count exact and sigma at the FP64 bar, with cuts
    that keep most, some and none of the points."""
    for pt_min in (20.0, 200.0, 300.0):
        kw = dict(seed=23, npoints=npoints, sqrt_s=500.0, pt_min=pt_min, eta_max=2.5, dr_min=0.0)
        hc, oc = _cfgs(H, orc, H.FIXED_SHAT, prec=H.FP64, **kw)
        got = H.xsec(2, hc)
        want = orc.xsec(2, oc)
        print(npoints, pt_min, got["n_acc"], want["n_acc"], flush=True)
        assert got["n_gen"] == npoints and got["n_acc"] == want["n_acc"], (pt_min, got, want)
        if want["n_acc"] == 0:
            assert got["sigma_fb"] == 0.0
        else:
            assert abs(got["sigma_fb"] / want["sigma_fb"] - 1) < 1e-10


def test_xsec_deterministic_and_empty(H):
    cfg = H.Config(prec=H.FP32, seed=5, npoints=50000 + 3, sqrt_s=1000.0)
    a = H.xsec(4, cfg)
    b = H.xsec(4, cfg)
    assert a == b
    z = H.xsec(4, H.Config(prec=H.FP32, npoints=0, sqrt_s=1000.0))
    assert z["n_gen"] == 0 and z["sigma_fb"] == 0.0


def test_xsec_device_and_async_match_sync(H):
    import torch
    cfg = H.Config(prec=H.FP32, seed=8, npoints=20000 + 11, sqrt_s=1000.0)
    ref = H.xsec(4, cfg)
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    H.xsec_device(4, cfg, buf)
    h = H.XsecAsync(4, cfg)
    torch.cuda.synchronize()
    assert H.result_from_bytes(buf.cpu().numpy()) == ref
    assert h.result() == ref


def test_back_to_back_calls_match_one_by_one(H):
    """Five calls enqueued back to back on one stream (different seeds and
    sizes, sharing the stream's scratch) equal the same five made one at a
    time."""
    import torch
    cfgs = [H.Config(prec=H.FP32, seed=20 + k, npoints=30000 + 7919 * k, sqrt_s=1000.0)
            for k in range(5)]
    ref = [H.xsec(4, c) for c in cfgs]
    buf = torch.zeros((len(cfgs), 64), dtype=torch.uint8, device="cuda")
    for k, c in enumerate(cfgs):
        H.xsec_device(4, c, buf[k])
    torch.cuda.synchronize()
    host = buf.cpu().numpy()
    for k in range(len(cfgs)):
        assert H.result_from_bytes(host[k]) == ref[k], k


@pytest.mark.parametrize("n,mode,extra,npoints", [
    (2, "FIXED_SHAT", dict(sqrt_s=500.0, dr_min=0.0), 16384),
    (3, "FIXED_SHAT", dict(sqrt_s=1000.0), 3000),
    (4, "UNIFORM_SQRTSHAT", dict(sqrt_shat_lo=200.0, sqrt_shat_hi=2000.0), 2000),
    (5, "PP_TOY", dict(sqrt_s=14000.0, sqrt_shat_lo=150.0), 1500),
    (6, "FIXED_SHAT", dict(sqrt_s=1500.0), 300),
    (7, "FIXED_SHAT", dict(sqrt_s=1500.0), 200),
    (8, "FIXED_SHAT", dict(sqrt_s=2000.0), 64),
])
def test_helicity_sampling_matches_oracle_same_sample(H, orc, n, mode, extra, npoints):
    """One drawn helicity configuration per point (the paper's per-event
    helicities): same draws, same |M_h|^2 estimator, same sigma as the oracle."""
    kw = dict(seed=6, npoints=npoints, pt_min=20.0, eta_max=2.5, dr_min=0.4)
    kw.update(extra)
    for prec, tol in (("FP64", 1e-10), ("FP32", 1e-5)):
        hc, oc = _cfgs(H, orc, getattr(H, mode), prec=getattr(H, prec), helicity_sampling=1, **kw)
        got = H.xsec(n, hc)
        want = orc.xsec(n, oc)
        print(mode, n, prec, "sampled", got["sigma_fb"], want["sigma_fb"], got["n_acc"], flush=True)
        assert got["n_acc"] == want["n_acc"]
        assert abs(got["sigma_fb"] / want["sigma_fb"] - 1) < tol
        assert abs(got["err_fb"] / want["err_fb"] - 1) < 1e-4


def test_helicity_sampling_is_unbiased_on_the_device(H):
    """n = 4, 2^18 points: the sampled sigma agrees with the summed sigma of the
    same points within four combined standard errors."""
    kw = dict(prec=H.FP32, seed=12, npoints=1 << 18, sqrt_s=1000.0)
    s = H.xsec(4, H.Config(**kw))
    h = H.xsec(4, H.Config(helicity_sampling=1, **kw))
    assert h["n_acc"] == s["n_acc"]
    assert abs(h["sigma_fb"] - s["sigma_fb"]) < 4.0 * (h["err_fb"] ** 2 + s["err_fb"] ** 2) ** 0.5


@pytest.mark.parametrize("n,which,lo,hi,sampling", [
    (4, "PT_MAX", 20.0, 500.0, 0), (4, "DR_MIN", 0.4, 4.0, 0), (3, "PT_MAX", 20.0, 500.0, 1),
])
def test_histogram_matches_oracle_same_sample(H, orc, n, which, lo, hi, sampling):
    """Weighted distributions of Fig. 2's observables: per bin against the
    oracle's histogram of the same points (FP64 path: 1e-10 relative per bin
    with content; FP32: 1e-4 per bin, 1e-5 on the total), and the bins add up
    to the call's sigma."""
    kw = dict(seed=8, npoints=4000, sqrt_s=1000.0, pt_min=20.0, eta_max=2.5, dr_min=0.4)
    oc = orc.Config(mode=0, helicity_sampling=sampling, **kw)
    ref = orc.hist(n, oc, getattr(orc, which), 24, lo, hi)
    for prec, tol_bin, tol_tot in (("FP64", 1e-10, 1e-10), ("FP32", 1e-4, 1e-5)):
        hc = H.Config(mode=0, prec=getattr(H, prec), helicity_sampling=sampling, **kw)
        got, r = H.xsec_hist(n, hc, getattr(H, "OBS_" + which), 24, lo, hi)
        assert abs(got.sum() / r["sigma_fb"] - 1) < 1e-12
        assert abs(got.sum() / ref.sum() - 1) < tol_tot
        big = ref > 1e-3 * ref.max()
        assert np.all(np.abs(got[big] / ref[big] - 1) < tol_bin), (prec, got, ref)
        assert np.all((got > 0) == (ref > 0))


def _helicity_bits(orc, n, seed, i):
    h1, _, lam = orc.draw_helicity(n, seed, i)
    bits = 1 if h1 == 1 else 0
    for j, l in enumerate(lam):
        bits |= (1 << (1 + j)) if l == 1 else 0
    return bits


@pytest.mark.parametrize("n,mode,extra,npoints,sampling", [
    (3, "FIXED_SHAT", dict(sqrt_s=1000.0), 3000, 0),
    (2, "PP_TOY", dict(sqrt_s=14000.0, sqrt_shat_lo=150.0), 4100, 0),
    (4, "UNIFORM_SQRTSHAT", dict(sqrt_shat_lo=200.0, sqrt_shat_hi=2000.0), 1500, 1),
])
def test_event_records_match_oracle(H, orc, n, mode, extra, npoints, sampling):
    """heget_xsec_events: every generated point's weight, momenta, frame
    rapidity and drawn helicities against the oracle's own events."""
    kw = dict(seed=8, npoints=npoints, pt_min=20.0, eta_max=2.5, dr_min=0.4, **extra)
    hc, oc = _cfgs(H, orc, getattr(H, mode), prec=H.FP64, helicity_sampling=sampling, **kw)
    ev = H.xsec_events(n, hc, momenta=True, rapidity=True, helicity=bool(sampling))
    want = orc.xsec(n, oc, want_weights=True)
    r = ev["result"]
    assert r == H.xsec(n, hc)  # the same pass as heget_xsec
    assert r["n_acc"] == want["n_acc"]
    w, wo = ev["weight"], want["w"]
    # survivors and the scale of their weights: the helicity-summed weight
    # (with sampling, the drawn configuration may be one whose amplitude
    # vanishes, where both sides hold rounding noise of that scale)
    _, oc_sum = _cfgs(H, orc, getattr(H, mode), prec=H.FP64, **kw)
    scale = orc.xsec(n, oc_sum, want_weights=True)["w"] if sampling else wo
    surv = scale != 0
    assert int(surv.sum()) == r["n_acc"] and not w[~surv].any()
    # each side generates the momenta itself (they agree to 1e-12 of sqrt(shat),
    # nearly collinear n = 2 seeds amplifying the rounding of the generation):
    # the weights follow within 1e-11 of their scale, most of them to a few ulp
    err = np.abs(w[surv] - wo[surv]) / scale[surv]
    assert err.max() <= 1e-11 and np.median(err) <= 1e-14
    assert abs(w.sum() / r["n_gen"] / r["sigma_fb"] - 1) <= 1e-12
    checked = 0
    for i in range(0, npoints, 37):
        acc, p, y, _, _ = orc.point(n, oc, i)
        e_cm = p[0, 0] + p[1, 0]
        if mode == "PP_TOY" and e_cm < extra["sqrt_shat_lo"]:
            continue  # below threshold: no event, only the weight 0 is defined
        checked += 1
        assert np.abs(ev["momenta"][i] - p).max() <= 1e-12 * e_cm, i
        assert abs(ev["rapidity"][i] - y) <= 1e-12, i
        if sampling:
            assert int(ev["helicity"][i]) == _helicity_bits(orc, n, 8, i), i
    assert checked >= npoints // 37 // 2
    if mode != "PP_TOY":
        assert not ev["rapidity"].any()


def test_event_records_fp32_weights(H, orc):
    kw = dict(seed=9, npoints=2000, sqrt_s=1000.0, pt_min=20.0, eta_max=2.5, dr_min=0.4)
    hc, oc = _cfgs(H, orc, H.FIXED_SHAT, prec=H.FP32, **kw)
    w = H.xsec_events(4, hc)["weight"]
    wo = orc.xsec(4, oc, want_weights=True)["w"]
    assert np.array_equal(w == 0, wo == 0)
    rel = np.abs(w[wo != 0] / wo[wo != 0] - 1)
    assert np.median(rel) <= 1e-5 and np.quantile(rel, 0.999) <= 1e-3
