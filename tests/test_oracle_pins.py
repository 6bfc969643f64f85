"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself: a
closed form, a textbook result computed here independently (tests/pins.py),
an exact symmetry, or a published known-answer vector.  The paper prints no
|M|^2 values, so no paper fixture exists for them; the cross-section closed
forms below replace one.
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np
import pytest

import pins

HERE = os.path.dirname(os.path.abspath(__file__))
ALPHA, Q = 1.0 / 137.0, 2.0 / 3.0


def _events(orc, n, sqrt_s, seed, count, cut=True):
    ev = []
    i = 0
    while len(ev) < count:
        p = orc.cm_event(n, sqrt_s, seed, i)
        i += 1
        if not cut or orc.pass_cuts(p[2:], 0.0, 20.0, 2.5, 0.4):
            ev.append(p)
    return ev


# ---------------------------------------------------------------- random numbers

def test_philox_known_answers(orc):
    """Philox4x32-10 known-answer vectors (tests/golden/philox4x32_10_kat.txt)."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_uniforms_in_open_interval_and_flat(orc):
    from scipy.stats import kstest
    for draw in (orc.uniform_pair, orc.uniform_quad):
        u = np.array([draw(7, i, b, 0) for i in range(4000) for b in range(2)]).ravel()
        assert np.all(u > 0.0) and np.all(u < 1.0)
        assert kstest(u, "uniform").pvalue > 1e-3
        # distinct (point, block, stream) give distinct draws
        a = draw(7, 5, 0, 0)
        assert not np.allclose(a, draw(7, 5, 1, 0))
        assert not np.allclose(a, draw(7, 5, 0, 1))
        assert not np.allclose(a, draw(8, 5, 0, 0))


def test_uniform_words_are_the_philox_output(orc):
    """Each uniform is its Philox word w mapped to (w + 1/2) 2^-32 (quad) or its
    word pair's top 53 bits to (x + 1/2) 2^-53 (pair), so the extremes of the
    words give the extremes of the open interval."""
    for point, block, stream, seed in ((5, 0, 0, 7), (123456789012, 3, 0, 2 ** 40 + 9), (1, 1, 1, 0)):
        ctr = [point & 0xFFFFFFFF, point >> 32, block, stream]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        w = [int(x) for x in orc.philox(ctr, key)]
        q = orc.uniform_quad(seed, point, block, stream)
        assert list(q) == [(x + 0.5) / 2 ** 32 for x in w]
        p = orc.uniform_pair(seed, point, block, stream)
        for j in range(2):
            hi53 = ((w[2 * j + 1] << 32) | w[2 * j]) >> 11
            assert p[j] == (hi53 + 0.5) / 2 ** 53
    assert (0 + 0.5) / 2 ** 32 > 0 and (2 ** 32 - 1 + 0.5) / 2 ** 32 < 1


# ---------------------------------------------------------------- phase space

@pytest.mark.parametrize("n", [2, 3, 4, 5, 8])
def test_rambo_conserves_momentum_and_is_massless(orc, n):
    """To rounding, on every point: the second pass of the conformal map keeps
    nearly collinear seeds (large boost factors, frequent at n = 2) from
    amplifying the seeds' rounding into visible masses and momentum imbalance."""
    ev = orc.cm_events(n, 1000.0, 3, 0, 20000 if n <= 4 else 2000)
    k = ev[:, 2:]
    assert np.all(k[..., 0] > 0)
    tot = k.sum(axis=1)
    assert np.abs(tot - np.array([1000.0, 0, 0, 0])).max() < 4e-15 * 1000.0 * n
    mass = np.abs(k[..., 0] ** 2 - (k[..., 1:] ** 2).sum(-1)) / k[..., 0] ** 2
    assert mass.max() < 4e-15


def test_rambo_weight_textbook_values(orc):
    s = 1000.0 ** 2
    assert orc.rambo_weight(2, s) == pytest.approx(1.0 / (8.0 * math.pi), rel=1e-14)
    assert orc.rambo_weight(3, s) == pytest.approx(s / (256.0 * math.pi ** 3), rel=1e-14)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8])
def test_rambo_weight_matches_recursive_phase_space(orc, n):
    s = 2000.0 ** 2
    assert orc.rambo_weight(n, s) == pytest.approx(pins.phase_space_volume_recursive(n, s), rel=1e-10)


def test_rambo_two_body_isotropic(orc):
    from scipy.stats import kstest
    c = np.array([orc.cm_event(2, 500.0, 11, i)[2, 3] / 250.0 for i in range(4000)])
    assert kstest(c, "uniform", args=(-1, 2)).pvalue > 1e-3


def test_rambo_three_body_flat_dalitz(orc):
    """Flat massless 3-body phase space: energy fractions x_i = 2E_i/sqrt(s)
    are uniform on the Dalitz triangle, so x_1 has density 2 x on [0,1]."""
    from scipy.stats import kstest
    x = np.array([2.0 * orc.cm_event(3, 100.0, 12, i)[2, 0] / 100.0 for i in range(4000)])
    assert kstest(x, lambda t: np.clip(t, 0, 1) ** 2).pvalue > 1e-3


# ---------------------------------------------------------------- cuts

def test_cuts_hand_events(orc):
    def ph(pt, eta, phi):
        return [pt * math.cosh(eta), pt * math.cos(phi), pt * math.sin(phi), pt * math.sinh(eta)]

    ok = np.array([ph(50, 0.0, 0.0), ph(50, 1.0, 2.0)])
    assert orc.pass_cuts(ok)
    assert not orc.pass_cuts(np.array([ph(19.9, 0.0, 0.0), ph(50, 1.0, 2.0)]))
    assert not orc.pass_cuts(np.array([ph(50, 2.6, 0.0), ph(50, 1.0, 2.0)]))
    assert not orc.pass_cuts(np.array([ph(50, -2.6, 0.0), ph(50, 1.0, 2.0)]))
    # Delta R = sqrt(0.3^2 + 0.2^2) = 0.36 < 0.4
    assert not orc.pass_cuts(np.array([ph(50, 0.5, 0.1), ph(50, 0.8, 0.3)]))
    assert orc.pass_cuts(np.array([ph(50, 0.5, 0.1), ph(50, 0.8, 0.3)]), dr_min=0.0)
    # Delta phi folds across +-pi: phi = 3.0 and -3.0 are 0.283 apart
    assert not orc.pass_cuts(np.array([ph(50, 0.0, 3.0), ph(50, 0.1, -3.0)]))
    # a boost by y shifts every eta
    assert orc.pass_cuts(np.array([ph(50, 2.0, 0.0), ph(50, 0.0, 2.0)]), y=0.4)
    assert not orc.pass_cuts(np.array([ph(50, 2.0, 0.0), ph(50, 0.0, 2.0)]), y=0.6)


# ---------------------------------------------------------------- |M|^2

def test_n2_closed_form(orc):
    for p in _events(orc, 2, 500.0, 0, 64, cut=False):
        assert orc.me2(p) == pytest.approx(pins.me2_n2_closed(p, ALPHA, Q), rel=1e-13)


@pytest.mark.parametrize("n,count", [(2, 4), (3, 4), (4, 3), (5, 1)])
def test_trace_formula(orc, n, count):
    """Convention-free pin: spin/polarisation sums as Dirac traces (Dirac rep.)."""
    for p in _events(orc, n, 1000.0, 21, count):
        ref = pins.me2_trace(p, ALPHA, Q)
        assert orc.me2(p) == pytest.approx(ref, rel=1e-11)


def test_trace_formula_skewed_frame(orc):
    """Same pin with a boosted, rotated frame (E1 != E2) and skip_zero off."""
    p = _events(orc, 3, 800.0, 22, 1)[0]
    p = pins.rotate_z(pins.boost_z(p, 0.37), 1.1)
    assert orc.me2(p, skip_zero=False) == pytest.approx(pins.me2_trace(p, ALPHA, Q), rel=1e-11)


def _lams(n):
    return [tuple(1 if (b >> i) & 1 else -1 for i in range(n)) for b in range(1 << n)]


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_schedules_agree(orc, n):
    """Chains from the ubar end (fvoxx0), from the u end (fvixx0), and the
    two-sided schedule of Appendix A.1 give the same amplitude per helicity."""
    p = _events(orc, n, 1000.0, 23, 1)[0]
    typical = max(abs(orc.amp(p, -1, 1, lam)) for lam in _lams(n))
    for lam in _lams(n)[:8]:
        for h1, h2 in [(1, -1), (-1, 1)]:
            a = orc.amp(p, h1, h2, lam)
            b = orc.amp_from_u(p, h1, h2, lam)
            c = orc.amp_meet(p, h1, h2, lam, split=-1)
            d = orc.amp_meet(p, h1, h2, lam, split=n // 2)
            scale = max(abs(a), typical)
            assert abs(a - b) < 1e-12 * scale
            assert abs(a - c) < 1e-12 * scale
            assert abs(a - d) < 1e-12 * scale


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_subset_recursion_equals_ordering_sum(orc, n):
    for p in _events(orc, n, 1500.0, 24, 2 if n < 6 else 1):
        assert orc.me2_subsets(p) == pytest.approx(orc.me2(p), rel=1e-12)


@pytest.mark.parametrize("n", [3, 4, 5])
def test_gauge_invariance(orc, n):
    """Ward identity: eps_i -> k_i makes the ordering sum vanish for any other
    polarisation vectors (here random complex ones)."""
    rng = np.random.default_rng(5 + n)
    p = _events(orc, n, 1000.0, 25, 1)[0]
    for i in range(n):
        eps = rng.normal(size=(n, 4)) + 1j * rng.normal(size=(n, 4))
        eps[i] = p[2 + i] / p[2 + i][0]
        for h1, h2 in [(1, -1), (-1, 1)]:
            a, sabs = orc.amp_custom_eps(p, h1, h2, eps)
            assert abs(a) < 1e-13 * sabs


@pytest.mark.parametrize("n", [3, 4, 5])
def test_bose_symmetry(orc, n):
    p = _events(orc, n, 1000.0, 26, 1)[0]
    ref = orc.me2(p)
    rng = np.random.default_rng(n)
    for _ in range(3):
        perm = rng.permutation(n)
        q = p.copy()
        q[2:] = p[2:][perm]
        assert orc.me2(q) == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_helicity_selection(orc, n):
    p = _events(orc, n, 1000.0, 27, 1)[0]
    for lam in _lams(n):
        assert orc.amp(p, 1, 1, lam) == 0
        assert orc.amp(p, -1, -1, lam) == 0
    typical = max(abs(orc.amp(p, -1, 1, lam)) for lam in _lams(n))
    assert abs(orc.amp(p, -1, 1, (1,) * n)) < 1e-14 * typical
    assert abs(orc.amp(p, -1, 1, (-1,) * n)) < 1e-14 * typical


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_parity_flip(orc, n):
    """|M(-h1,-h2,-lam)| = |M(h1,h2,lam)| pointwise (vector coupling)."""
    p = _events(orc, n, 1000.0, 28, 1)[0]
    for lam in _lams(n):
        a = abs(orc.amp(p, -1, 1, lam)) ** 2
        b = abs(orc.amp(p, 1, -1, tuple(-l for l in lam))) ** 2
        assert a == pytest.approx(b, rel=1e-12, abs=1e-30 * (a + b + 1e-300))


@pytest.mark.parametrize("n", [2, 3, 5])
def test_rotation_swaps_quark_direction(orc, n):
    """Rotating by pi about x puts u along -z; |M|^2 is unchanged (this is
    what lets one |M|^2 serve both beam assignments of eq. (1))."""
    p = _events(orc, n, 900.0, 29, 1)[0]
    r = p.copy()
    r[:, 2] *= -1
    r[:, 3] *= -1
    assert orc.me2(r, u_along_minus_z=True) == pytest.approx(orc.me2(p), rel=1e-12)
    assert orc.me2(r, u_along_minus_z=True, skip_zero=False) == pytest.approx(orc.me2(p), rel=1e-12)


@pytest.mark.parametrize("n", [2, 4])
def test_lorentz_invariance(orc, n):
    p = _events(orc, n, 1000.0, 30, 1)[0]
    ref = orc.me2(p)
    assert orc.me2(pins.rotate_z(p, 0.7)) == pytest.approx(ref, rel=1e-12)
    assert orc.me2(pins.boost_z(p, -0.8)) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("n", [3, 4])
def test_soft_photon_limit(orc, n):
    """k_n -> 0: |M_n|^2 -> (eQ)^2 2 p1.p2 / (p1.k p2.k) |M_{n-1}|^2 (eikonal)."""
    sqrt_s = 1000.0
    base = _events(orc, n - 1, sqrt_s, 31, 1)[0]
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    e2 = 4 * math.pi * ALPHA * Q * Q
    errs = []
    for delta in (10.0, 1.0, 0.1):  # GeV, well above the rounding floor
        ks = delta * np.concatenate([[1.0], d])
        P = base[0] + base[1] - ks
        M = math.sqrt(pins.mdot(P, P))
        rest = base[2:] * (M / sqrt_s)  # the same hard event, rescaled to mass M
        hard = pins.boost_to(rest, P)
        p = np.vstack([base[:2], hard, ks[None, :]])
        assert np.allclose(p[2:].sum(axis=0), base[0] + base[1], atol=1e-9)
        eik = e2 * 2 * pins.mdot(base[0], base[1]) / (pins.mdot(base[0], ks) * pins.mdot(base[1], ks))
        ratio = orc.me2(p) / (eik * orc.me2(base))
        errs.append(abs(ratio - 1))
    assert errs[2] < 1e-3
    assert errs[2] < 0.2 * errs[1] and errs[1] < 0.2 * errs[0]


# ---------------------------------------------------------------- cross sections

def test_sigma_config1_closed_form(orc):
    """u ubar -> 2 gamma, sqrt(shat) = 500 GeV, pT > 20, |eta| < 2.5:
    sigma = 2 pi alpha^2 Q^4/(3 s) [ln((1+c)/(1-c)) - c], c = tanh 2.5 = 137.78 fb."""
    cfg = orc.Config(mode=orc.FIXED_SHAT, seed=0, npoints=16384, sqrt_s=500.0,
                     pt_min=20.0, eta_max=2.5, dr_min=0.0)
    r = orc.xsec(2, cfg)
    c = pins.cos_max_n2(500.0, 0.0, 20.0, 2.5)
    ref = pins.sigma_hat_n2(500.0 ** 2, ALPHA, Q, c)
    assert ref == pytest.approx(137.783, abs=1e-3)
    assert abs(r["sigma_fb"] - ref) < 3.5 * r["err_fb"]
    assert r["err_fb"] < 0.02 * ref
    assert r["n_gen"] == 16384 and 0.97 * 16384 < r["n_acc"] < 16384


def test_sigma_uniform_sqrtshat_n2(orc):
    from scipy.integrate import quad
    lo, hi = 200.0, 2000.0
    cfg = orc.Config(mode=orc.UNIFORM_SQRTSHAT, seed=3, npoints=20000, sqrt_shat_lo=lo,
                     sqrt_shat_hi=hi, pt_min=20.0, eta_max=2.5, dr_min=0.4)
    r = orc.xsec(2, cfg)
    ref = quad(lambda x: pins.sigma_hat_n2(x * x, ALPHA, Q, pins.cos_max_n2(x, 0.0, 20.0, 2.5)),
               lo, hi, epsrel=1e-10)[0] / (hi - lo)
    assert abs(r["sigma_fb"] - ref) < 3.5 * r["err_fb"]


def test_sigma_pp_toy_n2(orc):
    """pp with the toy densities: both beam assignments of eq. (1), lab-frame
    cuts after the longitudinal boost, sqrt(shat) >= 150 GeV; compared with a
    2-D quadrature of the analytic partonic cross section."""
    from scipy.integrate import dblquad
    S, lo = 14000.0, 150.0

    def integrand(r2, r1):
        # x_u = r1^2 and x_ub = r2^(1/0.7) make D(x) dx smooth: 2(1-x_u)^3 dr1 and (1-x_ub)^6/0.7 dr2
        xu, xub = r1 * r1, r2 ** (1 / 0.7)
        shat = xu * xub * S * S
        if shat < lo * lo:
            return 0.0
        y = 0.5 * math.log(xu / xub)
        c = pins.cos_max_n2(math.sqrt(shat), y, 20.0, 2.5)
        return 2.0 * (1 - xu) ** 3 * (1 - xub) ** 6 / 0.7 * 2.0 * pins.sigma_hat_n2(shat, ALPHA, Q, c)

    rmin = lo / S  # x_u x_ub >= (lo/S)^2 requires r1 >= lo/S
    ref = dblquad(integrand, rmin, 1.0, lambda r1: 0.0, lambda r1: 1.0, epsabs=0, epsrel=1e-6)[0]
    cfg = orc.Config(mode=orc.PP_TOY, seed=2, npoints=100000, sqrt_s=S, sqrt_shat_lo=lo,
                     pt_min=20.0, eta_max=2.5, dr_min=0.4)
    r = orc.xsec(2, cfg)
    assert abs(r["sigma_fb"] - ref) < 3.5 * r["err_fb"]
    assert r["err_fb"] < 0.05 * ref


def test_pp_point_uses_both_beam_assignments(orc):
    """Per point, the two beam assignments of eq. (1) have equal |M|^2 and the
    same cut decision, so w = 2 f_pdf (partonic weight of assignment A)."""
    cfg = orc.Config(mode=orc.PP_TOY, seed=2, npoints=1, sqrt_s=14000.0, sqrt_shat_lo=150.0)
    seen = 0
    for i in range(400):
        acc, p, y, m, w = orc.point(3, cfg, i)
        if not acc:
            continue
        seen += 1
        # rebuild the weight of assignment A alone from the oracle's own pieces
        r = orc.uniform_pair(2, i, 0, 1)
        xu, xub = r[0] ** 2, r[1] ** (1 / 0.7)
        f = (1 - xu) ** 3 / 0.5 * (1 - xub) ** 6 / 0.7
        shat = xu * xub * 14000.0 ** 2
        assert y == pytest.approx(0.5 * math.log(xu / xub), rel=1e-14)
        base = (1 / (2 * shat) * 0.25 / 3 / 6 * orc.rambo_weight(3, shat) * pins.GEV2_FB)
        assert w == pytest.approx(2 * f * base * orc.me2(p), rel=1e-11)
        if seen >= 5:
            break
    assert seen >= 5


# ---- helicity sampling (the paper's per-event helicities, Section 3.1)

def test_helicity_draw_is_a_nonvanishing_configuration_and_uniform(orc):
    """Draws cover exactly the 2^(n+1) configurations with h_u != h_ubar, about
    uniformly (chi-square over 2^(n+1) cells at n = 3, 20000 draws)."""
    n = 3
    counts = {}
    for i in range(20000):
        h1, h2, lam = orc.draw_helicity(n, 5, i)
        assert h1 == -h2 and all(l in (-1, 1) for l in lam)
        counts[(h1, lam)] = counts.get((h1, lam), 0) + 1
    assert len(counts) == 2 ** (n + 1)
    e = 20000 / 2 ** (n + 1)
    chi2 = sum((c - e) ** 2 / e for c in counts.values())
    assert chi2 < 40.0  # 15 degrees of freedom; p ~ 5e-4


@pytest.mark.parametrize("n", [2, 3, 4])
def test_sampled_estimator_averages_to_the_sum(orc, n):
    """Averaged over every configuration a draw can give, 2^(n+1) |M_h|^2 is
    the helicity sum (the estimator is unbiased), and the point's sampled
    |M|^2 is that estimator for the drawn configuration."""
    p = _events(orc, n, 1000.0, 41, 1)[0]
    total = 0.0
    for h1 in (-1, 1):
        for lam in _lams(n):
            total += 2 ** (n + 1) * abs(orc.amp(p, h1, -h1, lam)) ** 2
    assert total / 2 ** (n + 1) == pytest.approx(orc.me2(p), rel=1e-13)
    cfg = orc.Config(mode=0, seed=41, npoints=1, sqrt_s=1000.0, helicity_sampling=1,
                     pt_min=0.0, eta_max=0.0, dr_min=0.0)
    acc, ev, _, me, _ = orc.point(n, cfg, 0)
    h1, h2, lam = orc.draw_helicity(n, 41, 0)
    assert me == pytest.approx(2 ** (n + 1) * abs(orc.amp(ev, h1, h2, lam)) ** 2, rel=1e-14)


@pytest.mark.parametrize("n", [2, 3])
def test_rotation_keeps_each_helicity_amplitude(orc, n):
    """The rotation by pi about x that swaps the quark directions leaves every
    helicity amplitude's modulus unchanged (not only the sum), so one |M_h|^2
    serves both beam assignments in sampling mode too."""
    p = _events(orc, n, 900.0, 42, 1)[0]
    r = p.copy()
    r[:, 2] *= -1
    r[:, 3] *= -1
    for h1 in (-1, 1):
        for lam in _lams(n):
            a = abs(orc.amp(p, h1, -h1, lam)) ** 2
            b = abs(orc.amp(r, h1, -h1, lam, u_along_minus_z=True)) ** 2
            assert b == pytest.approx(a, rel=1e-12, abs=1e-30 * (a + b + 1e-300))


def test_sampled_sigma_agrees_with_summed_sigma(orc):
    """n = 2 at 500 GeV (config 1 cuts): the sampled sigma and the summed sigma
    of the same points agree within their combined Monte-Carlo error."""
    kw = dict(mode=0, seed=0, npoints=16384, sqrt_s=500.0, pt_min=20.0, eta_max=2.5, dr_min=0.0)
    s = orc.xsec(2, orc.Config(**kw))
    h = orc.xsec(2, orc.Config(helicity_sampling=1, **kw))
    assert abs(h["sigma_fb"] - s["sigma_fb"]) < 4.0 * h["err_fb"]
    assert h["n_acc"] == s["n_acc"] and h["err_fb"] > s["err_fb"]


# ---- distributions (Fig. 2: leading photon pT, smallest photon-pair Delta R)

def test_observables_on_hand_built_photons(orc):
    import math
    def photon(pt, eta, phi):
        return [pt * math.cosh(eta), pt * math.cos(phi), pt * math.sin(phi), pt * math.sinh(eta)]
    k = np.array([photon(30.0, 0.1, 3.0), photon(50.0, 0.1, -3.0), photon(40.0, 1.5, 0.5)])
    assert orc.observable(k, orc.PT_MAX) == pytest.approx(50.0, rel=1e-14)
    # photons 0 and 1: same eta, azimuths 3.0 and -3.0 are 2 pi - 6 apart across the wrap
    assert orc.observable(k, orc.DR_MIN) == pytest.approx(2 * math.pi - 6.0, rel=1e-12)


@pytest.mark.parametrize("which,lo,hi", [(0, 20.0, 500.0), (1, 0.4, 4.0)])
def test_histogram_entries_add_up_to_sigma(orc, which, lo, hi):
    """Under- and overflow included, the bins hold every accepted weight once."""
    cfg = orc.Config(mode=0, seed=3, npoints=3000, sqrt_s=1000.0)
    h = orc.hist(3, cfg, which, 17, lo, hi)
    s = orc.xsec(3, cfg)
    assert h.sum() == pytest.approx(s["sigma_fb"], rel=1e-13)
    assert h[0] == 0.0  # the cuts put every accepted point above lo
    assert (h >= 0).all() and (h[1:-1] > 0).sum() >= 10


def _n2_observable(k, which):
    """Leading pT (which = 0) or Delta R of the photon pair (1), computed here."""
    if which == 0:
        return np.max(np.hypot(k[..., 1], k[..., 2]), axis=1)
    eta = np.arctanh(k[..., 3] / np.linalg.norm(k[..., 1:], axis=-1))
    phi = np.arctan2(k[..., 2], k[..., 1])
    dphi = np.abs(phi[:, 0] - phi[:, 1])
    dphi = np.minimum(dphi, 2.0 * math.pi - dphi)
    return np.hypot(eta[:, 0] - eta[:, 1], dphi)


@pytest.mark.parametrize("which,lo,hi", [(0, 0.0, 256.0), (1, 3.0, 6.2)])
def test_histogram_bins_against_the_n2_closed_form(orc, which, lo, hi):
    """Fig. 2 distributions at n = 2, sqrt(shat) = 500 GeV, pT > 20, |eta| < 2.5.
    The photons are back to back, so pT_max = (sqrt(shat)/2) sin(theta*) and
    Delta R = sqrt((2 eta*)^2 + pi^2) are both monotone in |cos theta*|: the
    expected content of a bin is sigma_hat(|cos| < c1) - sigma_hat(|cos| < c0)
    of the closed form at the bin's two edges.  Each bin of the oracle must
    agree within 4.5 of its own Monte-Carlo standard errors, and equal the
    oracle's weights binned here by the observable computed here."""
    sqrt_s, N, nb, seed = 500.0, 1 << 17, 8, 11
    cfg = orc.Config(mode=0, seed=seed, npoints=N, sqrt_s=sqrt_s, pt_min=20.0, eta_max=2.5,
                     dr_min=0.0)
    h = orc.hist(2, cfg, which, nb, lo, hi)
    w = orc.xsec(2, cfg, want_weights=True)["w"]
    x = _n2_observable(orc.cm_events(2, sqrt_s, seed, 0, N)[:, 2:], which)
    edges = lo + (hi - lo) * np.arange(nb + 1) / nb
    idx = np.digitize(x, edges)  # 0 below lo, nb + 1 at or above hi
    by_hand = np.array([w[idx == b].sum() for b in range(nb + 2)]) / N
    assert np.allclose(h, by_hand, rtol=1e-12, atol=1e-15 * h.sum())

    c_cut = pins.cos_max_n2(sqrt_s, 0.0, 20.0, 2.5)

    def cos_at(v):  # |cos theta*| where the observable equals v
        if which == 0:
            s = 2.0 * v / sqrt_s
            return math.sqrt(1.0 - s * s) if s < 1.0 else 0.0
        return math.tanh(math.sqrt(max(v * v - math.pi ** 2, 0.0)) / 2.0)

    def s_hat(c):
        return pins.sigma_hat_n2(sqrt_s ** 2, ALPHA, Q, min(c, c_cut))

    want = np.zeros(nb + 2)
    for b in range(nb):
        c0, c1 = cos_at(edges[b]), cos_at(edges[b + 1])
        want[b + 1] = abs(s_hat(c1) - s_hat(c0))
    assert want.sum() == pytest.approx(s_hat(1.0), rel=1e-12)  # every accepted point is in range
    se = np.sqrt(np.maximum([np.sum(w[idx == b] ** 2) / N - h[b] ** 2 for b in range(nb + 2)], 0.0)
                 / (N - 1))
    filled = want > 0
    assert filled.sum() >= 6
    assert np.all(se[filled] < 0.1 * want[filled])  # the comparison has power
    assert np.all(np.abs(h - want) <= 4.5 * se + 1e-12 * want.sum()), (h, want, se)


def test_mc_error_is_the_standard_error_of_the_weights(orc):
    """Section 3.1 step 6: sigma is the mean of the per-point weights and its
    error the standard error of that mean, std(w, ddof=1)/sqrt(N)."""
    cfg = orc.Config(mode=0, seed=5, npoints=4096, sqrt_s=1000.0)
    r = orc.xsec(3, cfg, want_weights=True)
    w = r["w"]
    assert (w > 0).sum() == r["n_acc"]
    assert r["sigma_fb"] == pytest.approx(np.mean(w), rel=1e-12)
    assert r["err_fb"] == pytest.approx(np.std(w, ddof=1) / math.sqrt(w.size), rel=1e-9)


def test_mc_error_matches_the_spread_over_seeds(orc):
    """The error estimate describes the scatter of sigma over independent
    samples: over 64 seeds of 4096 points, the sample standard deviation of
    sigma and the mean reported error agree (a dropped 1/(N-1) or square root
    is off by a factor of at least sqrt(4095))."""
    sig, err = [], []
    for seed in range(100, 164):
        r = orc.xsec(2, orc.Config(mode=0, seed=seed, npoints=4096, sqrt_s=500.0, pt_min=20.0,
                                   eta_max=2.5, dr_min=0.0))
        sig.append(r["sigma_fb"])
        err.append(r["err_fb"])
    ratio = np.std(sig, ddof=1) / np.mean(err)
    assert 0.7 < ratio < 1.35, ratio
    ref = pins.sigma_hat_n2(500.0 ** 2, ALPHA, Q, pins.cos_max_n2(500.0, 0.0, 20.0, 2.5))
    assert abs(np.mean(sig) - ref) < 4.0 * np.mean(err) / 8.0  # 64 samples: error / 8
