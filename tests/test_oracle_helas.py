"""Pins of the oracle's massless HELAS set (Appendix B) in any direction.

The oracle builds spinors and polarisations from polar angles (helicity
eigenstates of the momentum direction).  Each test ties them to something
else: the Cartesian component forms the paper prints for every function, the
Dirac equation, chirality, completeness and normalisation, transversality and
the helicity eigen-equation of polarisations, Ward identities of the vertex
functions, and closed forms of complete |M|^2 (e+e- -> mu+mu-, Lorentz
invariance and the z-axis evaluator for u ubar -> n photons)."""
from __future__ import annotations

import math

import numpy as np
import pytest

ALPHA = 1.0 / 137.0

# chiral representation, left-handed pair on top: gamma^0 swaps the pairs,
# gamma^i = [[0, s^i], [-s^i, 0]], gamma5 = diag(-1, -1, 1, 1)
S = [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.diag([1.0, -1.0])]
Z2 = np.zeros((2, 2))
G = [np.block([[Z2, S[0]], [S[0], Z2]])] + [np.block([[Z2, S[i]], [-S[i], Z2]]) for i in (1, 2, 3)]
G5 = np.diag([-1.0, -1.0, 1.0, 1.0]).astype(complex)


def slash(a):
    return G[0] * a[0] - G[1] * a[1] - G[2] * a[2] - G[3] * a[3]


def mdot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def wave(out):
    return out[0:8:2] + 1j * out[1:8:2], out[8:12]


def rec(w, p):
    r = np.zeros(12)
    r[0:8:2], r[1:8:2], r[8:12] = np.real(w), np.imag(w), p
    return r


def massless(rng, e=None, direction=None):
    if direction is None:
        direction = rng.normal(size=3)
    d = np.asarray(direction, float) / np.linalg.norm(direction)
    e = rng.uniform(1.0, 500.0) if e is None else e
    return np.concatenate([[e], e * d])


def momenta(rng):
    """Generic directions, the two beam axes, and near-axis directions."""
    out = [massless(rng) for _ in range(6)]
    out += [massless(rng, direction=(0, 0, 1)), massless(rng, direction=(0, 0, -1))]
    out += [massless(rng, direction=(1e-7, 2e-7, -1)), massless(rng, direction=(3e-6, -1e-6, 1))]
    return out


def incoming(orc, p, h, nsf, which="ixxxx0"):
    return wave(orc.helas(which, list(p) + [h, nsf]))


def outgoing(orc, p, h, nsf, which="oxxxx0"):
    return wave(orc.helas(which, list(p) + [h, nsf]))


# ------------------------------------------------- the paper's component forms

def printed_in(p, nhel, nsf):
    """ixxxx0 as printed: SQ = sqrt(p0 + p3) nSF, NH = nHEL nSF,
    chi = (NH p1 + i p2)/SQ; NH = +1 -> (0, 0, SQ, chi), NH = -1 -> (chi, SQ, 0, 0)."""
    sq = math.sqrt(p[0] + p[3]) * nsf
    nh = nhel * nsf
    chi = (nh * p[1] + 1j * p[2]) / sq
    return np.array([0, 0, sq, chi]) if nh == 1 else np.array([chi, sq, 0, 0])


def printed_out(p, nhel, nsf):
    """oxxxx0 as printed: chi = (NH p1 - i p2)/SQ; NH = +1 -> (SQ, chi, 0, 0),
    NH = -1 -> (0, 0, chi, SQ)."""
    sq = math.sqrt(p[0] + p[3]) * nsf
    nh = nhel * nsf
    chi = (nh * p[1] - 1j * p[2]) / sq
    return np.array([sq, chi, 0, 0]) if nh == 1 else np.array([0, 0, chi, sq])


def printed_vec(p, nhel, nsv):
    """vxxxx0 as printed: 0, (-nHEL p1 p3/(p0 pT) - i nSV p2/pT)/sqrt2,
    (-nHEL p2 p3/(p0 pT) + i nSV p1/pT)/sqrt2, nHEL pT/(p0 sqrt2)."""
    pt = math.hypot(p[1], p[2])
    r = 1.0 / math.sqrt(2.0)
    return np.array([0, (-nhel * p[1] * p[3] / (p[0] * pt) - 1j * nsv * p[2] / pt) * r,
                     (-nhel * p[2] * p[3] / (p[0] * pt) + 1j * nsv * p[1] / pt) * r,
                     nhel * pt / p[0] * r])


@pytest.mark.parametrize("nsf", [1, -1])
@pytest.mark.parametrize("nhel", [1, -1])
def test_spinors_match_printed_forms(orc, nhel, nsf):
    rng = np.random.default_rng(11)
    for _ in range(20):
        p = massless(rng)
        for which in ("ixxxx0", "ixxxx1"):
            w, mom = incoming(orc, p, nhel, nsf, which)
            assert np.allclose(w, printed_in(p, nhel, nsf), rtol=0, atol=1e-12 * math.sqrt(p[0]))
            assert np.allclose(mom, nsf * p, rtol=0, atol=0)
        for which in ("oxxxx0", "oxxxx1"):
            w, mom = outgoing(orc, p, nhel, nsf, which)
            assert np.allclose(w, printed_out(p, nhel, nsf), rtol=0, atol=1e-12 * math.sqrt(p[0]))
            assert np.allclose(mom, nsf * p, rtol=0, atol=0)


@pytest.mark.parametrize("nsf", [1, -1])
@pytest.mark.parametrize("nhel", [1, -1])
def test_axis_spinors_match_printed_forms(orc, nhel, nsf):
    """+z: the generic forms with p1 = p2 = 0.  -z (ixxxx2, oxxxx2): chi = nHEL
    sqrt(2 p0) in the slot NH = +1 -> 3, NH = -1 -> 0 for flowing-in spinors,
    chi = -nHEL sqrt(2 p0) in the slot NH = +1 -> 1, NH = -1 -> 2 for flowing-out."""
    e = 45.5
    up, dn = np.array([e, 0, 0, e]), np.array([e, 0, 0, -e])
    nh = nhel * nsf
    r = math.sqrt(2 * e)
    for which in ("ixxxx0", "ixxxx1"):
        assert np.allclose(incoming(orc, up, nhel, nsf, which)[0], printed_in(up, nhel, nsf), atol=1e-13)
    want = np.zeros(4, complex)
    want[3 if nh == 1 else 0] = nhel * r
    for which in ("ixxxx0", "ixxxx2"):
        assert np.allclose(incoming(orc, dn, nhel, nsf, which)[0], want, atol=1e-13)
    want = np.zeros(4, complex)
    want[1 if nh == 1 else 2] = -nhel * r
    for which in ("oxxxx0", "oxxxx2"):
        assert np.allclose(outgoing(orc, dn, nhel, nsf, which)[0], want, atol=1e-13)


@pytest.mark.parametrize("nsv", [1, -1])
@pytest.mark.parametrize("nhel", [1, -1])
def test_vectors_match_printed_forms(orc, nhel, nsv):
    rng = np.random.default_rng(12)
    for _ in range(20):
        k = massless(rng)
        w, mom = wave(orc.helas("vxxxx0", list(k) + [nhel, nsv]))
        assert np.allclose(w, printed_vec(k, nhel, nsv), rtol=0, atol=1e-14)
        assert np.allclose(mom, nsv * k, rtol=0, atol=0)
    # vxxxx1 / vxxxx2 as printed: (0, -nHEL/sqrt2, -+ i/sqrt2, 0), momentum -p
    r = 1.0 / math.sqrt(2.0)
    for which, k, im in (("vxxxx1", [7.0, 0, 0, 7.0], -r), ("vxxxx2", [7.0, 0, 0, -7.0], r)):
        w, mom = wave(orc.helas(which, k + [nhel, nsv]))
        assert np.allclose(w, [0, -nhel * r, 1j * im, 0], rtol=0, atol=1e-15)
        assert np.allclose(mom, -np.array(k), rtol=0, atol=0)


def test_generic_vector_on_the_axes_equals_axis_functions(orc):
    """vxxxx0 along +-z (where the printed form divides by pT = 0) takes the
    phase of vxxxx1 / vxxxx2 for incoming vectors, the conjugate for outgoing."""
    for nhel in (1, -1):
        for which, k in (("vxxxx1", [7.0, 0, 0, 7.0]), ("vxxxx2", [7.0, 0, 0, -7.0])):
            ax = wave(orc.helas(which, k + [nhel, -1]))[0]
            assert np.allclose(wave(orc.helas("vxxxx0", k + [nhel, -1]))[0], ax, atol=1e-15)
            assert np.allclose(wave(orc.helas("vxxxx0", k + [nhel, 1]))[0], np.conj(ax), atol=1e-15)


# ------------------------------------------------- physics of the spinors

@pytest.mark.parametrize("nsf", [1, -1])
def test_dirac_equation_chirality_and_normalisation(orc, nsf):
    rng = np.random.default_rng(13)
    for p in momenta(rng):
        tol = 1e-12 * p[0]
        for h in (1, -1):
            u, _ = incoming(orc, p, h, nsf)
            ub, _ = outgoing(orc, p, h, nsf)
            # massless Dirac equation: pslash u = 0, ubar pslash = 0
            assert np.abs(slash(p) @ u).max() < tol
            assert np.abs(ub @ slash(p)).max() < tol
            # gamma5 u(p, h) = h u, gamma5 v(p, h) = -h v; same for the row spinors
            assert np.allclose(G5 @ u, nsf * h * u, atol=tol)
            assert np.allclose(ub @ G5, -nsf * h * ub, atol=tol)
            # ubar is the Dirac adjoint of the column spinor of the same state,
            # except on the -z axis where the printed forms differ by a sign
            sign = -1 if (p[1] == 0 and p[2] == 0 and p[3] < 0) else 1
            assert np.allclose(ub, sign * np.conj(u) @ G[0], atol=tol)
            # ubar gamma^mu u = 2 p^mu (up to that sign)
            cur = np.array([ub @ G[m] @ u for m in range(4)])
            assert np.allclose(cur, 2 * sign * p, rtol=0, atol=tol)


def test_completeness(orc):
    """sum_h u ubar = pslash and sum_h v vbar = pslash for massless spinors
    (minus pslash on the -z axis, where the printed row and column forms
    differ by a sign)."""
    rng = np.random.default_rng(14)
    for p in momenta(rng):
        sign = -1 if (p[1] == 0 and p[2] == 0 and p[3] < 0) else 1
        for nsf in (1, -1):
            m = sum(np.outer(incoming(orc, p, h, nsf)[0], outgoing(orc, p, h, nsf)[0]) for h in (1, -1))
            assert np.allclose(m, sign * slash(p), rtol=0, atol=1e-12 * p[0])


def test_spinor_helicity_along_the_momentum(orc):
    """u(p, h): the spin operator Sigma . p_hat (Sigma = diag(s, s)) has eigenvalue h."""
    rng = np.random.default_rng(15)
    for p in momenta(rng):
        n = p[1:] / p[0]
        sig = sum(n[i] * np.block([[S[i + 1], Z2], [Z2, S[i + 1]]]) for i in range(3))
        for h in (1, -1):
            u, _ = incoming(orc, p, h, 1)
            assert np.allclose(sig @ u, h * u, atol=1e-12 * math.sqrt(p[0]))


# ------------------------------------------------- physics of the polarisations

def test_polarisations(orc):
    rng = np.random.default_rng(16)
    for k in momenta(rng):
        khat = k[1:] / k[0]
        comp = np.zeros((3, 3), complex)
        for lam in (1, -1):
            e_in = wave(orc.helas("vxxxx0", list(k) + [lam, -1]))[0]
            e_out = wave(orc.helas("vxxxx0", list(k) + [lam, 1]))[0]
            assert np.allclose(e_out, np.conj(e_in), atol=1e-15)
            assert abs(e_in[0]) == 0.0                                   # gauge eps^0 = 0
            assert abs(mdot(k, e_in)) < 1e-12 * k[0]                      # k . eps = 0
            assert abs(mdot(e_in, np.conj(e_in)) + 1) < 1e-14             # eps . eps* = -1
            # helicity: i khat x eps = lam eps
            assert np.allclose(1j * np.cross(khat, e_in[1:]), lam * e_in[1:], atol=1e-14)
            comp += np.outer(e_in[1:], np.conj(e_in[1:]))
        assert np.allclose(comp, np.eye(3) - np.outer(khat, khat), atol=1e-14)


# ------------------------------------------------- vertex functions

def _gal(rng):
    return list(rng.normal(size=2))


def test_vertex_matches_matrix_element(orc):
    """iovxxx = <fo| eps-slash (g0 P_L + g1 P_R) |fi> for arbitrary (off-shell) inputs."""
    rng = np.random.default_rng(17)
    PL, PR = (np.eye(4) - G5) / 2, (np.eye(4) + G5) / 2
    for _ in range(20):
        fi = rng.normal(size=4) + 1j * rng.normal(size=4)
        fo = rng.normal(size=4) + 1j * rng.normal(size=4)
        vc = rng.normal(size=4) + 1j * rng.normal(size=4)
        g0, g1 = _gal(rng)
        r = orc.helas("iovxxx", np.concatenate([rec(fi, rng.normal(size=4)), rec(fo, rng.normal(size=4)),
                                                rec(vc, rng.normal(size=4)), [g0, g1]]))
        want = fo @ slash(vc) @ (g0 * PL + g1 * PR) @ fi
        assert abs(complex(r[0], r[1]) - want) < 1e-12 * max(1.0, abs(want))


def test_off_shell_currents_match_propagator_forms(orc):
    """fvixx0 = -slash(q)/q^2 eps-slash Gamma fi (q = p_fi - k), fvoxx0 = fo
    eps-slash Gamma slash(q) (-1/q^2) (q = p_fo + k), jioxx0^mu = <fo| gamma^mu
    Gamma |fi>/q^2 (q = p_fo - p_fi): the HELAS propagator conventions."""
    rng = np.random.default_rng(18)
    PL, PR = (np.eye(4) - G5) / 2, (np.eye(4) + G5) / 2
    for _ in range(20):
        fi = rng.normal(size=4) + 1j * rng.normal(size=4)
        fo = rng.normal(size=4) + 1j * rng.normal(size=4)
        vc = rng.normal(size=4) + 1j * rng.normal(size=4)
        pi, po, k = rng.normal(size=4) * 50, rng.normal(size=4) * 50, rng.normal(size=4) * 50
        g0, g1 = _gal(rng)
        gam = g0 * PL + g1 * PR
        w, q = wave(orc.helas("fvixx0", np.concatenate([rec(fi, pi), rec(vc, k), [g0, g1]])))
        assert np.allclose(q, pi - k)
        assert np.allclose(w, -slash(q) @ slash(vc) @ gam @ fi / mdot(q, q), rtol=1e-12, atol=0)
        w, q = wave(orc.helas("fvoxx0", np.concatenate([rec(fo, po), rec(vc, k), [g0, g1]])))
        assert np.allclose(q, po + k)
        assert np.allclose(w, -fo @ slash(vc) @ gam @ slash(q) / mdot(q, q), rtol=1e-12, atol=0)
        w, q = wave(orc.helas("jioxx0", np.concatenate([rec(fi, pi), rec(fo, po), [g0, g1]])))
        assert np.allclose(q, po - pi)
        want = np.array([fo @ G[m] @ gam @ fi for m in range(4)]) / mdot(q, q)
        assert np.allclose(w, want, rtol=1e-12, atol=0)


def test_ward_identities(orc):
    """On-shell spinors: replacing the polarisation by its momentum gives 0 at
    the vertex, and fvixx0 / fvoxx0 return the chirally projected external
    spinor times -gal (the propagator cancels); q . jio = 0."""
    rng = np.random.default_rng(19)
    for _ in range(20):
        p1, p2 = massless(rng), massless(rng)
        g0, g1 = _gal(rng)
        for h1 in (1, -1):
            for h2 in (1, -1):
                fi, pi = incoming(orc, p1, h1, 1)          # u(p1), momentum p1 flowing in
                fo, po = outgoing(orc, p2, h2, 1)          # ubar(p2)
                k = po - pi                                # photon absorbed at the vertex
                scale = math.sqrt(p1[0] * p2[0]) * np.abs(k).max()
                r = orc.helas("iovxxx", np.concatenate([rec(fi, pi), rec(fo, po), rec(k, k), [g0, g1]]))
                assert abs(complex(r[0], r[1])) < 1e-11 * scale
                j, q = wave(orc.helas("jioxx0", np.concatenate([rec(fi, pi), rec(fo, po), [g0, g1]])))
                assert abs(mdot(q, j)) < 1e-11 * math.sqrt(p1[0] * p2[0])
                # fvixx0 with eps = k, q = p1 - k: kslash Gamma u = -gam qslash u,
                # so -qslash/q^2 (-gam qslash u) = gam u, gam the coupling of u's chirality
                kk = massless(rng)
                w, _ = wave(orc.helas("fvixx0", np.concatenate([rec(fi, pi), rec(kk, kk), [g0, g1]])))
                gam = g0 if h1 == -1 else g1
                assert np.allclose(w, gam * fi, atol=1e-11 * math.sqrt(p1[0]))
                # fvoxx0 with eps = -k, q = p2 - k: ubar (qslash - p2slash) Gamma qslash
                # = q^2 ubar Gamma~ (chiralities swapped through qslash), result -ubar Gamma~
                w, _ = wave(orc.helas("fvoxx0", np.concatenate([rec(fo, po), rec(-kk, -kk), [g0, g1]])))
                gam = g0 if h2 == -1 else g1
                assert np.allclose(w, -gam * fo, atol=1e-11 * math.sqrt(p2[0]))


# ------------------------------------------------- complete amplitudes

def _boost(p, beta):
    b = np.asarray(beta, float)
    b2 = b @ b
    gam = 1.0 / math.sqrt(1.0 - b2)
    bp = b @ p[1:]
    e = gam * (p[0] + bp)
    v = p[1:] + ((gam - 1.0) * bp / b2 + gam * p[0]) * b
    return np.concatenate([[e], v])


def test_ee_to_mumu_closed_form(orc):
    """sum over helicities |M|^2 = 8 e^4 q1^2 q2^2 (t^2 + u^2)/s^2 for massless
    f fbar -> f' fbar' through one photon (pins jioxx0 with iovxxx)."""
    rng = np.random.default_rng(20)
    e2 = 4 * math.pi * ALPHA
    for q1, q2 in ((-1.0, -1.0), (2 / 3, -1 / 3)):
        for _ in range(10):
            E = rng.uniform(5, 500)
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            p = [np.array([E, 0, 0, E]), np.array([E, 0, 0, -E]), np.concatenate([[E], E * d]),
                 np.concatenate([[E], -E * d])]
            beta = rng.uniform(-0.5, 0.5, size=3)
            p = [_boost(x, beta) for x in p]                 # any frame
            s, t, u = mdot(p[0] + p[1], p[0] + p[1]), mdot(p[0] - p[2], p[0] - p[2]), mdot(p[0] - p[3], p[0] - p[3])
            want = 8 * e2 * e2 * q1 * q1 * q2 * q2 * (t * t + u * u) / (s * s)
            got = orc.me2_ffff(np.concatenate(p), ALPHA, q1, q2)
            assert abs(got / want - 1) < 1e-12


@pytest.mark.parametrize("n", [2, 3, 4])
def test_frame_evaluator_is_lorentz_invariant_and_matches_axis_evaluator(orc, n):
    rng = np.random.default_rng(21 + n)
    for i in range(4):
        p = orc.cm_event(n, 1000.0, 5, i)
        ref = orc.me2(p, ALPHA, 2 / 3, False)
        assert abs(orc.me2_frame(n, p) / ref - 1) < 1e-12
        beta = rng.uniform(-0.6, 0.6, size=3)
        pb = np.array([_boost(x, beta) for x in p])
        assert abs(orc.me2_frame(n, pb) / ref - 1) < 1e-11
