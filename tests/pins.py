"""Independent closed forms and textbook results that pin the oracle.

Nothing here imports the oracle or the HIP library.  The Dirac algebra uses
the Dirac (standard) representation on purpose -- the oracle uses the chiral
one -- because the spin-summed trace formula does not depend on it.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

GEV2_FB = 0.3893793721e12  # (hbar c)^2 in GeV^2 fb (PDG)

_I2 = np.eye(2, dtype=complex)
_Z2 = np.zeros((2, 2), dtype=complex)
_SIG = [np.array([[0, 1], [1, 0]], dtype=complex),
        np.array([[0, -1j], [1j, 0]], dtype=complex),
        np.array([[1, 0], [0, -1]], dtype=complex)]
# Dirac representation: gamma^0 = diag(1,1,-1,-1), gamma^k = [[0, s_k], [-s_k, 0]]
DIRAC = np.array([np.block([[_I2, _Z2], [_Z2, -_I2]])] +
                 [np.block([[_Z2, s], [-s, _Z2]]) for s in _SIG])
METRIC = np.array([1.0, -1.0, -1.0, -1.0])


def mdot(a, b) -> float:
    return float(a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3])


def slash(a) -> np.ndarray:
    return DIRAC[0] * a[0] - DIRAC[1] * a[1] - DIRAC[2] * a[2] - DIRAC[3] * a[3]


def me2_trace(p: np.ndarray, alpha: float, charge: float) -> float:
    """sum over spins and polarisations of |M|^2 for q(p1) qbar(p2) -> n gamma.

    M^{mu_1..mu_n} = vbar(p2) Gamma u(p1), Gamma = sum over orderings of
    gamma^{mu} S(p1-K) gamma^{mu} ... S(p1-K1) gamma^{mu}, S(q) = qslash/q^2;
    spin sums give Tr[Gamma p1slash Gammabar p2slash] and the polarisation sum
    of each photon gives -g_{mu nu} (exact for the full gauge-invariant sum).
    """
    p = np.asarray(p, dtype=float)
    n = p.shape[0] - 2
    p1, p2, k = p[0], p[1], p[2:]
    total = np.zeros((4,) * n + (4, 4), dtype=complex)
    for perm in itertools.permutations(range(n)):
        # chain tensor, axes (mu of photon perm[0], ..., mu of perm[l], a, b)
        chain = DIRAC.copy()
        K = k[perm[0]].copy()
        for l in range(1, n):
            q = p1 - K
            S = slash(q) / mdot(q, q)
            chain = np.einsum("ab,...bc->...ac", S, chain)
            chain = np.einsum("mab,...bc->...mac", DIRAC, chain)
            # move the new Lorentz axis (just before the matrix axes) to the end of the photon axes
            K = K + k[perm[l]]
        # chain axes are ordered by position in the chain: axis i <-> photon perm[i];
        # einsum above inserted each new axis at position l (after the older ones)
        inv = [perm.index(j) for j in range(n)]
        total += np.transpose(chain, inv + [n, n + 1])
    G = total.reshape(4 ** n, 4, 4)
    g0 = DIRAC[0]
    Gbar = np.einsum("ab,xcb,cd->xad", g0, G.conj(), g0)
    tr = np.einsum("xab,bc,xcd,da->x", G, slash(p1), Gbar, slash(p2))
    sgn = np.array([-1.0, 1.0, 1.0, 1.0])  # -g_{mu mu}
    signs = np.ones(1)
    for _ in range(n):
        signs = np.multiply.outer(signs, sgn).reshape(-1)
    e2 = 4.0 * math.pi * alpha * charge * charge
    return float(np.real(np.sum(signs * tr)) * e2 ** n)


def me2_n2_closed(p: np.ndarray, alpha: float, charge: float) -> float:
    """q qbar -> gamma gamma, massless: sum |M|^2 = 8 (eQ)^4 (t/u + u/t)."""
    p1, k1, k2 = p[0], p[2], p[3]
    t = mdot(p1 - k1, p1 - k1)
    u = mdot(p1 - k2, p1 - k2)
    e2 = 4.0 * math.pi * alpha * charge * charge
    return 8.0 * e2 * e2 * (t / u + u / t)


def sigma_hat_n2(shat: float, alpha: float, charge: float, cos_max: float) -> float:
    """q qbar -> gamma gamma partonic sigma (fb) for |cos theta*| < cos_max, with
    spin 1/4, colour 1/3 and identical-photon 1/2 factors:
    sigma = 2 pi alpha^2 Q^4 / (3 shat) [ln((1+c)/(1-c)) - c]."""
    c = cos_max
    if c <= 0.0:
        return 0.0
    return (2.0 * math.pi * alpha ** 2 * charge ** 4 / (3.0 * shat) *
            (math.log((1.0 + c) / (1.0 - c)) - c) * GEV2_FB)


def cos_max_n2(sqrt_shat: float, y: float, pt_min: float, eta_max: float) -> float:
    """|cos theta*| bound for two back-to-back photons in a CM frame boosted by
    rapidity y: |eta* +- y| < eta_max and (sqrt_shat/2) sin theta* > pt_min."""
    lim_eta = eta_max - abs(y)
    if lim_eta <= 0:
        return 0.0
    c_eta = math.tanh(lim_eta)
    s = 2.0 * pt_min / sqrt_shat
    if s >= 1.0:
        return 0.0
    return min(c_eta, math.sqrt(1.0 - s * s))


def phase_space_volume_recursive(n: int, s: float) -> float:
    """Massless n-body phase-space volume of eq. (4) by the textbook recursion
    Phi_n(s) = int_0^s dM2/(2 pi) Phi_2(s; M2, 0) Phi_{n-1}(M2), with the
    two-body volume Phi_2 = (1 - M2/s)/(8 pi) (one mass M, one massless)."""
    from scipy.integrate import quad
    if n == 2:
        return 1.0 / (8.0 * math.pi)

    def inner(m2):
        return (1.0 - m2 / s) / (8.0 * math.pi) * phase_space_volume_recursive(n - 1, m2) / (2 * math.pi)

    # Phi_{n-1}(m2) is a power of m2, so evaluate it symbolically via the scaling
    # Phi_{n-1}(m2) = Phi_{n-1}(1) m2^(n-3)
    c = phase_space_volume_recursive(n - 1, 1.0)
    val, _ = quad(lambda m2: (1.0 - m2 / s) / (8.0 * math.pi) * c * m2 ** (n - 3) / (2 * math.pi),
                  0.0, s, epsabs=0, epsrel=1e-13)
    return val


def boost_z(p: np.ndarray, y: float) -> np.ndarray:
    """Longitudinal boost by rapidity y of momenta p[..., 4]."""
    ch, sh = math.cosh(y), math.sinh(y)
    out = np.array(p, dtype=float, copy=True)
    out[..., 0] = ch * p[..., 0] + sh * p[..., 3]
    out[..., 3] = sh * p[..., 0] + ch * p[..., 3]
    return out


def rotate_z(p: np.ndarray, a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    out = np.array(p, dtype=float, copy=True)
    out[..., 1] = c * p[..., 1] - s * p[..., 2]
    out[..., 2] = s * p[..., 1] + c * p[..., 2]
    return out


def boost_to(p: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Boost momenta p given in the rest frame of P into the frame where P has
    the given 4-momentum (textbook general boost)."""
    M = math.sqrt(mdot(P, P))
    b = P[1:] / P[0]
    b2 = float(b @ b)
    g = P[0] / M
    out = np.array(p, dtype=float, copy=True)
    for i in range(p.shape[0]):
        bp = float(b @ p[i, 1:])
        out[i, 0] = g * (p[i, 0] + bp)
        coef = (g - 1.0) * bp / b2 + g * p[i, 0] if b2 > 0 else 0.0
        out[i, 1:] = p[i, 1:] + coef * b
    return out
