// The massless HELAS set of Appendix B as a device library, in FP32 or FP64:
// external wavefunctions of spin-1/2 fermions (B.1: ixxxx0/1/2, oxxxx0/1/2)
// and massless vectors (B.2: vxxxx0/1/2), and the four functions of the
// fermion-fermion-vector vertex (B.3: iovxxx, fvixx0, fvoxx0, jioxx0) for the
// Lagrangian  psibar_F1 gamma^mu (gal0 P_L + gal1 P_R) psi_F2 V*_mu.
//
// Conventions.  Spinors are in the chiral representation with the
// left-handed pair first, so a Dirac 4-spinor is two Weyl pairs (L, R) and
//     eps-slash = [[0, V-], [V+, 0]],  V+- = eps^0 +- sigma.eps,
// the only algebra the vertex functions need: they are written as 2x2
// complex matrices acting on Weyl pairs, with no 4x4 gamma matrix anywhere.
// A wavefunction carries its momentum along the flow (p nSF for fermions,
// p nSV for vectors), as the HELAS records do.  Propagators follow from vertex
// factors i Gamma, fermion propagators i slash(q)/q^2 and photon propagators
// -i g/q^2: an amplitude is i M with M the product of the Gamma's, a factor
// -slash(q)/q^2 per internal fermion and +g/q^2 per internal photon.
//
// Spinors of momentum p are helicity eigenstates; in Cartesian form, with
// p+ = p0 + p3, NH = nHEL nSF and s = nSF sqrt(p+),
//     |fi> (ixxxx):  NH = +1: (0, 0, s, (p1 + i p2)/s)
//                    NH = -1: ((-p1 + i p2)/s, s, 0, 0)
//     <fo| (oxxxx):  NH = +1: (s, (p1 - i p2)/s, 0, 0)
//                    NH = -1: (0, 0, (-p1 - i p2)/s, s)
// (v(p, h) = -u(p, -h), ubar = u^dagger gamma^0).  These break down when
// p+ -> 0 (p along -z): p+ is formed as pT^2/(p0 - p3) for p3 < 0, which
// keeps its relative accuracy for momenta close to -z, and on the -z axis
// itself the phase conventions of ixxxx2 / oxxxx2 apply (azimuth 0 for
// flowing-in and pi for flowing-out spinors).  Polarisations are
//     eps(k, lam) = (-lam e_theta - i e_phi)/sqrt(2)   (nSV = -1, incoming)
// and their conjugates (nSV = +1, outgoing), e_theta and e_phi the polar unit
// vectors of k, eps^0 = 0; on the z axis the azimuth is 0 along +z and pi
// along -z, which are the phases of vxxxx1 / vxxxx2.
//
// The includer provides __host__ and __device__ (hip_runtime.h), so that a
// CPU test can compile the same functions for the host.
#pragma once
#include <math.h>

namespace heget {
namespace helas {

template <typename R>
struct Cx {
    R re, im;
};

template <typename R>
__host__ __device__ inline Cx<R> cx(R re, R im = R(0)) { return {re, im}; }
template <typename R>
__host__ __device__ inline Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ inline Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ inline Cx<R> operator-(Cx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__host__ __device__ inline Cx<R> operator*(Cx<R> a, Cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ inline Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__host__ __device__ inline Cx<R> conj(Cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__host__ __device__ inline Cx<R> times_i(Cx<R> a) { return {-a.im, a.re}; }

// A wavefunction: four complex components (a Dirac spinor as Weyl pairs
// c[0..1] = L, c[2..3] = R, or a vector's contravariant components) and the
// real momentum along the flow.
template <typename R>
struct Wave {
    Cx<R> c[4];
    R p[4];
};

// 2x2 complex matrix [[a, b], [c, d]] acting on Weyl pairs.
template <typename R>
struct M2 {
    Cx<R> a, b, c, d;
};

// V+ = v^0 + sigma.v and V- = v^0 - sigma.v of a complex 4-vector.
template <typename R>
__host__ __device__ inline M2<R> sig_plus(const Cx<R> v[4])
{
    return {v[0] + v[3], v[1] - times_i(v[2]), v[1] + times_i(v[2]), v[0] - v[3]};
}
template <typename R>
__host__ __device__ inline M2<R> sig_minus(const Cx<R> v[4])
{
    return {v[0] - v[3], times_i(v[2]) - v[1], -v[1] - times_i(v[2]), v[0] + v[3]};
}
// The same for a real momentum.
template <typename R>
__host__ __device__ inline M2<R> sig_plus(const R q[4])
{
    return {cx(q[0] + q[3]), cx(q[1], -q[2]), cx(q[1], q[2]), cx(q[0] - q[3])};
}
template <typename R>
__host__ __device__ inline M2<R> sig_minus(const R q[4])
{
    return {cx(q[0] - q[3]), cx(-q[1], q[2]), cx(-q[1], -q[2]), cx(q[0] + q[3])};
}

// column: M x;  row: x M
template <typename R>
__host__ __device__ inline void col(const M2<R> &m, Cx<R> x0, Cx<R> x1, Cx<R> &y0, Cx<R> &y1)
{
    y0 = m.a * x0 + m.b * x1;
    y1 = m.c * x0 + m.d * x1;
}
template <typename R>
__host__ __device__ inline void row(Cx<R> x0, Cx<R> x1, const M2<R> &m, Cx<R> &y0, Cx<R> &y1)
{
    y0 = x0 * m.a + x1 * m.c;
    y1 = x0 * m.b + x1 * m.d;
}

template <typename R>
__host__ __device__ inline R minkowski2(const R q[4])
{
    return q[0] * q[0] - (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
}

// ---- B.1 fermion wavefunctions ----

// p+ = p0 + p3 without cancellation for p near -z (massless p).
template <typename R>
__host__ __device__ inline R light_cone_plus(const R p[4])
{
    return p[3] >= R(0) ? p[0] + p[3] : (p[1] * p[1] + p[2] * p[2]) / (p[0] - p[3]);
}

template <typename R>
__host__ __device__ inline void set_momentum(Wave<R> &w, const R p[4], int sign)
{
    for (int m = 0; m < 4; ++m) w.p[m] = R(sign) * p[m];
}

// Flowing-in spinor for p along -z (ixxxx2): nHEL sqrt(2 p0) in slot 3 for
// NH = +1, in slot 0 for NH = -1.
template <typename R>
__host__ __device__ inline Wave<R> ixxxx2(const R p[4], int nhel, int nsf)
{
    Wave<R> w;
    const Cx<R> z = cx(R(0)), chi = cx(R(nhel) * sqrt(R(2) * p[0]));
    const bool up = nhel * nsf == 1;
    w.c[0] = up ? z : chi;
    w.c[1] = z;
    w.c[2] = z;
    w.c[3] = up ? chi : z;
    set_momentum(w, p, nsf);
    return w;
}

// Flowing-in spinor, any direction (ixxxx0).
template <typename R>
__host__ __device__ inline Wave<R> ixxxx0(const R p[4], int nhel, int nsf)
{
    const R pp = light_cone_plus(p);
    if (!(pp > R(0))) return ixxxx2(p, nhel, nsf);
    Wave<R> w;
    const int nh = nhel * nsf;
    const R s = R(nsf) * sqrt(pp), rs = R(1) / s;
    const Cx<R> z = cx(R(0)), sq = cx(s), chi = cx(R(nh) * p[1] * rs, p[2] * rs);
    const bool up = nh == 1;
    w.c[0] = up ? z : chi;
    w.c[1] = up ? z : sq;
    w.c[2] = up ? sq : z;
    w.c[3] = up ? chi : z;
    set_momentum(w, p, nsf);
    return w;
}

// Flowing-in spinor for p along +z (ixxxx1): the general form with pT = 0.
template <typename R>
__host__ __device__ inline Wave<R> ixxxx1(const R p[4], int nhel, int nsf)
{
    Wave<R> w;
    const R s = R(nsf) * sqrt(p[0] + p[3]);
    const Cx<R> z = cx(R(0)), sq = cx(s);
    const bool up = nhel * nsf == 1;
    w.c[0] = z;
    w.c[1] = up ? z : sq;
    w.c[2] = up ? sq : z;
    w.c[3] = z;
    set_momentum(w, p, nsf);
    return w;
}

// Flowing-out spinor for p along -z (oxxxx2): -nHEL sqrt(2 p0) in slot 1 for
// NH = +1, in slot 2 for NH = -1.
template <typename R>
__host__ __device__ inline Wave<R> oxxxx2(const R p[4], int nhel, int nsf)
{
    Wave<R> w;
    const Cx<R> z = cx(R(0)), chi = cx(-R(nhel) * sqrt(R(2) * p[0]));
    const bool up = nhel * nsf == 1;
    w.c[0] = z;
    w.c[1] = up ? chi : z;
    w.c[2] = up ? z : chi;
    w.c[3] = z;
    set_momentum(w, p, nsf);
    return w;
}

// Flowing-out spinor, any direction (oxxxx0).
template <typename R>
__host__ __device__ inline Wave<R> oxxxx0(const R p[4], int nhel, int nsf)
{
    const R pp = light_cone_plus(p);
    if (!(pp > R(0))) return oxxxx2(p, nhel, nsf);
    Wave<R> w;
    const int nh = nhel * nsf;
    const R s = R(nsf) * sqrt(pp), rs = R(1) / s;
    const Cx<R> z = cx(R(0)), sq = cx(s), chi = cx(R(nh) * p[1] * rs, -p[2] * rs);
    const bool up = nh == 1;
    w.c[0] = up ? sq : z;
    w.c[1] = up ? chi : z;
    w.c[2] = up ? z : chi;
    w.c[3] = up ? z : sq;
    set_momentum(w, p, nsf);
    return w;
}

// Flowing-out spinor for p along +z (oxxxx1).
template <typename R>
__host__ __device__ inline Wave<R> oxxxx1(const R p[4], int nhel, int nsf)
{
    Wave<R> w;
    const R s = R(nsf) * sqrt(p[0] + p[3]);
    const Cx<R> z = cx(R(0)), sq = cx(s);
    const bool up = nhel * nsf == 1;
    w.c[0] = up ? sq : z;
    w.c[1] = z;
    w.c[2] = z;
    w.c[3] = up ? z : sq;
    set_momentum(w, p, nsf);
    return w;
}

// ---- B.2 vector wavefunctions ----

// Massless polarisation, any direction (vxxxx0): with cos/sin of the polar
// angle (ct, st) and of the azimuth (cf, sf),
//   eps^1 = (-lam ct cf - i nsv sf)/sqrt2,  eps^2 = (-lam ct sf + i nsv cf)/sqrt2,
//   eps^3 = lam st/sqrt2   (the conjugate of eps for nsv = +1).
template <typename R>
__host__ __device__ inline Wave<R> vxxxx0(const R k[4], int nhel, int nsv)
{
    Wave<R> w;
    const R pt2 = k[1] * k[1] + k[2] * k[2];
    const R pt = sqrt(pt2), kabs = sqrt(pt2 + k[3] * k[3]);
    const R r2 = R(0.70710678118654752440);
    const R lam = R(nhel), sv = R(nsv);
    R cf, sf;
    if (pt > R(0)) {
        const R rpt = R(1) / pt;
        cf = k[1] * rpt;
        sf = k[2] * rpt;
    } else {
        cf = k[3] < R(0) ? R(-1) : R(1);
        sf = R(0);
    }
    const R rk = R(1) / kabs, ct = k[3] * rk, st = pt * rk;
    w.c[0] = cx(R(0));
    w.c[1] = cx(-lam * ct * cf * r2, -sv * sf * r2);
    w.c[2] = cx(-lam * ct * sf * r2, sv * cf * r2);
    w.c[3] = cx(lam * st * r2);
    set_momentum(w, k, nsv);
    return w;
}

// Incoming vector along +z (vxxxx1) and along -z (vxxxx2); momentum -k.
// They serve initial-state vectors only (the flow sign is not an argument).
template <typename R>
__host__ __device__ inline Wave<R> vxxxx1(const R k[4], int nhel)
{
    const R r2 = R(0.70710678118654752440);
    Wave<R> w;
    w.c[0] = cx(R(0));
    w.c[1] = cx(-R(nhel) * r2);
    w.c[2] = cx(R(0), -r2);
    w.c[3] = cx(R(0));
    set_momentum(w, k, -1);
    return w;
}
template <typename R>
__host__ __device__ inline Wave<R> vxxxx2(const R k[4], int nhel)
{
    const R r2 = R(0.70710678118654752440);
    Wave<R> w;
    w.c[0] = cx(R(0));
    w.c[1] = cx(-R(nhel) * r2);
    w.c[2] = cx(R(0), r2);
    w.c[3] = cx(R(0));
    set_momentum(w, k, -1);
    return w;
}

// ---- B.3 fermion-fermion-vector vertex ----

// Amplitude <fo| eps-slash Gamma |fi> = gal0 R_o V+ L_i + gal1 L_o V- R_i (iovxxx).
template <typename R>
__host__ __device__ inline Cx<R> iovxxx(const Wave<R> &fi, const Wave<R> &fo, const Wave<R> &vc,
                                        R gal0, R gal1)
{
    const M2<R> vp = sig_plus(vc.c), vm = sig_minus(vc.c);
    Cx<R> a0, a1, b0, b1;
    col(vp, fi.c[0], fi.c[1], a0, a1);
    col(vm, fi.c[2], fi.c[3], b0, b1);
    return gal0 * (fo.c[2] * a0 + fo.c[3] * a1) + gal1 * (fo.c[0] * b0 + fo.c[1] * b1);
}

// Off-shell flowing-in fermion (-1/q^2) slash(q) eps-slash Gamma |fi>,
// q = p_fi - k (fvixx0): L' = d Q- (gal0 V+ L), R' = d Q+ (gal1 V- R).
template <typename R>
__host__ __device__ inline Wave<R> fvixx0(const Wave<R> &fi, const Wave<R> &vc, R gal0, R gal1)
{
    Wave<R> w;
    for (int m = 0; m < 4; ++m) w.p[m] = fi.p[m] - vc.p[m];
    const R d = R(-1) / minkowski2(w.p);
    Cx<R> l0, l1, r0, r1;
    col(sig_plus(vc.c), fi.c[0], fi.c[1], l0, l1);
    col(sig_minus(vc.c), fi.c[2], fi.c[3], r0, r1);
    const R gl = d * gal0, gr = d * gal1;
    col(sig_minus(w.p), gl * l0, gl * l1, w.c[0], w.c[1]);
    col(sig_plus(w.p), gr * r0, gr * r1, w.c[2], w.c[3]);
    return w;
}

// Off-shell flowing-out fermion <fo| eps-slash Gamma slash(q) (-1/q^2),
// q = p_fo + k (fvoxx0): L' = d (gal1 L V-) Q+, R' = d (gal0 R V+) Q-.
template <typename R>
__host__ __device__ inline Wave<R> fvoxx0(const Wave<R> &fo, const Wave<R> &vc, R gal0, R gal1)
{
    Wave<R> w;
    for (int m = 0; m < 4; ++m) w.p[m] = fo.p[m] + vc.p[m];
    const R d = R(-1) / minkowski2(w.p);
    Cx<R> l0, l1, r0, r1;
    row(fo.c[0], fo.c[1], sig_minus(vc.c), l0, l1);
    row(fo.c[2], fo.c[3], sig_plus(vc.c), r0, r1);
    const R gl = d * gal1, gr = d * gal0;
    row(gl * l0, gl * l1, sig_plus(w.p), w.c[0], w.c[1]);
    row(gr * r0, gr * r1, sig_minus(w.p), w.c[2], w.c[3]);
    return w;
}

// Off-shell vector current J^mu = <fo| gamma^mu Gamma |fi>/q^2, q = p_fo - p_fi
// (jioxx0, Feynman gauge): with gamma^mu = [[0, sigma^mu], [sigmabar^mu, 0]],
//   J^0 = gal0 R_o.L_i + gal1 L_o.R_i,  J^j = gal1 L_o s^j R_i - gal0 R_o s^j L_i.
template <typename R>
__host__ __device__ inline Wave<R> jioxx0(const Wave<R> &fi, const Wave<R> &fo, R gal0, R gal1)
{
    Wave<R> w;
    for (int m = 0; m < 4; ++m) w.p[m] = fo.p[m] - fi.p[m];
    const R dd = R(1) / minkowski2(w.p);
    const R g0 = dd * gal0, g1 = dd * gal1;
    // bilinears of the right-handed row with the left-handed column and v.v.
    const Cx<R> a00 = fo.c[2] * fi.c[0], a01 = fo.c[2] * fi.c[1];
    const Cx<R> a10 = fo.c[3] * fi.c[0], a11 = fo.c[3] * fi.c[1];
    const Cx<R> b00 = fo.c[0] * fi.c[2], b01 = fo.c[0] * fi.c[3];
    const Cx<R> b10 = fo.c[1] * fi.c[2], b11 = fo.c[1] * fi.c[3];
    // x s^1 y = x0 y1 + x1 y0;  x s^2 y = -i (x0 y1 - x1 y0);  x s^3 y = x0 y0 - x1 y1
    w.c[0] = g0 * (a00 + a11) + g1 * (b00 + b11);
    w.c[1] = g1 * (b01 + b10) - g0 * (a01 + a10);
    w.c[2] = times_i(g0 * (a01 - a10) - g1 * (b01 - b10));
    w.c[3] = g1 * (b00 - b11) - g0 * (a00 - a11);
    return w;
}

}  // namespace helas
}  // namespace heget
