// Helicity-summed |M|^2 of u(p1) ubar(p2) -> n photons on one lane per point,
// by a shared-prefix tree over the n! photon orderings of eq. (6)-(8).
//
// Every diagram is one chain from the ubar end (Appendix A.2): the outgoing
// current is updated photon by photon with fvoxx0 (Appendix B.3.3) and closed
// on the u spinor with iovxx0 (Appendix B.3.1).  Chains that share their first
// j photons share their first j currents, so the orderings are visited as a
// depth-first walk of the tree of ordered prefixes: a node at depth j holds the
// current after j photons; it has one child per photon not yet used; the n!
// leaves close the chain.  Per helicity this costs sum_{j=1}^{n-1} n!/(n-j)!
// current updates and n! closings instead of (n-1) n! updates.
//
// Reductions of the HELAS 4-spinor algebra used here (all exact):
//  * Massless fermions keep their chirality along the line, so only one
//    2-component block of the 4-spinor is ever non-zero.  Quark helicities
//    h_u = h_ubar vanish identically.  Of the two non-vanishing pairs this
//    code evaluates (h_u, h_ubar) = (-1, +1): the ubar current lives in the
//    lower block (fvoxx0 outputs 3-4, coupling gal[0]) and closes on the upper
//    block of u.  The other pair is its parity image, |M(-h,-lam)| = |M(h,lam)|
//    pointwise for a vector coupling, so the helicity sum is twice the sum over
//    this block's 2^n photon helicities.
//  * For an outgoing photon the polarisation vxxxx0 of Appendix B.2 is
//    eps*(k,lam) = (-lam e_theta + i e_phi)/sqrt(2) with eps^0 = 0.  Its
//    2x2 vertex block sl = V g (fvoxx0 sl1, sl2) is
//        V = [[ a3, beta ], [ gamma, -a3 ]],  a3 = eps^3,
//        beta = eps^1 + i eps^2,  gamma = eps^1 - i eps^2,
//    and with light-cone components k+ = E + kz, k- = E - kz, kappa = kx + i ky,
//        sqrt(2) E pT V(+1) = [[ k+k-, -k+ kappa ], [ k- conj(kappa), -k+k- ]]
//        sqrt(2) E pT V(-1) = [[ -k+k-, -k- kappa ], [ k+ conj(kappa), k+k- ]].
//    Divided by its diagonal entry +-k+k- = +-pT^2 the block is
//        V'(+1) = [[ 1, -kappa / k- ], [  conj(kappa) / k+, -1 ]]
//        V'(-1) = [[ 1,  kappa / k+ ], [ -conj(kappa) / k-, -1 ]],
//    so V(lam) = +-(pT / (sqrt(2) E)) V'(lam).  Every diagram contains each
//    photon once, so the factors are common to all orderings of one helicity
//    configuration: their signs change no |M|^2, and the magnitudes
//    pT^2 / (2 E^2) per photon are applied to |M|^2 in FP64 at the end.  The
//    tree works with V' = [[1, beta'], [gamma', -1]], whose unit diagonal
//    turns every vertex product into fused multiply-adds on the current.
//  * The ubar spinor of oxxxx2 is (0, 0, -sqrt(2 E2), 0) and the u spinor of
//    ixxxx1 is (0, sqrt(E1 + p1z), 0, 0); their sizes are pulled out too, so
//    the chain starts at g = (1, 0) and closes with amp = gamma g2 - a3 g3
//    (gamma' g2 - g3 with the normalised block).
//  * Current update (fvoxx0, lower block): with q the momentum after adding k
//    and d = -1/q^2,
//        sl1 = a3 g2 + beta g3,     sl2 = gamma g2 - a3 g3,
//        g2' = d [ q- sl1 - (qx + i qy) sl2 ],
//        g3' = d [ q+ sl2 - (qx - i qy) sl1 ].
//    q starts at -p2 (HELAS stores the ubar momentum times nSF = -1).
//  * Momenta are scaled by an exact power of two 2^-m with 2^m ~ E1 + E2, so
//    FP32 values stay near 1; |M(p)|^2 = 2^(2m(2-n)) |M(2^-m p)|^2.
//  * Pair closing (CL = 2), the two-sided current reuse of the MadGraph
//    program of Appendix A.1 applied to the last two photons: before the last
//    photon r the current carries momentum p1 - k_r whatever the ordering, so
//    the last update plus closing of ordering (.., j, r) is a fixed row vector
//        u_jr = c_r d(p1 - k_r) P(p1 - k_r) V_j,   c_r = (gamma_r, -a3_r),
//    i.e. the incoming current from the u end after photon r (fvixx0) met at
//    the vertex of photon j.  The two orderings of a remaining pair {j, r}
//    close with U_jr = u_jr + u_rj, so a node with two photons left ends the
//    walk with one 2-vector product and the n! last-level updates disappear.
//    p1 - k_r is formed from p1 directly, free of the cancellation the
//    incremental sum from -p2 carries for photons close to the beam.
//
// Tree layout on the device.  The bottom MB levels of the tree (the subtree
// below a node with MB photons left) are unrolled at compile time with the
// remaining photons held in registers ("slots"), so their indices are
// constants.  The top n-MB levels walk the remaining-photon bitmask with a
// wave-uniform loop; photon data for those levels sit in LDS as
// [field][photon][lane] and are read with a wave-uniform photon index.  H
// helicity configurations ("variants") share each walk, which amortises the
// momentum part of every node (q update, q^2, 1/q^2) and the walk itself.
// All control flow is uniform across the wave: lanes only differ in data.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

namespace heget {

// Light-cone momentum: p = E + z, m = E - z, x, y; for photons also
// ip = 1 / p and im = 1 / m (unused for internal momenta).
template <typename R>
struct LMom {
    R p, m, x, y, ip, im;
};

// Chain currents (g2, g3) for H helicity variants.
template <typename R, int H>
struct Chain {
    R g2r[H], g2i[H], g3r[H], g3i[H];
};

// Normalised vertex block V' = [[1, beta], [gamma, -1]] for H variants.
template <typename R, int H>
struct Vert {
    R br[H], bi[H], gr[H], gi[H];
};

template <int H>
struct Acc {
    double re[H], im[H];
};

template <typename R, int H, int NS>
struct Slots {
    LMom<R> k[NS];
    Vert<R, H> v[NS];
};


// Unused placeholder when the walk closes photon by photon (CL = 1).
struct NoPairs {};

// V'(lam) of photon j for the H variants whose helicity configurations are
// cfg0 .. cfg0+H-1 (bit j set = helicity +1).  cfg0 is wave-uniform and a
// multiple of H, so configuration cfg0 + h is cfg0 | h: written so, a photon
// at or above log2(H) visibly has one block for all H variants.
template <typename R, int H>
__device__ __forceinline__ Vert<R, H> make_vert(const LMom<R> &k, uint32_t cfg0, int j)
{
    Vert<R, H> v;
    const R xp = k.x * k.ip, yp = k.y * k.ip;  // kappa / k+
    const R xm = k.x * k.im, ym = k.y * k.im;  // kappa / k-
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const bool plus = ((cfg0 | static_cast<uint32_t>(h)) >> j) & 1u;
        v.br[h] = plus ? -xm : xp;
        v.bi[h] = plus ? -ym : yp;
        v.gr[h] = plus ? xp : -xm;
        v.gi[h] = plus ? -yp : ym;
    }
    return v;
}

// -1/x: one v_rcp_f32 (1 ulp) in FP32; in FP64 v_rcp_f64 refined by two
// Newton steps r <- r + r (1 - x r), which restores full double precision.
__device__ __forceinline__ float neg_recip(float x) { return -__builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double neg_recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return -r;
}

// Momentum part of a node: q' = q + k, and d * (q'-, q'+, q'x, q'y), d = -1/q'^2.
template <typename R>
struct Prop {
    R m, p, x, y;
};

// d * (q-, q+, qx, qy), d = -1/q^2, for an internal momentum q.
template <typename R>
__device__ __forceinline__ Prop<R> prop_at(const LMom<R> &q)
{
    const R q2 = q.p * q.m - q.x * q.x - q.y * q.y;
    const R d = neg_recip(q2);
    return {d * q.m, d * q.p, d * q.x, d * q.y};
}

template <typename R>
__device__ __forceinline__ Prop<R> propagate(const LMom<R> &q, const LMom<R> &k, LMom<R> &qn)
{
    qn.p = q.p + k.p;
    qn.m = q.m + k.m;
    qn.x = q.x + k.x;
    qn.y = q.y + k.y;
    qn.ip = R(0);
    qn.im = R(0);
    const R q2 = qn.p * qn.m - qn.x * qn.x - qn.y * qn.y;
    const R d = neg_recip(q2);
    return {d * qn.m, d * qn.p, d * qn.x, d * qn.y};
}

// The vertex half of a current update, (sl1, sl2) = V' g, for every variant.
template <typename R, int H>
struct Half {
    R s1r[H], s1i[H], s2r[H], s2i[H];
};

template <typename R, int H>
__device__ __forceinline__ Half<R, H> vertex_half(const Vert<R, H> &v, const Chain<R, H> &c)
{
    Half<R, H> s;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        s.s1r[h] = fma(v.br[h], c.g3r[h], fma(-v.bi[h], c.g3i[h], c.g2r[h]));
        s.s1i[h] = fma(v.br[h], c.g3i[h], fma(v.bi[h], c.g3r[h], c.g2i[h]));
        s.s2r[h] = fma(v.gr[h], c.g2r[h], fma(-v.gi[h], c.g2i[h], -c.g3r[h]));
        s.s2i[h] = fma(v.gr[h], c.g2i[h], fma(v.gi[h], c.g2r[h], -c.g3i[h]));
    }
    return s;
}

// s += V' g for every variant, as one chain of fused multiply-adds per
// component (the pair sums of quad_close).
template <typename R, int H>
__device__ __forceinline__ void vertex_half_add(const Vert<R, H> &v, const Chain<R, H> &c, Half<R, H> &s)
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        s.s1r[h] = fma(v.br[h], c.g3r[h], fma(-v.bi[h], c.g3i[h], s.s1r[h] + c.g2r[h]));
        s.s1i[h] = fma(v.br[h], c.g3i[h], fma(v.bi[h], c.g3r[h], s.s1i[h] + c.g2i[h]));
        s.s2r[h] = fma(v.gr[h], c.g2r[h], fma(-v.gi[h], c.g2i[h], s.s2r[h] - c.g3r[h]));
        s.s2i[h] = fma(v.gr[h], c.g2i[h], fma(v.gi[h], c.g2r[h], s.s2i[h] - c.g3i[h]));
    }
}

// The propagator half: g' = d P(q') (sl1, sl2).
template <typename R, int H>
__device__ __forceinline__ void propagator_half(const Prop<R> &P, const Half<R, H> &s, Chain<R, H> &o)
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        o.g2r[h] = P.m * s.s1r[h] - P.x * s.s2r[h] + P.y * s.s2i[h];
        o.g2i[h] = P.m * s.s1i[h] - P.x * s.s2i[h] - P.y * s.s2r[h];
        o.g3r[h] = P.p * s.s2r[h] - P.x * s.s1r[h] - P.y * s.s1i[h];
        o.g3i[h] = P.p * s.s2i[h] - P.x * s.s1i[h] + P.y * s.s1r[h];
    }
}

// One fvoxx0 current update for every variant.
template <typename R, int H>
__device__ __forceinline__ void update(const Vert<R, H> &v, const Chain<R, H> &c, const Prop<R> &P,
                                       Chain<R, H> &o)
{
    propagator_half<R, H>(P, vertex_half<R, H>(v, c), o);
}

// Closing vertex (iovxx0 with the u spinor): amp = gamma g2 - g3, summed in FP64.
template <typename R, int H>
__device__ __forceinline__ void close_chain(const Vert<R, H> &v, const Chain<R, H> &c, Acc<H> &acc)
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const R ar = fma(v.gr[h], c.g2r[h], fma(-v.gi[h], c.g2i[h], -c.g3r[h]));
        const R ai = fma(v.gr[h], c.g2i[h], fma(v.gi[h], c.g2r[h], -c.g3i[h]));
        acc.re[h] += static_cast<double>(ar);
        acc.im[h] += static_cast<double>(ai);
    }
}

// Compile-time loop over the set bits of MASK, calling f(integral_constant<int, bit>).
template <unsigned MASK, int BIT = 0, typename F>
__device__ __forceinline__ void for_each_bit(F &&f)
{
    if constexpr (MASK != 0u) {
        if constexpr ((MASK & 1u) != 0u) f(std::integral_constant<int, BIT>{});
        for_each_bit<(MASK >> 1), BIT + 1>(static_cast<F &&>(f));
    }
}

// The u-end currents of the slot photons: w_r = c_r d(q_r) P(q_r) with
// q_r = p1 - k_r and c_r = (gamma_r, -1) (the current after photon r met the
// u spinor).
template <typename R, int H, int NS>
struct PairW {
    R w1r[NS][H], w1i[NS][H], w2r[NS][H], w2i[NS][H];
};

template <typename R, int H, int NS>
__device__ __forceinline__ void make_w(const Slots<R, H, NS> &S, const LMom<R> &p1, PairW<R, H, NS> &W)
{
#pragma unroll
    for (int r = 0; r < NS; ++r) {
        LMom<R> q;
        q.p = p1.p - S.k[r].p;
        q.m = p1.m - S.k[r].m;
        q.x = -S.k[r].x;
        q.y = -S.k[r].y;
        const R q2 = q.p * q.m - q.x * q.x - q.y * q.y;
        const R d = neg_recip(q2);
        const R Pm = d * q.m, Pp = d * q.p, Px = d * q.x, Py = d * q.y;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const R gr = S.v[r].gr[h], gi = S.v[r].gi[h];
            W.w1r[r][h] = fma(gr, Pm, Px);
            W.w1i[r][h] = fma(gi, Pm, -Py);
            W.w2r[r][h] = -(gr * Px - gi * Py) - Pp;
            W.w2i[r][h] = -(gr * Py + gi * Px);
        }
    }
}

// The pair vector U_ab = u_ab + u_ba for helicity variant h, u_jr = w_r V_j.
template <typename R, int H, int NS>
__device__ __forceinline__ void pair_u(const Slots<R, H, NS> &S, const PairW<R, H, NS> &W, int a, int b,
                                       int h, R &u1r, R &u1i, R &u2r, R &u2i)
{
    // u_ab = w_b V_a and u_ba = w_a V_b; V = [[1, beta], [gamma, -1]]
    const Vert<R, H> &va = S.v[a], &vb = S.v[b];
    const R x1r = fma(W.w2r[b][h], va.gr[h], fma(-W.w2i[b][h], va.gi[h], W.w1r[b][h]));
    const R x1i = fma(W.w2r[b][h], va.gi[h], fma(W.w2i[b][h], va.gr[h], W.w1i[b][h]));
    const R x2r = fma(W.w1r[b][h], va.br[h], fma(-W.w1i[b][h], va.bi[h], -W.w2r[b][h]));
    const R x2i = fma(W.w1r[b][h], va.bi[h], fma(W.w1i[b][h], va.br[h], -W.w2i[b][h]));
    // + u_ba, continued as fused multiply-adds on u_ab
    u1r = fma(W.w2r[a][h], vb.gr[h], fma(-W.w2i[a][h], vb.gi[h], x1r + W.w1r[a][h]));
    u1i = fma(W.w2r[a][h], vb.gi[h], fma(W.w2i[a][h], vb.gr[h], x1i + W.w1i[a][h]));
    u2r = fma(W.w1r[a][h], vb.br[h], fma(-W.w1i[a][h], vb.bi[h], x2r - W.w2r[a][h]));
    u2i = fma(W.w1r[a][h], vb.bi[h], fma(W.w1i[a][h], vb.br[h], x2i - W.w2i[a][h]));
}

// Table of every pair vector, built once per subtree entry.
template <typename R, int H, int NS>
struct PairTab {
    R u1r[NS][NS][H], u1i[NS][NS][H], u2r[NS][NS][H], u2i[NS][NS][H];
    __device__ __forceinline__ void get(int a, int b, int h, R &x1r, R &x1i, R &x2r, R &x2i) const
    {
        x1r = u1r[a][b][h];
        x1i = u1i[a][b][h];
        x2r = u2r[a][b][h];
        x2i = u2i[a][b][h];
    }
};

template <typename R, int H, int NS>
__device__ __forceinline__ void make_pairs(const Slots<R, H, NS> &S, const PairW<R, H, NS> &W,
                                           PairTab<R, H, NS> &T)
{
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int b = a + 1; b < NS; ++b)
#pragma unroll
            for (int h = 0; h < H; ++h)
                pair_u<R, H, NS>(S, W, a, b, h, T.u1r[a][b][h], T.u1i[a][b][h], T.u2r[a][b][h],
                                 T.u2i[a][b][h]);
}

// Pair vectors formed where they are used (a subtree whose every pair is
// closed once, as the four-photon subtree is).
template <typename R, int H, int NS>
struct PairLazy {
    const Slots<R, H, NS> &S;
    const PairW<R, H, NS> &W;
    __device__ __forceinline__ void get(int a, int b, int h, R &x1r, R &x1i, R &x2r, R &x2i) const
    {
        pair_u<R, H, NS>(S, W, a, b, h, x1r, x1i, x2r, x2i);
    }
};

// Close a node with slots a < b left: amp = U_ab . g, summed in FP64.
template <typename R, int H, typename PT>
__device__ __forceinline__ void close_pair(const PT &T, int a, int b, const Chain<R, H> &c, Acc<H> &acc)
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        R u1r, u1i, u2r, u2i;
        T.get(a, b, h, u1r, u1i, u2r, u2i);
        const R ar = u1r * c.g2r[h] - u1i * c.g2i[h] + u2r * c.g3r[h] - u2i * c.g3i[h];
        const R ai = u1r * c.g2i[h] + u1i * c.g2r[h] + u2r * c.g3i[h] + u2i * c.g3r[h];
        acc.re[h] += static_cast<double>(ar);
        acc.im[h] += static_cast<double>(ai);
    }
}

template <typename R, int H, typename PT>
__device__ __forceinline__ void close_pair_wide(const PT &T, int a, int b, const Chain<R, H> &c,
                                                Acc<H> &acc);

// The last four photons of every ordering below a node (slots in MASK,
// four of them) with pair sums at both ends (CL = 3).  The 24 orderings
// (x, y, a, b) group by the split {x, y} | {a, b}: the u end contributes the
// pair vector U_ab (both orders of a, b), the ubar end the sum of the
// currents after x then y and after y then x.  Those two currents carry the
// same momentum q + k_x + k_y, so they share their propagator:
//     G_xy = d P(q + k_x + k_y) [V_y g_x + V_x g_y],  g_x = current after x,
// and the node closes with six products U_ab . G_xy instead of twelve.
// CL = 3 takes each split's product in FP64 where H >= 8 (close_pair_wide);
// CL = 4 always in the working precision, converted once into the FP64 sum;
// CL = 5 sums the products of complementary splits, {x, y} | {a, b} and
// {a, b} | {x, y} (the eight orderings whose first two photons form either
// set), in the working precision and enters each such sum into the FP64
// ordering sum once: three FP64 entries per helicity instead of six.
template <typename R, int H, int NS, int CL, unsigned MASK, typename PT>
__device__ __forceinline__ void quad_close(const Slots<R, H, NS> &S, const PT &T, const Chain<R, H> &c,
                                           const LMom<R> &q, Acc<H> &acc)
{
    constexpr int s0 = __builtin_ctz(MASK);
    constexpr unsigned m1 = MASK & (MASK - 1u);
    constexpr int s1 = __builtin_ctz(m1);
    constexpr unsigned m2 = m1 & (m1 - 1u);
    constexpr int s2 = __builtin_ctz(m2);
    constexpr int s3 = __builtin_ctz(m2 & (m2 - 1u));
    constexpr int sl[4] = {s0, s1, s2, s3};
    Chain<R, H> g1[4];
    LMom<R> q1[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const Prop<R> P = propagate<R>(q, S.k[sl[i]], q1[i]);
        update<R, H>(S.v[sl[i]], c, P, g1[i]);
    }
    // (x, y) index pairs into sl and the closing pair (a, b) of the other two;
    // split 5 - t is the complement of split t
    constexpr int X[6] = {0, 0, 0, 1, 1, 2}, Y[6] = {1, 2, 3, 2, 3, 3};
    constexpr int A[6] = {2, 1, 1, 0, 0, 0}, B[6] = {3, 3, 2, 3, 2, 1};
    // G_xy of split t
    auto split_current = [&](int t) {
        LMom<R> q2;
        const Prop<R> P = propagate<R>(q1[X[t]], S.k[sl[Y[t]]], q2);
        Half<R, H> s = vertex_half<R, H>(S.v[sl[Y[t]]], g1[X[t]]);
        vertex_half_add<R, H>(S.v[sl[X[t]]], g1[Y[t]], s);
        Chain<R, H> g2;
        propagator_half<R, H>(P, s, g2);
        return g2;
    };
    if constexpr (CL == 5 && !std::is_same<R, double>::value) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const Chain<R, H> ga = split_current(t);
            const Chain<R, H> gb = split_current(5 - t);
#pragma unroll
            for (int h = 0; h < H; ++h) {
                R u1r, u1i, u2r, u2i, v1r, v1i, v2r, v2i;
                T.get(sl[A[t]], sl[B[t]], h, u1r, u1i, u2r, u2i);
                T.get(sl[A[5 - t]], sl[B[5 - t]], h, v1r, v1i, v2r, v2i);
                R ar = u1r * ga.g2r[h];
                ar = fma(-u1i, ga.g2i[h], ar);
                ar = fma(u2r, ga.g3r[h], ar);
                ar = fma(-u2i, ga.g3i[h], ar);
                ar = fma(v1r, gb.g2r[h], ar);
                ar = fma(-v1i, gb.g2i[h], ar);
                ar = fma(v2r, gb.g3r[h], ar);
                ar = fma(-v2i, gb.g3i[h], ar);
                R ai = u1r * ga.g2i[h];
                ai = fma(u1i, ga.g2r[h], ai);
                ai = fma(u2r, ga.g3i[h], ai);
                ai = fma(u2i, ga.g3r[h], ai);
                ai = fma(v1r, gb.g2i[h], ai);
                ai = fma(v1i, gb.g2r[h], ai);
                ai = fma(v2r, gb.g3i[h], ai);
                ai = fma(v2i, gb.g3r[h], ai);
                acc.re[h] += static_cast<double>(ar);
                acc.im[h] += static_cast<double>(ai);
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const Chain<R, H> g2 = split_current(t);
            // FP64 products pay off where a split's conversions are shared by
            // many configurations and FP64 issues as fast as FP32 (and always in
            // FP64, where there are none)
            if constexpr (std::is_same<R, double>::value || (H >= 8 && CL == 3))
                close_pair_wide<R, H>(T, sl[A[t]], sl[B[t]], g2, acc);
            else
                close_pair<R, H>(T, sl[A[t]], sl[B[t]], g2, acc);
        }
    }
}

// Close a node with slots a < b left as close_pair does, with the product
// taken in FP64: the FP32 factors convert exactly and every product of two
// is exact in FP64, so each split enters the FP64 ordering sum through fused
// multiply-adds, with no FP32 rounding of its own.  In quad_close the
// conversions of the four pair vectors and four currents of a split are
// shared by up to sixteen helicity configurations, which makes this cheaper
// than an FP32 product followed by a conversion and an FP64 add.
template <typename R, int H, typename PT>
__device__ __forceinline__ void close_pair_wide(const PT &T, int a, int b, const Chain<R, H> &c,
                                                Acc<H> &acc)
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        R x1r, x1i, x2r, x2i;
        T.get(a, b, h, x1r, x1i, x2r, x2i);
        const double u1r = x1r, u1i = x1i, u2r = x2r, u2i = x2i;
        const double g2r = c.g2r[h], g2i = c.g2i[h], g3r = c.g3r[h], g3i = c.g3i[h];
        acc.re[h] = fma(u1r, g2r, fma(-u1i, g2i, fma(u2r, g3r, fma(-u2i, g3i, acc.re[h]))));
        acc.im[h] = fma(u1r, g2i, fma(u1i, g2r, fma(u2r, g3i, fma(u2i, g3r, acc.im[h]))));
    }
}

// Unrolled subtree over the slot photons in MASK, entered with current c at
// momentum q.  CL = 1 closes photon by photon; CL = 2 closes the last pair;
// CL = 3, 4 and 5 close the last four photons with pair sums at both ends.
template <typename R, int H, int NS, int CL, unsigned MASK, typename PT>
__device__ __forceinline__ void subtree(const Slots<R, H, NS> &S, const PT &T, const Chain<R, H> &c,
                                        const LMom<R> &q, Acc<H> &acc)
{
    if constexpr (CL == 1 && __builtin_popcount(MASK) == 1) {
        close_chain<R, H>(S.v[__builtin_ctz(MASK)], c, acc);
    } else if constexpr (CL >= 3 && __builtin_popcount(MASK) == 4) {
        quad_close<R, H, NS, CL, MASK>(S, T, c, q, acc);
    } else if constexpr (CL >= 2 && __builtin_popcount(MASK) == 2) {
        constexpr int a = __builtin_ctz(MASK);
        constexpr int b = __builtin_ctz(MASK & (MASK - 1u));
        close_pair<R, H>(T, a, b, c, acc);
    } else {
        for_each_bit<MASK>([&](auto bit) {
            constexpr int s = decltype(bit)::value;
            LMom<R> qn;
            const Prop<R> P = propagate<R>(q, S.k[s], qn);
            Chain<R, H> cn;
            update<R, H>(S.v[s], c, P, cn);
            subtree<R, H, NS, CL, (MASK & ~(1u << s))>(S, T, cn, qn, acc);
        });
    }
}

// Enter a subtree over all NS slots (forms the u-end currents first for CL >= 2).
template <typename R, int H, int NS, int CL>
__device__ __forceinline__ void run_subtree(const Slots<R, H, NS> &S, const LMom<R> &p1,
                                            const Chain<R, H> &c, const LMom<R> &q, Acc<H> &acc)
{
    if constexpr (CL >= 2) {
        PairW<R, H, NS> W;
        make_w<R, H, NS>(S, p1, W);
        if constexpr (NS == 4 && CL >= 3) {
            // every pair of a four-photon subtree closes exactly once: form
            // each pair vector where it is used instead of holding the table
            const PairLazy<R, H, NS> T{S, W};
            subtree<R, H, NS, CL, (1u << NS) - 1u>(S, T, c, q, acc);
        } else {
            PairTab<R, H, NS> T;
            make_pairs<R, H, NS>(S, W, T);
            subtree<R, H, NS, CL, (1u << NS) - 1u>(S, T, c, q, acc);
        }
    } else {
        subtree<R, H, NS, CL, (1u << NS) - 1u>(S, NoPairs{}, c, q, acc);
    }
}

// LDS photon table of one wave: [field 0..5][photon][lane] = (k+, k-, kx, ky, 1/k+, 1/k-).
constexpr int kPhotonFields = 6;

template <typename R, int N>
__device__ __forceinline__ LMom<R> lds_photon(const R *tab, int j, int lane)
{
    const R *b = tab + j * 64 + lane;
    return {b[0], b[N * 64], b[2 * N * 64], b[3 * N * 64], b[4 * N * 64], b[5 * N * 64]};
}

// Wave-uniform walk of the top n-MB levels.  `rem` = photons not yet used.
template <typename R, int N, int MB, int H, int CL, int DEPTH>
__device__ __forceinline__ void top_levels(const R *tab, int lane, uint32_t rem, uint32_t cfg0,
                                           const LMom<R> &p1, const Chain<R, H> &c,
                                           const LMom<R> &q, Acc<H> &acc)
{
    // kept as a loop (not unrolled even where rem is a constant): the walk stays
    // compact and register pressure stays that of one subtree
#pragma nounroll
    for (uint32_t left = rem; left != 0u; left &= left - 1u) {
        const int j = __builtin_ctz(left);
        const LMom<R> k = lds_photon<R, N>(tab, j, lane);
        const Vert<R, H> v = make_vert<R, H>(k, cfg0, j);
        LMom<R> qn;
        const Prop<R> P = propagate<R>(q, k, qn);
        Chain<R, H> cn;
        update<R, H>(v, c, P, cn);
        const uint32_t rest = rem & ~(1u << j);
        if constexpr (N - DEPTH - 1 == MB) {
            Slots<R, H, MB> S;
            uint32_t m = rest;
#pragma unroll
            for (int s = 0; s < MB; ++s) {
                const int js = __builtin_ctz(m);
                m &= m - 1u;
                S.k[s] = lds_photon<R, N>(tab, js, lane);
                S.v[s] = make_vert<R, H>(S.k[s], cfg0, js);
            }
            run_subtree<R, H, MB, CL>(S, p1, cn, qn, acc);
        } else {
            top_levels<R, N, MB, H, CL, DEPTH + 1>(tab, lane, rest, cfg0, p1, cn, qn, acc);
        }
    }
}

// Compile-time loop over I = B .. E-1, calling f(integral_constant<int, I>).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(static_cast<F &&>(f));
    }
}

// The next bitmask with the same number of set bits (Gosper's rule,
// HAKMEM item 175): subsets of one size in increasing order.
__device__ __forceinline__ uint32_t next_subset(uint32_t v)
{
    const uint32_t t = v | (v - 1u);
    return (t + 1u) | (((~t & (t + 1u)) - 1u) >> (__builtin_ctz(v) + 1));
}

// Prefix sets (shape field prefix_sets = 1) for the top n-MB levels.  Every
// ordering of the same prefix set P reaches the subtree over the remaining
// photons with the same momentum -p2 + sum_{i in P} k_i, and the subtree is
// linear in the current it is entered with.  So the currents of all orderings
// of P are summed first and the subtree runs once per set, C(n, n-MB) times
// instead of n!/MB! times.  The sum is the subset recursion over the subsets
// Q of P (momenta q_Q = -p2 + sum_{i in Q} k_i, J(empty) = the vbar current):
//     J(Q) = d(q_Q) P(q_Q) sum_{j in Q} V_j J(Q \ j),
// one propagator per subset for the vertex halves of all its last photons,
// as the four-photon closing does for its pairs.  The sums over the orderings
// of P are taken in the working precision; the subtree's closings enter the
// FP64 ordering sum as before.
template <typename R, int N, int MB, int H, int CL>
__device__ __forceinline__ void prefix_sets(const R *tab, int lane, uint32_t cfg0, const LMom<R> &p1,
                                            const Chain<R, H> &c0, const LMom<R> &q0, Acc<H> &acc)
{
    constexpr int K = N - MB;
    constexpr uint32_t kFull = (1u << K) - 1u;
#pragma nounroll
    for (uint32_t set = kFull; set < (1u << N); set = next_subset(set)) {
        LMom<R> kq[K];
        Vert<R, H> vq[K];
        uint32_t m = set;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int j = __builtin_ctz(m);
            m &= m - 1u;
            kq[s] = lds_photon<R, N>(tab, j, lane);
            vq[s] = make_vert<R, H>(kq[s], cfg0, j);
        }
        Chain<R, H> J[1 << K];
        LMom<R> q[1 << K];
        J[0] = c0;
        q[0] = q0;
        // every proper subset precedes its supersets in increasing order
        static_for<1, (1 << K)>([&](auto mi) {
            constexpr uint32_t mask = decltype(mi)::value;
            constexpr int low = __builtin_ctz(mask);
            const LMom<R> &qb = q[mask & (mask - 1u)];
            q[mask] = {qb.p + kq[low].p, qb.m + kq[low].m, qb.x + kq[low].x, qb.y + kq[low].y, R(0), R(0)};
            Half<R, H> sl = vertex_half<R, H>(vq[low], J[mask & ~(1u << low)]);
            for_each_bit<(mask & (mask - 1u))>([&](auto bit) {
                constexpr int b = decltype(bit)::value;
                vertex_half_add<R, H>(vq[b], J[mask & ~(1u << b)], sl);
            });
            propagator_half<R, H>(prop_at<R>(q[mask]), sl, J[mask]);
        });
        const uint32_t rest = ((1u << N) - 1u) & ~set;
        Slots<R, H, MB> S;
        m = rest;
#pragma unroll
        for (int s = 0; s < MB; ++s) {
            const int js = __builtin_ctz(m);
            m &= m - 1u;
            S.k[s] = lds_photon<R, N>(tab, js, lane);
            S.v[s] = make_vert<R, H>(S.k[s], cfg0, js);
        }
        run_subtree<R, H, MB, CL>(S, p1, J[kFull], q[kFull], acc);
    }
}

// Row vector of the u end (a current flowing towards the u spinor) for H
// variants: (r1, r2) complex, contracted with a v-bar-end current g as
// r1 g2 + r2 g3.
template <typename R, int H>
struct Row {
    R r1r[H], r1i[H], r2r[H], r2i[H];
};

// s = r V' for every variant (V' = [[1, beta], [gamma, -1]]), started or added.
template <typename R, int H>
__device__ __forceinline__ Half<R, H> row_vertex(const Vert<R, H> &v, const Row<R, H> &r)
{
    Half<R, H> s;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        s.s1r[h] = fma(v.gr[h], r.r2r[h], fma(-v.gi[h], r.r2i[h], r.r1r[h]));
        s.s1i[h] = fma(v.gr[h], r.r2i[h], fma(v.gi[h], r.r2r[h], r.r1i[h]));
        s.s2r[h] = fma(v.br[h], r.r1r[h], fma(-v.bi[h], r.r1i[h], -r.r2r[h]));
        s.s2i[h] = fma(v.br[h], r.r1i[h], fma(v.bi[h], r.r1r[h], -r.r2i[h]));
    }
    return s;
}

template <typename R, int H>
__device__ __forceinline__ void row_vertex_add(const Vert<R, H> &v, const Row<R, H> &r, Half<R, H> &s)
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        s.s1r[h] = fma(v.gr[h], r.r2r[h], fma(-v.gi[h], r.r2i[h], s.s1r[h] + r.r1r[h]));
        s.s1i[h] = fma(v.gr[h], r.r2i[h], fma(v.gi[h], r.r2r[h], s.s1i[h] + r.r1i[h]));
        s.s2r[h] = fma(v.br[h], r.r1r[h], fma(-v.bi[h], r.r1i[h], s.s2r[h] - r.r2r[h]));
        s.s2i[h] = fma(v.br[h], r.r1i[h], fma(v.bi[h], r.r1r[h], s.s2i[h] - r.r2i[h]));
    }
}

// r' = s d P(q) for a row: P(q) = [[q-, -(qx + i qy)], [-(qx - i qy), q+]]
// acts from the right.
template <typename R, int H>
__device__ __forceinline__ void row_propagator(const Prop<R> &P, const Half<R, H> &s, Row<R, H> &o)
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        o.r1r[h] = P.m * s.s1r[h] - P.x * s.s2r[h] - P.y * s.s2i[h];
        o.r1i[h] = P.m * s.s1i[h] - P.x * s.s2i[h] + P.y * s.s2r[h];
        o.r2r[h] = P.p * s.s2r[h] - P.x * s.s1r[h] + P.y * s.s1i[h];
        o.r2i[h] = P.p * s.s2i[h] - P.x * s.s1i[h] - P.y * s.s1r[h];
    }
}

// Momentum base + SIGN * sum of the photons in MASK (in increasing photon order).
template <int SIGN, unsigned MASK, typename R, int H, int N>
__device__ __forceinline__ LMom<R> set_momentum(const LMom<R> &base, const Slots<R, H, N> &S)
{
    LMom<R> q = {base.p, base.m, base.x, base.y, R(0), R(0)};
    for_each_bit<MASK>([&](auto bit) {
        constexpr int b = decltype(bit)::value;
        if constexpr (SIGN > 0) {
            q.p += S.k[b].p, q.m += S.k[b].m, q.x += S.k[b].x, q.y += S.k[b].y;
        } else {
            q.p -= S.k[b].p, q.m -= S.k[b].m, q.x -= S.k[b].x, q.y -= S.k[b].y;
        }
    });
    return q;
}

// Compile-time loop over the masks of n bits with L bits set, in increasing order.
template <int N, int L, typename F>
__device__ __forceinline__ void for_each_subset(F &&f)
{
    static_for<1, (1 << N)>([&](auto mi) {
        constexpr uint32_t mask = decltype(mi)::value;
        if constexpr (__builtin_popcount(mask) == L) f(std::integral_constant<uint32_t, mask>{});
    });
}

// Rank of MASK among the n-bit masks with as many bits set (increasing order).
template <int N>
constexpr int subset_rank(uint32_t mask)
{
    int r = 0;
    for (uint32_t m = 1; m < mask; ++m) r += __builtin_popcount(m) == __builtin_popcount(mask);
    return r;
}

constexpr int binomial(int n, int k)
{
    int r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// The i-th mask with k bits set, in increasing order (Gosper's rule).
constexpr uint32_t nth_subset(int k, int i)
{
    uint32_t v = (1u << k) - 1u;
    for (int t = 0; t < i; ++t) {
        const uint32_t c = v | (v - 1u);
        v = (c + 1u) | (((~c & (c + 1u)) - 1u) >> (__builtin_ctz(v) + 1));
    }
    return v;
}

// Index of the j-th set bit of m (j = 0: the lowest).
constexpr int nth_bit(uint32_t m, int j)
{
    for (int t = 0; t < j; ++t) m &= m - 1u;
    return __builtin_ctz(m);
}

// LDS values per lane of meet_sets with LDS staging: the v-bar-end currents of
// level K - 1, 4 H components each.
template <int N, int H>
constexpr int meet_lds_values()
{
    return binomial(N, (N + 1) / 2 - 1) * 4 * H;
}

// Level-(K - 1) current of set MASK in the wave's LDS region:
// [rank][component][lane], component c of variant h at 4 h + c.
template <typename R, int N, int H, uint32_t MASK>
__device__ __forceinline__ void lds_put(R *lds, int lane, const Chain<R, H> &c)
{
    R *b = lds + subset_rank<N>(MASK) * 4 * H * 64 + lane;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        b[(4 * h + 0) * 64] = c.g2r[h];
        b[(4 * h + 1) * 64] = c.g2i[h];
        b[(4 * h + 2) * 64] = c.g3r[h];
        b[(4 * h + 3) * 64] = c.g3i[h];
    }
}

template <typename R, int N, int H, uint32_t MASK>
__device__ __forceinline__ Chain<R, H> lds_get(const R *lds, int lane)
{
    const R *b = lds + subset_rank<N>(MASK) * 4 * H * 64 + lane;
    Chain<R, H> c;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        c.g2r[h] = b[(4 * h + 0) * 64];
        c.g2i[h] = b[(4 * h + 1) * 64];
        c.g3r[h] = b[(4 * h + 2) * 64];
        c.g3i[h] = b[(4 * h + 3) * 64];
    }
    return c;
}

// Meet in the middle (shape field prefix_sets = 2, 3, 4; the whole tree
// unrolled, photons in registers).  Every ordering of the n photons splits
// uniquely into the set A of its first K photons (from the v-bar end) and the
// set B of the other n - K, and its amplitude factorises at the propagator
// between them:
// the v-bar-end current after A times the u-end row vector arriving from B.
// Summed over the orderings of A and of B,
//     sum over all orderings = sum over |A| = K of W(B) . J(A),
//     J(Q) = d(q_Q) P(q_Q) sum_{j in Q} V_j J(Q \ j),  q_Q = -p2 + sum_Q k,
//     R(C) = [sum_{c in C} R(C \ c) V_c] d(p1 - sum_C k) P(p1 - sum_C k),
//     W(B) = sum_{b in B} R(B \ b) V_b,
// with J(empty) the v-bar spinor and R(empty) V_c = (gamma_c, -1) the u-end
// closing vertex.  This is the two-sided current reuse of the MadGraph program
// (Appendix A.1) taken to the middle of every chain: each subset current is
// formed once per helicity walk instead of once per ordering prefix.  The
// C(n, K) contractions W(B) . J(A) are taken in the working precision and
// each enters the FP64 ordering sum.  Levels up to K - 1 (v-bar end) and
// n - K - 1 (u end) are held; level K and the row vectors W are formed at the
// contraction that uses them.  With kLds the v-bar-end currents of level
// K - 1 go to the wave's LDS region `lds` (meet_lds_values<N, H>() values per
// lane) instead of registers, for the shapes whose held currents would not
// fit in registers.
template <typename R, int N, int K, int H, bool kLds = false>
__device__ __forceinline__ void meet_sets(const Slots<R, H, N> &S, const LMom<R> &p1, const LMom<R> &q0,
                                          Acc<H> &acc, R *lds = nullptr, int lane = 0)
{
    static_assert(K >= 2 && N - K >= 2, "both ends need at least two photons");
    constexpr uint32_t kAll = (1u << N) - 1u;
    constexpr int kU = N - K;
    Chain<R, H> J[1 << N];
    Row<R, H> Rw[1 << N];
    // v-bar end, level by level (a level's currents die once the next is formed)
    static_for<1, K>([&](auto li) {
        constexpr int L = decltype(li)::value;
        for_each_subset<N, L>([&](auto mi) {
            constexpr uint32_t mask = decltype(mi)::value;
            constexpr int low = __builtin_ctz(mask);
            const Prop<R> P = prop_at<R>(set_momentum<1, mask>(q0, S));
            if constexpr (L == 1) {
                // V (1, 0) = (1, gamma)
                const Vert<R, H> &v = S.v[low];
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    J[mask].g2r[h] = fma(-P.x, v.gr[h], fma(P.y, v.gi[h], P.m));
                    J[mask].g2i[h] = -fma(P.x, v.gi[h], P.y * v.gr[h]);
                    J[mask].g3r[h] = fma(P.p, v.gr[h], -P.x);
                    J[mask].g3i[h] = fma(P.p, v.gi[h], P.y);
                }
            } else {
                Half<R, H> sl = vertex_half<R, H>(S.v[low], J[mask & ~(1u << low)]);
                for_each_bit<(mask & (mask - 1u))>([&](auto bit) {
                    constexpr int b = decltype(bit)::value;
                    vertex_half_add<R, H>(S.v[b], J[mask & ~(1u << b)], sl);
                });
                propagator_half<R, H>(P, sl, J[mask]);
            }
            if constexpr (kLds && L == K - 1) lds_put<R, N, H, mask>(lds, lane, J[mask]);
            if constexpr (kLds) __builtin_amdgcn_sched_barrier(0);
        });
    });
    // u end, levels 1 .. n - K - 1
    static_for<1, kU>([&](auto li) {
        constexpr int L = decltype(li)::value;
        for_each_subset<N, L>([&](auto mi) {
            constexpr uint32_t mask = decltype(mi)::value;
            constexpr int low = __builtin_ctz(mask);
            const Prop<R> P = prop_at<R>(set_momentum<-1, mask>(p1, S));
            if constexpr (L == 1) {
                // (gamma, -1) d P(p1 - k): the u-end current after one photon
                const Vert<R, H> &v = S.v[low];
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    Rw[mask].r1r[h] = fma(v.gr[h], P.m, P.x);
                    Rw[mask].r1i[h] = fma(v.gi[h], P.m, -P.y);
                    Rw[mask].r2r[h] = -fma(v.gr[h], P.x, fma(-v.gi[h], P.y, P.p));
                    Rw[mask].r2i[h] = -fma(v.gr[h], P.y, v.gi[h] * P.x);
                }
            } else {
                Half<R, H> sl = row_vertex<R, H>(S.v[low], Rw[mask & ~(1u << low)]);
                for_each_bit<(mask & (mask - 1u))>([&](auto bit) {
                    constexpr int b = decltype(bit)::value;
                    row_vertex_add<R, H>(S.v[b], Rw[mask & ~(1u << b)], sl);
                });
                row_propagator<R, H>(P, sl, Rw[mask]);
            }
            if constexpr (kLds) __builtin_amdgcn_sched_barrier(0);
        });
    });
    // the contraction of set A, given the currents of A minus each of its
    // photons (hA[j]: A without its j-th photon)
    auto contract = [&](auto ai, const Chain<R, H> (&hA)[K]) {
        constexpr uint32_t A = decltype(ai)::value;
        constexpr uint32_t B = kAll & ~A;
        Half<R, H> sl = vertex_half<R, H>(S.v[nth_bit(A, 0)], hA[0]);
        static_for<1, K>([&](auto ji) {
            constexpr int j = decltype(ji)::value;
            vertex_half_add<R, H>(S.v[nth_bit(A, j)], hA[j], sl);
        });
        Chain<R, H> ja;
        propagator_half<R, H>(prop_at<R>(set_momentum<1, A>(q0, S)), sl, ja);
        constexpr int lowb = __builtin_ctz(B);
        Half<R, H> w = row_vertex<R, H>(S.v[lowb], Rw[B & ~(1u << lowb)]);
        for_each_bit<(B & (B - 1u))>([&](auto bit) {
            constexpr int b = decltype(bit)::value;
            row_vertex_add<R, H>(S.v[b], Rw[B & ~(1u << b)], w);
        });
#pragma unroll
        for (int h = 0; h < H; ++h) {
            R ar = w.s1r[h] * ja.g2r[h];
            ar = fma(-w.s1i[h], ja.g2i[h], ar);
            ar = fma(w.s2r[h], ja.g3r[h], ar);
            ar = fma(-w.s2i[h], ja.g3i[h], ar);
            R ai = w.s1r[h] * ja.g2i[h];
            ai = fma(w.s1i[h], ja.g2r[h], ai);
            ai = fma(w.s2r[h], ja.g3i[h], ai);
            ai = fma(w.s2i[h], ja.g3r[h], ai);
            acc.re[h] += static_cast<double>(ar);
            acc.im[h] += static_cast<double>(ai);
        }
    };
    // the contractions, one per set A of K photons in increasing order
    constexpr int kSets = binomial(N, K);
    if constexpr (kLds) {
        // the held currents of the next set are read from LDS before the
        // current contraction, so the reads overlap its arithmetic; no
        // instruction moves across a contraction (the scheduler would
        // otherwise hoist later contractions' reads and products and hold
        // their values together)
        auto load_set = [&](auto ai, Chain<R, H>(&dst)[K]) {
            constexpr uint32_t A = nth_subset(K, decltype(ai)::value);
            static_for<0, K>([&](auto ji) {
                constexpr int j = decltype(ji)::value;
                dst[j] = lds_get<R, N, H, (A & ~(1u << nth_bit(A, j)))>(lds, lane);
            });
        };
        Chain<R, H> cur[K];
        load_set(std::integral_constant<int, 0>{}, cur);
        static_for<0, kSets>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            Chain<R, H> nxt[K];
            if constexpr (i + 1 < kSets) load_set(std::integral_constant<int, i + 1>{}, nxt);
            contract(std::integral_constant<uint32_t, nth_subset(K, i)>{}, cur);
            if constexpr (i + 1 < kSets) {
#pragma unroll
                for (int j = 0; j < K; ++j) cur[j] = nxt[j];
            }
            __builtin_amdgcn_sched_barrier(0);
        });
    } else {
        static_for<0, kSets>([&](auto ii) {
            constexpr uint32_t A = nth_subset(K, decltype(ii)::value);
            Chain<R, H> hA[K];
            static_for<0, K>([&](auto ji) {
                constexpr int j = decltype(ji)::value;
                hA[j] = J[A & ~(1u << nth_bit(A, j))];
            });
            contract(std::integral_constant<uint32_t, A>{}, hA);
        });
    }
}

// Per-point inputs after the FP64 set-up.
template <typename R, int N>
struct PointIn {
    LMom<R> k[N];   // scaled photon momenta
    LMom<R> q0;     // -p2, scaled
    LMom<R> p1;     // p1, scaled (pair closing)
};

// Sum over helicity passes [pass0, pass1) of |ordering sum|^2 (scaled units,
// without the external normalisations).  Each pass covers H configurations.
template <typename R, int N, int MB, int H, int CL, int PS = 0>
__device__ __forceinline__ double tree_sum(const PointIn<R, N> &in, R *tab, int lane, int pass0,
                                           int pass1)
{
    double total = 0.0;
    Chain<R, H> c0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        c0.g2r[h] = R(1);
        c0.g2i[h] = R(0);
        c0.g3r[h] = R(0);
        c0.g3i[h] = R(0);
    }
    for (int pass = pass0; pass < pass1; ++pass) {
        const uint32_t cfg0 = static_cast<uint32_t>(pass) * H;
        Acc<H> acc;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            acc.re[h] = 0.0;
            acc.im[h] = 0.0;
        }
        if constexpr (PS >= 2) {
            static_assert(N <= MB, "meeting in the middle keeps every photon in registers");
            // PS = 2 leaves it to the compiler where the momentum part of the
            // nodes (the same in every pass) is formed: it hoists it out of
            // the pass loop and holds all of it across.  PS = 3 and 4 hide the
            // momenta behind empty asm statements, so that part is formed per
            // pass next to its use (for walks whose held values would
            // otherwise not fit in registers); PS = 4 also holds the v-bar-end
            // currents of level K - 1 in LDS.
            Slots<R, H, N> S;
            LMom<R> p1 = in.p1, q0 = in.q0;
#pragma unroll
            for (int s = 0; s < N; ++s) {
                S.k[s] = in.k[s];
                if constexpr (PS >= 3)
                    asm volatile("" : "+v"(S.k[s].p), "+v"(S.k[s].m), "+v"(S.k[s].x), "+v"(S.k[s].y));
                S.v[s] = make_vert<R, H>(in.k[s], cfg0, s);
            }
            if constexpr (PS >= 3) asm volatile("" : "+v"(p1.p), "+v"(p1.m), "+v"(q0.p), "+v"(q0.m));
            meet_sets<R, N, (N + 1) / 2, H, PS == 4>(S, p1, q0, acc, tab, lane);
        } else if constexpr (N <= MB) {
            Slots<R, H, N> S;
#pragma unroll
            for (int s = 0; s < N; ++s) {
                S.k[s] = in.k[s];
                S.v[s] = make_vert<R, H>(in.k[s], cfg0, s);
            }
            run_subtree<R, H, N, CL>(S, in.p1, c0, in.q0, acc);
        } else if constexpr (PS == 1 && N - MB >= 2) {
            prefix_sets<R, N, MB, H, CL>(tab, lane, cfg0, in.p1, c0, in.q0, acc);
        } else {
            top_levels<R, N, MB, H, CL, 0>(tab, lane, (1u << N) - 1u, cfg0, in.p1, c0, in.q0, acc);
        }
#pragma unroll
        for (int h = 0; h < H; ++h) total += acc.re[h] * acc.re[h] + acc.im[h] * acc.im[h];
    }
    return total;
}

// One walk per lane with the lane's own helicity configuration `cfg` (bit j
// set = photon j has helicity +1): |ordering sum|^2 of that configuration
// (scaled units, without the external normalisations).
template <typename R, int N, int MB, int CL, int PS = 0>
__device__ __forceinline__ double tree_one(const PointIn<R, N> &in, R *tab, int lane, uint32_t cfg)
{
    Chain<R, 1> c0;
    c0.g2r[0] = R(1);
    c0.g2i[0] = R(0);
    c0.g3r[0] = R(0);
    c0.g3i[0] = R(0);
    Acc<1> acc;
    acc.re[0] = 0.0;
    acc.im[0] = 0.0;
    if constexpr (PS >= 2) {
        static_assert(N <= MB, "meeting in the middle keeps every photon in registers");
        Slots<R, 1, N> S;
#pragma unroll
        for (int s = 0; s < N; ++s) {
            S.k[s] = in.k[s];
            S.v[s] = make_vert<R, 1>(in.k[s], cfg, s);
        }
        meet_sets<R, N, (N + 1) / 2, 1, PS == 4>(S, in.p1, in.q0, acc, tab, lane);
    } else if constexpr (N <= MB) {
        Slots<R, 1, N> S;
#pragma unroll
        for (int s = 0; s < N; ++s) {
            S.k[s] = in.k[s];
            S.v[s] = make_vert<R, 1>(in.k[s], cfg, s);
        }
        run_subtree<R, 1, N, CL>(S, in.p1, c0, in.q0, acc);
    } else if constexpr (PS == 1 && N - MB >= 2) {
        prefix_sets<R, N, MB, 1, CL>(tab, lane, cfg, in.p1, c0, in.q0, acc);
    } else {
        top_levels<R, N, MB, 1, CL, 0>(tab, lane, (1u << N) - 1u, cfg, in.p1, c0, in.q0, acc);
    }
    return acc.re[0] * acc.re[0] + acc.im[0] * acc.im[0];
}

}  // namespace heget
