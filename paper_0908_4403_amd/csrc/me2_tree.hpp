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
//    The tree builds V = t V' from the momentum and t ~ 1/(sqrt(2) E pT)
//    rounded to the working precision; every diagram contains each photon
//    once, so the exact factor (1/(sqrt(2) E pT t))^2 per photon is applied
//    to |M|^2 in FP64 at the end and the rounding of t cancels.
//  * The ubar spinor of oxxxx2 is (0, 0, -sqrt(2 E2), 0) and the u spinor of
//    ixxxx1 is (0, sqrt(E1 + p1z), 0, 0); their sizes are pulled out too, so
//    the chain starts at g = (1, 0) and closes with amp = gamma g2 - a3 g3.
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

// Light-cone momentum: p = E + z, m = E - z, x, y; for photons t is the
// vertex normalisation ~ 1/(sqrt(2) E pT) (unused for internal momenta).
template <typename R>
struct LMom {
    R p, m, x, y, t;
};

// Chain currents (g2, g3) for H helicity variants.
template <typename R, int H>
struct Chain {
    R g2r[H], g2i[H], g3r[H], g3i[H];
};

// Vertex block V' = [[a3, beta], [gamma, -a3]] for H variants.
template <typename R, int H>
struct Vert {
    R a3[H], br[H], bi[H], gr[H], gi[H];
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

// Pair-closing row vectors U_ab (a < b) for the slot photons, per variant.
template <typename R, int H, int NS>
struct PairTab {
    R u1r[NS][NS][H], u1i[NS][NS][H], u2r[NS][NS][H], u2i[NS][NS][H];
};

// Unused placeholder when the walk closes photon by photon (CL = 1).
struct NoPairs {};

// V'(lam) of photon j for the H variants whose helicity configurations are
// cfg0 .. cfg0+H-1 (bit j set = helicity +1).  cfg0 is wave-uniform.
template <typename R, int H>
__device__ __forceinline__ Vert<R, H> make_vert(const LMom<R> &k, uint32_t cfg0, int j)
{
    Vert<R, H> v;
    const R tp = k.t * k.p, tm = k.t * k.m;
    const R a3 = tp * k.m;  // t pT^2
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const bool plus = ((cfg0 + h) >> j) & 1u;
        const R cb = plus ? tp : tm;  // coefficient of -kappa in beta
        const R cg = plus ? tm : tp;  // coefficient of conj(kappa) in gamma
        v.a3[h] = plus ? a3 : -a3;
        v.br[h] = -cb * k.x;
        v.bi[h] = -cb * k.y;
        v.gr[h] = cg * k.x;
        v.gi[h] = -cg * k.y;
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

template <typename R>
__device__ __forceinline__ Prop<R> propagate(const LMom<R> &q, const LMom<R> &k, LMom<R> &qn)
{
    qn.p = q.p + k.p;
    qn.m = q.m + k.m;
    qn.x = q.x + k.x;
    qn.y = q.y + k.y;
    qn.t = R(0);
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
        s.s1r[h] = v.a3[h] * c.g2r[h] + v.br[h] * c.g3r[h] - v.bi[h] * c.g3i[h];
        s.s1i[h] = v.a3[h] * c.g2i[h] + v.br[h] * c.g3i[h] + v.bi[h] * c.g3r[h];
        s.s2r[h] = v.gr[h] * c.g2r[h] - v.gi[h] * c.g2i[h] - v.a3[h] * c.g3r[h];
        s.s2i[h] = v.gr[h] * c.g2i[h] + v.gi[h] * c.g2r[h] - v.a3[h] * c.g3i[h];
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
        s.s1r[h] = fma(v.a3[h], c.g2r[h], fma(v.br[h], c.g3r[h], fma(-v.bi[h], c.g3i[h], s.s1r[h])));
        s.s1i[h] = fma(v.a3[h], c.g2i[h], fma(v.br[h], c.g3i[h], fma(v.bi[h], c.g3r[h], s.s1i[h])));
        s.s2r[h] = fma(v.gr[h], c.g2r[h], fma(-v.gi[h], c.g2i[h], fma(-v.a3[h], c.g3r[h], s.s2r[h])));
        s.s2i[h] = fma(v.gr[h], c.g2i[h], fma(v.gi[h], c.g2r[h], fma(-v.a3[h], c.g3i[h], s.s2i[h])));
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

// Closing vertex (iovxx0 with the u spinor): amp = gamma g2 - a3 g3, summed in FP64.
template <typename R, int H>
__device__ __forceinline__ void close_chain(const Vert<R, H> &v, const Chain<R, H> &c, Acc<H> &acc)
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const R ar = v.gr[h] * c.g2r[h] - v.gi[h] * c.g2i[h] - v.a3[h] * c.g3r[h];
        const R ai = v.gr[h] * c.g2i[h] + v.gi[h] * c.g2r[h] - v.a3[h] * c.g3i[h];
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

// Pair vectors of the slot photons: w_r = c_r d(q_r) P(q_r) with q_r = p1 - k_r,
// u_jr = w_r V_j, U_jr = u_jr + u_rj.
template <typename R, int H, int NS>
__device__ __forceinline__ void make_pairs(const Slots<R, H, NS> &S, const LMom<R> &p1,
                                           PairTab<R, H, NS> &T)
{
    R w1r[NS][H], w1i[NS][H], w2r[NS][H], w2i[NS][H];
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
            const R gr = S.v[r].gr[h], gi = S.v[r].gi[h], a3 = S.v[r].a3[h];
            w1r[r][h] = gr * Pm + a3 * Px;
            w1i[r][h] = gi * Pm - a3 * Py;
            w2r[r][h] = -(gr * Px - gi * Py) - a3 * Pp;
            w2i[r][h] = -(gr * Py + gi * Px);
        }
    }
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int b = a + 1; b < NS; ++b)
#pragma unroll
            for (int h = 0; h < H; ++h) {
                // u_ab = w_b V_a and u_ba = w_a V_b; V = [[a3, beta], [gamma, -a3]]
                const Vert<R, H> &va = S.v[a], &vb = S.v[b];
                const R x1r = w1r[b][h] * va.a3[h] + w2r[b][h] * va.gr[h] - w2i[b][h] * va.gi[h];
                const R x1i = w1i[b][h] * va.a3[h] + w2r[b][h] * va.gi[h] + w2i[b][h] * va.gr[h];
                const R x2r = w1r[b][h] * va.br[h] - w1i[b][h] * va.bi[h] - w2r[b][h] * va.a3[h];
                const R x2i = w1r[b][h] * va.bi[h] + w1i[b][h] * va.br[h] - w2i[b][h] * va.a3[h];
                // + u_ba, continued as fused multiply-adds on u_ab
                T.u1r[a][b][h] = fma(w1r[a][h], vb.a3[h], fma(w2r[a][h], vb.gr[h], fma(-w2i[a][h], vb.gi[h], x1r)));
                T.u1i[a][b][h] = fma(w1i[a][h], vb.a3[h], fma(w2r[a][h], vb.gi[h], fma(w2i[a][h], vb.gr[h], x1i)));
                T.u2r[a][b][h] = fma(w1r[a][h], vb.br[h], fma(-w1i[a][h], vb.bi[h], fma(-w2r[a][h], vb.a3[h], x2r)));
                T.u2i[a][b][h] = fma(w1r[a][h], vb.bi[h], fma(w1i[a][h], vb.br[h], fma(-w2i[a][h], vb.a3[h], x2i)));
            }
}

// Close a node with slots a < b left: amp = U_ab . g, summed in FP64.
template <typename R, int H, int NS>
__device__ __forceinline__ void close_pair(const PairTab<R, H, NS> &T, int a, int b,
                                           const Chain<R, H> &c, Acc<H> &acc)
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const R ar = T.u1r[a][b][h] * c.g2r[h] - T.u1i[a][b][h] * c.g2i[h] +
                     T.u2r[a][b][h] * c.g3r[h] - T.u2i[a][b][h] * c.g3i[h];
        const R ai = T.u1r[a][b][h] * c.g2i[h] + T.u1i[a][b][h] * c.g2r[h] +
                     T.u2r[a][b][h] * c.g3i[h] + T.u2i[a][b][h] * c.g3r[h];
        acc.re[h] += static_cast<double>(ar);
        acc.im[h] += static_cast<double>(ai);
    }
}

template <typename R, int H, int NS>
__device__ __forceinline__ void close_pair_wide(const PairTab<R, H, NS> &T, int a, int b,
                                                const Chain<R, H> &c, Acc<H> &acc);

// The last four photons of every ordering below a node (slots in MASK,
// four of them) with pair sums at both ends (CL = 3).  The 24 orderings
// (x, y, a, b) group by the split {x, y} | {a, b}: the u end contributes the
// pair vector U_ab (both orders of a, b), the ubar end the sum of the
// currents after x then y and after y then x.  Those two currents carry the
// same momentum q + k_x + k_y, so they share their propagator:
//     G_xy = d P(q + k_x + k_y) [V_y g_x + V_x g_y],  g_x = current after x,
// and the node closes with six products U_ab . G_xy instead of twelve.
template <typename R, int H, int NS, unsigned MASK, typename PT>
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
    // (x, y) index pairs into sl and the closing pair (a, b) of the other two
    constexpr int X[6] = {0, 0, 0, 1, 1, 2}, Y[6] = {1, 2, 3, 2, 3, 3};
    constexpr int A[6] = {2, 1, 1, 0, 0, 0}, B[6] = {3, 3, 2, 3, 2, 1};
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        LMom<R> q2;
        const Prop<R> P = propagate<R>(q1[X[t]], S.k[sl[Y[t]]], q2);
        Half<R, H> s = vertex_half<R, H>(S.v[sl[Y[t]]], g1[X[t]]);
        vertex_half_add<R, H>(S.v[sl[X[t]]], g1[Y[t]], s);
        Chain<R, H> g2;
        propagator_half<R, H>(P, s, g2);
        // FP64 products pay off where a split's conversions are shared by
        // many configurations (and always in FP64, where there are none)
        if constexpr (std::is_same<R, double>::value || H >= 8)
            close_pair_wide<R, H, NS>(T, sl[A[t]], sl[B[t]], g2, acc);
        else
            close_pair<R, H, NS>(T, sl[A[t]], sl[B[t]], g2, acc);
    }
}

// Close a node with slots a < b left as close_pair does, with the product
// taken in FP64: the FP32 factors convert exactly and every product of two
// is exact in FP64, so each split enters the FP64 ordering sum through fused
// multiply-adds, with no FP32 rounding of its own.  In quad_close the
// conversions of the four pair vectors and four currents of a split are
// shared by up to sixteen helicity configurations, which makes this cheaper
// than an FP32 product followed by a conversion and an FP64 add.
template <typename R, int H, int NS>
__device__ __forceinline__ void close_pair_wide(const PairTab<R, H, NS> &T, int a, int b,
                                                const Chain<R, H> &c, Acc<H> &acc)
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const double u1r = T.u1r[a][b][h], u1i = T.u1i[a][b][h];
        const double u2r = T.u2r[a][b][h], u2i = T.u2i[a][b][h];
        const double g2r = c.g2r[h], g2i = c.g2i[h], g3r = c.g3r[h], g3i = c.g3i[h];
        acc.re[h] = fma(u1r, g2r, fma(-u1i, g2i, fma(u2r, g3r, fma(-u2i, g3i, acc.re[h]))));
        acc.im[h] = fma(u1r, g2i, fma(u1i, g2r, fma(u2r, g3i, fma(u2i, g3r, acc.im[h]))));
    }
}

// Unrolled subtree over the slot photons in MASK, entered with current c at
// momentum q.  CL = 1 closes photon by photon; CL = 2 closes the last pair;
// CL = 3 closes the last four photons with pair sums at both ends.
template <typename R, int H, int NS, int CL, unsigned MASK, typename PT>
__device__ __forceinline__ void subtree(const Slots<R, H, NS> &S, const PT &T, const Chain<R, H> &c,
                                        const LMom<R> &q, Acc<H> &acc)
{
    if constexpr (CL == 1 && __builtin_popcount(MASK) == 1) {
        close_chain<R, H>(S.v[__builtin_ctz(MASK)], c, acc);
    } else if constexpr (CL == 3 && __builtin_popcount(MASK) == 4) {
        quad_close<R, H, NS, MASK>(S, T, c, q, acc);
    } else if constexpr (CL >= 2 && __builtin_popcount(MASK) == 2) {
        constexpr int a = __builtin_ctz(MASK);
        constexpr int b = __builtin_ctz(MASK & (MASK - 1u));
        close_pair<R, H, NS>(T, a, b, c, acc);
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

// Enter a subtree over all NS slots (builds the pair vectors first for CL >= 2).
template <typename R, int H, int NS, int CL>
__device__ __forceinline__ void run_subtree(const Slots<R, H, NS> &S, const LMom<R> &p1,
                                            const Chain<R, H> &c, const LMom<R> &q, Acc<H> &acc)
{
    if constexpr (CL >= 2) {
        PairTab<R, H, NS> T;
        make_pairs<R, H, NS>(S, p1, T);
        subtree<R, H, NS, CL, (1u << NS) - 1u>(S, T, c, q, acc);
    } else {
        subtree<R, H, NS, CL, (1u << NS) - 1u>(S, NoPairs{}, c, q, acc);
    }
}

// LDS photon table of one wave: [field 0..4][photon][lane] = (k+, k-, kx, ky, t).
constexpr int kPhotonFields = 5;

template <typename R, int N>
__device__ __forceinline__ LMom<R> lds_photon(const R *tab, int j, int lane)
{
    const R *b = tab + j * 64 + lane;
    return {b[0], b[N * 64], b[2 * N * 64], b[3 * N * 64], b[4 * N * 64]};
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

// Per-point inputs after the FP64 set-up.
template <typename R, int N>
struct PointIn {
    LMom<R> k[N];   // scaled photon momenta
    LMom<R> q0;     // -p2, scaled
    LMom<R> p1;     // p1, scaled (pair closing)
};

// Sum over helicity passes [pass0, pass1) of |ordering sum|^2 (scaled units,
// without the external normalisations).  Each pass covers H configurations.
template <typename R, int N, int MB, int H, int CL>
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
        if constexpr (N <= MB) {
            Slots<R, H, N> S;
#pragma unroll
            for (int s = 0; s < N; ++s) {
                S.k[s] = in.k[s];
                S.v[s] = make_vert<R, H>(in.k[s], cfg0, s);
            }
            run_subtree<R, H, N, CL>(S, in.p1, c0, in.q0, acc);
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
template <typename R, int N, int MB, int CL>
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
    if constexpr (N <= MB) {
        Slots<R, 1, N> S;
#pragma unroll
        for (int s = 0; s < N; ++s) {
            S.k[s] = in.k[s];
            S.v[s] = make_vert<R, 1>(in.k[s], cfg, s);
        }
        run_subtree<R, 1, N, CL>(S, in.p1, c0, in.q0, acc);
    } else {
        top_levels<R, N, MB, 1, CL, 0>(tab, lane, (1u << N) - 1u, cfg, in.p1, c0, in.q0, acc);
    }
    return acc.re[0] * acc.re[0] + acc.im[0] * acc.im[0];
}

}  // namespace heget
