/*
 * FP64 CPU oracle for u ubar -> n gamma (arXiv:0908.4403).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, the smoke check and the
 * cpu_baseline leg of the benchmark; never by the product library.
 *
 * Written from the definitions, not from the printed CUDA listings: the
 * vertex functions are products of explicit 4x4 Dirac matrices in the chiral
 * representation that the HELAS conventions of Appendix B use, the amplitude
 * is the plain sum over all n! orderings of eq. (6)-(8), and the cross
 * section is eq. (1)-(2) summed point by point.  Slow on purpose.
 */
#define _GNU_SOURCE
#include "heget_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of the 4x32 Philox S-box with         */
/* multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments 0x9E3779B9      */
/* (golden ratio) and 0xBB67AE85 (sqrt(3)-1).                                 */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
    memcpy(out, c, sizeof c);
}

static double u53(uint32_t lo, uint32_t hi)
{
    uint64_t w = ((uint64_t)hi << 32) | lo;
    return ((double)(w >> 11) + 0.5) * 0x1.0p-53;
}

void orc_uniform_pair(uint64_t seed, uint64_t point, uint32_t block, uint32_t stream,
                      double u[2])
{
    uint32_t ctr[4] = {(uint32_t)point, (uint32_t)(point >> 32), block, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    u[0] = u53(r[0], r[1]);
    u[1] = u53(r[2], r[3]);
}

/* Four uniforms in (0,1) from one call, one per 32-bit word: (w + 1/2) 2^-32
 * (the photons' draws, one call per photon). */
void orc_uniform_quad(uint64_t seed, uint64_t point, uint32_t block, uint32_t stream,
                      double u[4])
{
    uint32_t ctr[4] = {(uint32_t)point, (uint32_t)(point >> 32), block, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    for (int j = 0; j < 4; ++j) u[j] = ((double)r[j] + 0.5) * 0x1.0p-32;
}

/* ------------------------------------------------------------------------ */
/* RAMBO for massless momenta (Kleiss, Stirling, Ellis 1986).                */
/* ------------------------------------------------------------------------ */
/* RAMBO's conformal transformation: boost the n vectors q to the rest frame
 * of their sum Q and rescale so that the sum becomes (sqrt_s, 0, 0, 0). */
static void conformal_map(int n, double sqrt_s, double q[][4], double *k)
{
    double Q[4] = {0, 0, 0, 0};
    for (int i = 0; i < n; ++i)
        for (int m = 0; m < 4; ++m) Q[m] += q[i][m];
    double M = sqrt(Q[0] * Q[0] - Q[1] * Q[1] - Q[2] * Q[2] - Q[3] * Q[3]);
    double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
    double x = sqrt_s / M;
    double gam = Q[0] / M;
    double a = 1.0 / (1.0 + gam);
    for (int i = 0; i < n; ++i) {
        double bq = b[0] * q[i][1] + b[1] * q[i][2] + b[2] * q[i][3];
        k[4 * i + 0] = x * (gam * q[i][0] + bq);
        for (int m = 1; m < 4; ++m)
            k[4 * i + m] = x * (q[i][m] + b[m - 1] * q[i][0] + a * bq * b[m - 1]);
    }
}

void orc_rambo(int n, double sqrt_s, const double *u, double *k)
{
    double q[8][4];
    for (int i = 0; i < n; ++i) {
        /* isotropic direction and energy density q0 exp(-q0) */
        double c = 2.0 * u[4 * i + 0] - 1.0;
        double s = sqrt(1.0 - c * c);
        double f = 2.0 * M_PI * u[4 * i + 1];
        double e = -log(u[4 * i + 2] * u[4 * i + 3]);
        q[i][0] = e;
        q[i][1] = e * s * cos(f);
        q[i][2] = e * s * sin(f);
        q[i][3] = e * c;
    }
    conformal_map(n, sqrt_s, q, k);
    /* The map scales the rounding-level masses of the q's by about the square
     * of its boost factor, which is large when the q's are nearly collinear.
     * Put every momentum back on shell (energy = |3-momentum|) and apply the
     * map once more: it is now a near-identity, so the result is massless and
     * conserves momentum to rounding.  Exact arithmetic gives the same points. */
    for (int i = 0; i < n; ++i) {
        q[i][1] = k[4 * i + 1];
        q[i][2] = k[4 * i + 2];
        q[i][3] = k[4 * i + 3];
        q[i][0] = sqrt(q[i][1] * q[i][1] + q[i][2] * q[i][2] + q[i][3] * q[i][3]);
    }
    conformal_map(n, sqrt_s, q, k);
}

/* Volume of the massless n-body phase space of eq. (4):
 * (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!). */
double orc_rambo_weight(int n, double s)
{
    double fact_n1 = 1.0, fact_n2 = 1.0;
    for (int i = 2; i <= n - 1; ++i) fact_n1 *= i;
    for (int i = 2; i <= n - 2; ++i) fact_n2 *= i;
    return pow(2.0 * M_PI, 4.0 - 3.0 * n) * pow(M_PI / 2.0, n - 1) * pow(s, n - 2) /
           (fact_n1 * fact_n2);
}

void orc_cm_event(int n, double sqrt_shat, uint64_t seed, uint64_t point, double *p)
{
    double u[32];
    for (int i = 0; i < n; ++i) orc_uniform_quad(seed, point, (uint32_t)i, 0, &u[4 * i]);
    double e = 0.5 * sqrt_shat;
    double p1[4] = {e, 0, 0, e}, p2[4] = {e, 0, 0, -e};
    memcpy(p, p1, sizeof p1);
    memcpy(p + 4, p2, sizeof p2);
    orc_rambo(n, sqrt_shat, u, p + 8);
}

void orc_cm_events(int n, double sqrt_shat, uint64_t seed, uint64_t first, int64_t np,
                   double *p_aos)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np; ++i)
        orc_cm_event(n, sqrt_shat, seed, first + (uint64_t)i, p_aos + i * (n + 2) * 4);
}

/* ------------------------------------------------------------------------ */
/* Cuts, eq. (9)-(10).  eta = rapidity (= pseudorapidity for photons).       */
/* ------------------------------------------------------------------------ */
int orc_pass_cuts(int n, const double *k, double y, double pt_min, double eta_max,
                  double dr_min)
{
    double eta[8], phi[8];
    for (int i = 0; i < n; ++i) {
        const double *ki = k + 4 * i;
        double pt = sqrt(ki[1] * ki[1] + ki[2] * ki[2]);
        double pabs = sqrt(ki[1] * ki[1] + ki[2] * ki[2] + ki[3] * ki[3]);
        eta[i] = atanh(ki[3] / pabs) + y;
        phi[i] = atan2(ki[2], ki[1]);
        if (pt_min > 0 && !(pt > pt_min)) return 0;
        if (eta_max > 0 && !(fabs(eta[i]) < eta_max)) return 0;
    }
    if (dr_min > 0) {
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                double deta = eta[i] - eta[j];
                double dphi = fabs(phi[i] - phi[j]);
                if (dphi > M_PI) dphi = 2.0 * M_PI - dphi;
                if (!(sqrt(deta * deta + dphi * dphi) > dr_min)) return 0;
            }
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Dirac algebra, chiral representation (the one HELAS uses):                */
/*   gamma^0 = [[0,1],[1,0]], gamma^k = [[0,sigma^k],[-sigma^k,0]],            */
/*   gamma5 = diag(-1,-1,1,1), P_L = (1-gamma5)/2 = diag(1,1,0,0).              */
/* Spinors are stored as 4 complex components; a "flowing-out" wavefunction  */
/* <fo| is a row vector (already barred).                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    cplx m[4][4];
} mat4;

static mat4 GAMMA[4];
static int gamma_ready = 0;

/* built once when the library loads, so OpenMP threads only ever read it */
__attribute__((constructor)) static void init_gamma(void)
{
    if (gamma_ready) return;
    const cplx iu = _Complex_I;
    /* Pauli matrices */
    cplx sig[4][2][2] = {
        {{1, 0}, {0, 1}},
        {{0, 1}, {1, 0}},
        {{0, -iu}, {iu, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAMMA, 0, sizeof GAMMA);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            GAMMA[0].m[a][2 + b] = sig[0][a][b];
            GAMMA[0].m[2 + a][b] = sig[0][a][b];
            for (int k = 1; k < 4; ++k) {
                GAMMA[k].m[a][2 + b] = sig[k][a][b];
                GAMMA[k].m[2 + a][b] = -sig[k][a][b];
            }
        }
    gamma_ready = 1;
}

/* slash(a) = gamma^mu a_mu = gamma^0 a^0 - gamma^k a^k, a given with upper index */
static mat4 slash_c(const cplx a[4])
{
    mat4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            r.m[i][j] = GAMMA[0].m[i][j] * a[0] - GAMMA[1].m[i][j] * a[1] -
                        GAMMA[2].m[i][j] * a[2] - GAMMA[3].m[i][j] * a[3];
    return r;
}

static mat4 slash_r(const double a[4])
{
    cplx c[4] = {a[0], a[1], a[2], a[3]};
    return slash_c(c);
}

/* chiral coupling Gamma = gal0 P_L + gal1 P_R of the FFV Lagrangian (Appendix B.3) */
static mat4 chiral_coupling(double gal0, double gal1)
{
    mat4 r;
    memset(&r, 0, sizeof r);
    r.m[0][0] = r.m[1][1] = gal0;
    r.m[2][2] = r.m[3][3] = gal1;
    return r;
}

static void row_times(const cplx v[4], const mat4 *m, cplx out[4])
{
    for (int j = 0; j < 4; ++j) {
        cplx s = 0;
        for (int i = 0; i < 4; ++i) s += v[i] * m->m[i][j];
        out[j] = s;
    }
}

static void mat_times(const mat4 *m, const cplx v[4], cplx out[4])
{
    for (int i = 0; i < 4; ++i) {
        cplx s = 0;
        for (int j = 0; j < 4; ++j) s += m->m[i][j] * v[j];
        out[i] = s;
    }
}

/* A wavefunction: 4 spinor (or polarisation) components and the momentum it
 * carries along the fermion-number (or particle) flow, as in HELAS where
 * components 4-5 hold the momentum times nSF (fermions) or nSV (vectors). */
typedef struct {
    cplx s[4];
    double p[4];
} wf;

/* ---- external wavefunctions (Appendix B.1-B.2) ---- */

/* Flowing-in massless u spinor u(p, h/2) (nSF = +1) for p on the z axis, in the
 * HELAS phase convention.  Chirality: h = +1 lives in the lower (right-handed)
 * pair, h = -1 in the upper (left-handed) pair, each of size sqrt(2E). */
static wf u_spinor_z(const double p[4], int h, int along_minus_z)
{
    wf w;
    memset(&w, 0, sizeof w);
    double r = sqrt(2.0 * p[0]);
    if (!along_minus_z) { /* ixxxx1 */
        if (h == 1) w.s[2] = r;
        else w.s[1] = r;
    } else { /* ixxxx2 */
        if (h == 1) w.s[3] = r;
        else w.s[0] = -r;
    }
    for (int m = 0; m < 4; ++m) w.p[m] = p[m];
    return w;
}

/* Flowing-out massless vbar spinor vbar(p, h/2) (nSF = -1) for p on the z axis,
 * HELAS phase convention; the stored momentum is -p (fermion-number flow). */
static wf vbar_spinor_z(const double p[4], int h, int along_plus_z)
{
    wf w;
    memset(&w, 0, sizeof w);
    double r = sqrt(2.0 * p[0]);
    if (!along_plus_z) { /* oxxxx2 */
        if (h == 1) w.s[2] = -r;
        else w.s[1] = r;
    } else { /* oxxxx1 */
        if (h == 1) w.s[3] = -r;
        else w.s[0] = -r;
    }
    for (int m = 0; m < 4; ++m) w.p[m] = -p[m];
    return w;
}

/* Outgoing photon (nSV = +1): eps*(k, lam) = (-lam e_theta + i e_phi)/sqrt(2)
 * with e_theta, e_phi the polar unit vectors of k; eps^0 = 0, so eps.k = 0
 * and eps.n = 0 for n = (k^0, -k).  Singular for pT = 0. */
static wf photon_eps(const double k[4], int lam)
{
    wf w;
    double pt = sqrt(k[1] * k[1] + k[2] * k[2]);
    double pabs = sqrt(pt * pt + k[3] * k[3]);
    double ct = k[3] / pabs, st = pt / pabs;
    double cf = k[1] / pt, sf = k[2] / pt;
    double eth[3] = {ct * cf, ct * sf, -st};
    double eph[3] = {-sf, cf, 0.0};
    w.s[0] = 0;
    for (int m = 0; m < 3; ++m)
        w.s[m + 1] = (-lam * eth[m] + _Complex_I * eph[m]) / sqrt(2.0);
    for (int m = 0; m < 4; ++m) w.p[m] = k[m];
    return w;
}

/* ---- FFV vertex functions (Appendix B.3), from the Lagrangian ----
 *   L = psibar_F1 gamma^mu (gal0 P_L + gal1 P_R) psi_F2 V*_mu,
 * fermion propagator numerator slash(q) with factor d = -1/q^2 (massless). */

static double mdot(const double a[4], const double b[4])
{
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* amplitude <fo| eps-slash Gamma |fi> (iovxx0) */
static cplx iov(const wf *fi, const wf *fo, const wf *vc, double gal0, double gal1)
{
    mat4 e = slash_c(vc->s), G = chiral_coupling(gal0, gal1);
    cplx t1[4], t2[4];
    row_times(fo->s, &e, t1);
    row_times(t1, &G, t2);
    cplx r = 0;
    for (int i = 0; i < 4; ++i) r += t2[i] * fi->s[i];
    return r;
}

/* off-shell outgoing fermion <fo| eps-slash Gamma slash(q) (-1/q^2), q = p_fo + k (fvoxx0) */
static wf fvo(const wf *fo, const wf *vc, double gal0, double gal1)
{
    wf r;
    for (int m = 0; m < 4; ++m) r.p[m] = fo->p[m] + vc->p[m];
    double d = -1.0 / mdot(r.p, r.p);
    mat4 e = slash_c(vc->s), G = chiral_coupling(gal0, gal1), q = slash_r(r.p);
    cplx t1[4], t2[4];
    row_times(fo->s, &e, t1);
    row_times(t1, &G, t2);
    row_times(t2, &q, r.s);
    for (int i = 0; i < 4; ++i) r.s[i] *= d;
    return r;
}

/* off-shell incoming fermion (-1/q^2) slash(q) eps-slash Gamma |fi>, q = p_fi - k (fvixx0) */
static wf fvi(const wf *fi, const wf *vc, double gal0, double gal1)
{
    wf r;
    for (int m = 0; m < 4; ++m) r.p[m] = fi->p[m] - vc->p[m];
    double d = -1.0 / mdot(r.p, r.p);
    mat4 e = slash_c(vc->s), G = chiral_coupling(gal0, gal1), q = slash_r(r.p);
    cplx t1[4], t2[4];
    mat_times(&G, fi->s, t1);
    mat_times(&e, t1, t2);
    mat_times(&q, t2, r.s);
    for (int i = 0; i < 4; ++i) r.s[i] *= d;
    return r;
}

/* ---- the massless HELAS set in any direction (Appendix B.1-B.3) ----
 * Written from the definitions: helicity eigenspinors of p with polar angles
 * (theta, phi),
 *   xi_+ = (cos(theta/2), e^{i phi} sin(theta/2)),
 *   xi_- = (-e^{-i phi} sin(theta/2), cos(theta/2)),
 * u(p, +1/2) = sqrt(2E) (0, 0, xi_+) and u(p, -1/2) = sqrt(2E) (xi_-, 0, 0) in
 * the chiral representation (left-handed pair on top), v(p, h) = -u(p, -h),
 * ubar = u^dagger gamma^0.  Polarisations eps(p, lam) = (-lam e_theta -
 * i e_phi)/sqrt(2) and their conjugates (nsv = +1 for final-state vectors).
 * Phase conventions on the z axis, where phi is undefined, are those of the
 * HELAS functions: phi = 0 along +z; along -z phi = 0 for flowing-in spinors
 * and phi = pi for flowing-out spinors and for vectors. */
static void polar_angles(const double p[4], double *theta, double *phi, int minus_z_phi_pi)
{
    double pt = hypot(p[1], p[2]);
    *theta = atan2(pt, p[3]);
    if (pt > 0) *phi = atan2(p[2], p[1]);
    else *phi = (p[3] < 0 && minus_z_phi_pi) ? M_PI : 0.0;
}

static wf spinor_in_any(const double p[4], int nhel, int nsf)
{
    wf w;
    memset(&w, 0, sizeof w);
    int h = nsf == 1 ? nhel : -nhel; /* v(p, h) = -u(p, -h) */
    double th, ph;
    polar_angles(p, &th, &ph, 0);
    double r = sqrt(2.0 * p[0]) * (nsf == 1 ? 1.0 : -1.0);
    if (h == 1) {
        w.s[2] = r * cos(th / 2);
        w.s[3] = r * cexp(_Complex_I * ph) * sin(th / 2);
    } else {
        w.s[0] = -r * cexp(-_Complex_I * ph) * sin(th / 2);
        w.s[1] = r * cos(th / 2);
    }
    for (int m = 0; m < 4; ++m) w.p[m] = nsf * p[m];
    return w;
}

static wf spinor_out_any(const double p[4], int nhel, int nsf)
{
    wf w;
    memset(&w, 0, sizeof w);
    int h = nsf == 1 ? nhel : -nhel;
    double th, ph;
    polar_angles(p, &th, &ph, 1);
    double r = sqrt(2.0 * p[0]) * (nsf == 1 ? 1.0 : -1.0);
    cplx c[4] = {0, 0, 0, 0};
    if (h == 1) {
        c[2] = r * cos(th / 2);
        c[3] = r * cexp(_Complex_I * ph) * sin(th / 2);
    } else {
        c[0] = -r * cexp(-_Complex_I * ph) * sin(th / 2);
        c[1] = r * cos(th / 2);
    }
    /* row u^dagger gamma^0: gamma^0 swaps the two pairs */
    w.s[0] = conj(c[2]);
    w.s[1] = conj(c[3]);
    w.s[2] = conj(c[0]);
    w.s[3] = conj(c[1]);
    for (int m = 0; m < 4; ++m) w.p[m] = nsf * p[m];
    return w;
}

static wf vector_any(const double k[4], int nhel, int nsv)
{
    wf w;
    double th, ph;
    polar_angles(k, &th, &ph, 1);
    double eth[3] = {cos(th) * cos(ph), cos(th) * sin(ph), -sin(th)};
    double eph[3] = {-sin(ph), cos(ph), 0.0};
    w.s[0] = 0;
    for (int m = 0; m < 3; ++m)
        w.s[m + 1] = (-nhel * eth[m] + nsv * _Complex_I * eph[m]) / sqrt(2.0);
    for (int m = 0; m < 4; ++m) w.p[m] = nsv * k[m];
    return w;
}

/* off-shell vector current J^mu = d <fo| gamma^mu Gamma |fi>, q = p_fo - p_fi
 * (jioxx0), Feynman gauge.  d = +1/q^2: with vertex factors i Gamma, fermion
 * propagators i slash(q)/q^2 and photon propagators -i g/q^2, a tree amplitude
 * is i M with M the product of Gamma's, -slash(q)/q^2 per fermion line and
 * +g/q^2 per photon line, which fixes the signs of both d's. */
static wf jio(const wf *fi, const wf *fo, double gal0, double gal1)
{
    wf r;
    for (int m = 0; m < 4; ++m) r.p[m] = fo->p[m] - fi->p[m];
    double d = 1.0 / mdot(r.p, r.p);
    mat4 G = chiral_coupling(gal0, gal1);
    cplx t[4];
    mat_times(&G, fi->s, t);
    for (int mu = 0; mu < 4; ++mu) {
        cplx u[4];
        row_times(fo->s, &GAMMA[mu], u);
        cplx s = 0;
        for (int i = 0; i < 4; ++i) s += u[i] * t[i];
        r.s[mu] = d * s;
    }
    return r;
}

static void wf_unpack(const double *x, wf *w)
{
    for (int i = 0; i < 4; ++i) w->s[i] = x[2 * i] + _Complex_I * x[2 * i + 1];
    for (int m = 0; m < 4; ++m) w->p[m] = x[8 + m];
}

static void wf_pack(const wf *w, double *x)
{
    for (int i = 0; i < 4; ++i) {
        x[2 * i] = creal(w->s[i]);
        x[2 * i + 1] = cimag(w->s[i]);
    }
    for (int m = 0; m < 4; ++m) x[8 + m] = w->p[m];
}

int orc_helas(int func, const double *in, double *out)
{
    init_gamma();
    wf a, b, c, r;
    switch (func) {
    case 0: case 1: case 2: /* ixxxx0/1/2 */
        r = spinor_in_any(in, (int)in[4], (int)in[5]);
        wf_pack(&r, out);
        return 12;
    case 3: case 4: case 5: /* oxxxx0/1/2 */
        r = spinor_out_any(in, (int)in[4], (int)in[5]);
        wf_pack(&r, out);
        return 12;
    case 6: /* vxxxx0 */
        r = vector_any(in, (int)in[4], (int)in[5]);
        wf_pack(&r, out);
        return 12;
    case 7: case 8: /* vxxxx1/2: incoming vectors only, nsv is not read */
        r = vector_any(in, (int)in[4], -1);
        wf_pack(&r, out);
        return 12;
    case 9: { /* iovxxx(fi, fo, vc, gal) */
        wf_unpack(in, &a);
        wf_unpack(in + 12, &b);
        wf_unpack(in + 24, &c);
        cplx v = iov(&a, &b, &c, in[36], in[37]);
        out[0] = creal(v);
        out[1] = cimag(v);
        return 2;
    }
    case 10: /* fvixx0(fi, vc, gal) */
        wf_unpack(in, &a);
        wf_unpack(in + 12, &c);
        r = fvi(&a, &c, in[24], in[25]);
        wf_pack(&r, out);
        return 12;
    case 11: /* fvoxx0(fo, vc, gal) */
        wf_unpack(in, &b);
        wf_unpack(in + 12, &c);
        r = fvo(&b, &c, in[24], in[25]);
        wf_pack(&r, out);
        return 12;
    case 12: /* jioxx0(fi, fo, gal) */
        wf_unpack(in, &a);
        wf_unpack(in + 12, &b);
        r = jio(&a, &b, in[24], in[25]);
        wf_pack(&r, out);
        return 12;
    default:
        return -1;
    }
}

/* forward declarations for the frame-independent evaluators below */
static int next_perm(int *a, int n);

/* Helicity-summed |M|^2 of u(p1) ubar(p2) -> n photons for momenta in any
 * frame (eq. (6)-(8)), from the direction-general wavefunctions: u from
 * ixxxx0, vbar from oxxxx0 (nSF = -1), eps* from vxxxx0 (nSV = +1), every
 * ordering a chain of fvoxx0 closed with iovxxx.  All 2^(n+2) helicities. */
double orc_me2_frame(int n, const double *p, double alpha, double charge)
{
    init_gamma();
    double g = -sqrt(4.0 * M_PI * alpha) * charge;
    double sum = 0.0;
    for (int h1 = -1; h1 <= 1; h1 += 2)
        for (int h2 = -1; h2 <= 1; h2 += 2)
            for (int bits = 0; bits < (1 << n); ++bits) {
                wf u = spinor_in_any(p, h1, 1), vb = spinor_out_any(p + 4, h2, -1), eps[8];
                for (int i = 0; i < n; ++i)
                    eps[i] = vector_any(p + 8 + 4 * i, ((bits >> i) & 1) ? 1 : -1, 1);
                int a[8];
                for (int i = 0; i < n; ++i) a[i] = i;
                cplx total = 0;
                do {
                    wf w = vb;
                    for (int j = 0; j < n - 1; ++j) w = fvo(&w, &eps[a[j]], g, g);
                    total += iov(&u, &w, &eps[a[n - 1]], g, g);
                } while (next_perm(a, n));
                sum += creal(total) * creal(total) + cimag(total) * cimag(total);
            }
    return sum;
}

/* Helicity-summed |M|^2 of f(p1) fbar(p2) -> f'(p3) fbar'(p4) through one
 * photon: the current jioxx0 of the incoming pair closed with iovxxx on the
 * outgoing pair; couplings -e q1 and -e q2. */
double orc_me2_ffff(const double *p, double alpha, double q1, double q2)
{
    init_gamma();
    double e = sqrt(4.0 * M_PI * alpha);
    double sum = 0.0;
    for (int h = 0; h < 16; ++h) {
        wf fi1 = spinor_in_any(p, (h & 1) ? 1 : -1, 1);
        wf fo1 = spinor_out_any(p + 4, (h & 2) ? 1 : -1, -1);
        wf fo2 = spinor_out_any(p + 8, (h & 4) ? 1 : -1, 1);
        wf fi2 = spinor_in_any(p + 12, (h & 8) ? 1 : -1, -1);
        wf j = jio(&fi1, &fo1, -e * q1, -e * q1);
        cplx a = iov(&fi2, &fo2, &j, -e * q2, -e * q2);
        sum += creal(a) * creal(a) + cimag(a) * cimag(a);
    }
    return sum;
}

/* next permutation in lexicographic order; returns 0 after the last one */
static int next_perm(int *a, int n)
{
    int i = n - 2;
    while (i >= 0 && a[i] >= a[i + 1]) --i;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] <= a[i]) --j;
    int t = a[i];
    a[i] = a[j];
    a[j] = t;
    for (int l = i + 1, r = n - 1; l < r; ++l, --r) {
        t = a[l];
        a[l] = a[r];
        a[r] = t;
    }
    return 1;
}

static void external_wfs(int n, const double *p, int h1, int h2, const int *lam,
                         int u_minus_z, wf *u, wf *vb, wf *eps)
{
    *u = u_spinor_z(p, h1, u_minus_z);
    *vb = vbar_spinor_z(p + 4, h2, u_minus_z);
    for (int i = 0; i < n; ++i) eps[i] = photon_eps(p + 8 + 4 * i, lam[i]);
}

/* sum over all orderings of: ubar end -> fvo ... fvo -> iov with u (Appendix A.2) */
static cplx ordering_sum(int n, const wf *u, const wf *vb, const wf *eps, double g,
                         double *sum_abs)
{
    int a[8];
    for (int i = 0; i < n; ++i) a[i] = i;
    cplx total = 0;
    double sabs = 0;
    do {
        wf w = *vb;
        for (int j = 0; j < n - 1; ++j) w = fvo(&w, &eps[a[j]], g, g);
        cplx amp = iov(u, &w, &eps[a[n - 1]], g, g);
        total += amp;
        sabs += cabs(amp);
    } while (next_perm(a, n));
    if (sum_abs) *sum_abs = sabs;
    return total;
}

void orc_amp(int n, const double *p, int h1, int h2, const int *lam, double g,
             int u_along_minus_z, double *re, double *im)
{
    init_gamma();
    wf u, vb, eps[8];
    external_wfs(n, p, h1, h2, lam, u_along_minus_z, &u, &vb, eps);
    cplx r = ordering_sum(n, &u, &vb, eps, g, NULL);
    *re = creal(r);
    *im = cimag(r);
}

void orc_amp_from_u(int n, const double *p, int h1, int h2, const int *lam, double g,
                    double *re, double *im)
{
    init_gamma();
    wf u, vb, eps[8];
    external_wfs(n, p, h1, h2, lam, 0, &u, &vb, eps);
    int a[8];
    for (int i = 0; i < n; ++i) a[i] = i;
    cplx total = 0;
    do {
        wf w = u;
        for (int j = 0; j < n - 1; ++j) w = fvi(&w, &eps[a[j]], g, g);
        total += iov(&w, &vb, &eps[a[n - 1]], g, g);
    } while (next_perm(a, n));
    *re = creal(total);
    *im = cimag(total);
}

void orc_amp_custom_eps(int n, const double *p, int h1, int h2, const double *epsv,
                        double g, double *re, double *im, double *sum_abs)
{
    init_gamma();
    wf u, vb, eps[8];
    int lam[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    external_wfs(n, p, h1, h2, lam, 0, &u, &vb, eps);
    for (int i = 0; i < n; ++i)
        for (int m = 0; m < 4; ++m)
            eps[i].s[m] = epsv[(i * 4 + m) * 2] + _Complex_I * epsv[(i * 4 + m) * 2 + 1];
    cplx r = ordering_sum(n, &u, &vb, eps, g, sum_abs);
    *re = creal(r);
    *im = cimag(r);
}

/* Two-sided schedule (the current reuse of the MadGraph-generated program of
 * Appendix A.1): every ordering a[0..n-1] (listed from the ubar end) is
 * evaluated by meeting an outgoing current built from the ubar end over
 * a[0..s-1] with an incoming current built from the u end over
 * a[n-1], ..., a[s+1] at the vertex of photon a[s].  split >= 0 fixes s;
 * split < 0 takes s = (ordering index) mod n, so every split is exercised. */
void orc_amp_meet(int n, const double *p, int h1, int h2, const int *lam, double g,
                  int split, double *re, double *im)
{
    init_gamma();
    wf u, vb, eps[8];
    external_wfs(n, p, h1, h2, lam, 0, &u, &vb, eps);
    int a[8];
    for (int i = 0; i < n; ++i) a[i] = i;
    cplx total = 0;
    int idx = 0;
    do {
        int s = split >= 0 ? split % n : idx % n;
        wf wo = vb, wi = u;
        for (int j = 0; j < s; ++j) wo = fvo(&wo, &eps[a[j]], g, g);
        for (int j = n - 1; j > s; --j) wi = fvi(&wi, &eps[a[j]], g, g);
        total += iov(&wi, &wo, &eps[a[s]], g, g);
        ++idx;
    } while (next_perm(a, n));
    *re = creal(total);
    *im = cimag(total);
}

double orc_me2(int n, const double *p, double alpha, double charge, int skip_zero,
               int u_along_minus_z)
{
    init_gamma();
    double g = -sqrt(4.0 * M_PI * alpha) * charge;
    double sum = 0.0;
    int lam[8];
    for (int h1 = -1; h1 <= 1; h1 += 2)
        for (int h2 = -1; h2 <= 1; h2 += 2) {
            if (skip_zero && h1 == h2) continue;
            for (int bits = 0; bits < (1 << n); ++bits) {
                for (int i = 0; i < n; ++i) lam[i] = ((bits >> i) & 1) ? 1 : -1;
                double re, im;
                orc_amp(n, p, h1, h2, lam, g, u_along_minus_z, &re, &im);
                sum += re * re + im * im;
            }
        }
    return sum;
}

/* Number of OpenMP threads the batch functions use from now on (k >= 1);
 * k <= 0 restores the runtime default.  Returns the count in effect. */
int orc_set_threads(int k)
{
#ifdef _OPENMP
    static int deflt = 0;
    if (deflt == 0) deflt = omp_get_max_threads();
    omp_set_num_threads(k >= 1 ? k : deflt);
    return omp_get_max_threads();
#else
    (void)k;
    return 1;
#endif
}

int orc_me2_batch(int n, int64_t np, const double *p_aos, double alpha, double charge,
                  double *out)
{
    init_gamma();
    int threads = 1;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        threads = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < np; ++i)
            out[i] = orc_me2(n, p_aos + i * (n + 2) * 4, alpha, charge, 1, 0);
    }
    return threads;
}

/* Subset recursion: J(S) = sum_{j in S} fvo(J(S \ j), eps_j); every J(S) carries
 * the momentum -p2 + sum_{i in S} k_i, so the sum of currents is well defined. */
double orc_me2_subsets(int n, const double *p, double alpha, double charge)
{
    init_gamma();
    double g = -sqrt(4.0 * M_PI * alpha) * charge;
    int full = (1 << n) - 1;
    wf *J = (wf *)malloc(sizeof(wf) * (size_t)(1 << n));
    double sum = 0.0;
    int lam[8];
    for (int h1 = -1; h1 <= 1; h1 += 2)
        for (int h2 = -1; h2 <= 1; h2 += 2) {
            if (h1 == h2) continue;
            for (int bits = 0; bits < (1 << n); ++bits) {
                for (int i = 0; i < n; ++i) lam[i] = ((bits >> i) & 1) ? 1 : -1;
                wf u, vb, eps[8];
                external_wfs(n, p, h1, h2, lam, 0, &u, &vb, eps);
                J[0] = vb;
                for (int S = 1; S < full; ++S) {
                    wf acc;
                    memset(&acc, 0, sizeof acc);
                    for (int j = 0; j < n; ++j) {
                        if (!((S >> j) & 1)) continue;
                        wf t = fvo(&J[S & ~(1 << j)], &eps[j], g, g);
                        for (int c = 0; c < 4; ++c) acc.s[c] += t.s[c];
                        memcpy(acc.p, t.p, sizeof acc.p);
                    }
                    J[S] = acc;
                }
                cplx amp = 0;
                for (int j = 0; j < n; ++j) amp += iov(&u, &J[full & ~(1 << j)], &eps[j], g, g);
                sum += creal(amp) * creal(amp) + cimag(amp) * cimag(amp);
            }
        }
    free(J);
    return sum;
}

int orc_me2_subsets_batch(int n, int64_t np, const double *p_aos, double alpha,
                          double charge, double *out)
{
    init_gamma();
    int threads = 1;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        threads = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < np; ++i)
            out[i] = orc_me2_subsets(n, p_aos + i * (n + 2) * 4, alpha, charge);
    }
    return threads;
}

/* ------------------------------------------------------------------------ */
/* Cross section, eq. (1)-(2).                                               */
/* ------------------------------------------------------------------------ */
double orc_gev2_fb(void) { return 0.3893793721e12; }

/* eq. (2) without |M|^2: 1/(2 shat) * 1/2^2 * 1/3^2 * 3 * 1/n! * Phi_n volume * (hbar c)^2 */
static double partonic_factor(int n, double shat)
{
    double nfact = 1.0;
    for (int i = 2; i <= n; ++i) nfact *= i;
    return 1.0 / (2.0 * shat) * 0.25 * (1.0 / 9.0) * 3.0 / nfact *
           orc_rambo_weight(n, shat) * orc_gev2_fb();
}

void orc_draw_helicity(int n, uint64_t seed, uint64_t point, int *h1, int *h2, int *lam)
{
    const uint32_t ctr[4] = {(uint32_t)point, (uint32_t)(point >> 32), 0u, 2u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    const uint32_t w = out[0];
    *h1 = (w & 1u) ? 1 : -1;
    *h2 = -*h1;
    for (int i = 0; i < n; ++i) lam[i] = ((w >> (1 + i)) & 1u) ? 1 : -1;
}

/* |M|^2 of the point: the helicity sum, or in sampling mode the estimator
 * 2^(n+1) |M_h|^2 of the drawn configuration (its mean over the uniform draw
 * is the sum over the 2^(n+1) non-vanishing configurations). */
static double point_me2(int n, const orc_config *cfg, const double *p, int u_minus_z,
                        uint64_t point)
{
    if (cfg->helicity_sampling) {
        int h1, h2, lam[8];
        orc_draw_helicity(n, cfg->seed, point, &h1, &h2, lam);
        const double g = -sqrt(4.0 * M_PI * cfg->alpha) * cfg->charge;
        double re, im;
        orc_amp(n, p, h1, h2, lam, g, u_minus_z, &re, &im);
        return ldexp(re * re + im * im, n + 1);
    }
    if (cfg->me2_method == 1 && !u_minus_z) return orc_me2_subsets(n, p, cfg->alpha, cfg->charge);
    return orc_me2(n, p, cfg->alpha, cfg->charge, 1, u_minus_z);
}

int orc_point(int n, const orc_config *cfg, uint64_t point, double *p, double *y,
              double *me2, double *w)
{
    double sqrt_shat = cfg->sqrt_s;
    double fpdf = 1.0, xu = 0, xub = 0;
    *y = 0.0;
    *me2 = 0.0;
    *w = 0.0;
    if (cfg->mode == ORC_UNIFORM_SQRTSHAT) {
        double r[2];
        orc_uniform_pair(cfg->seed, point, 1, 1, r);
        sqrt_shat = cfg->sqrt_shat_lo + (cfg->sqrt_shat_hi - cfg->sqrt_shat_lo) * r[0];
    } else if (cfg->mode == ORC_PP_TOY) {
        /* toy densities D_u = x^-0.5 (1-x)^3, D_ubar = x^-0.3 (1-x)^6, sampled
         * as x = r^(1/a) (density a x^(a-1)) with weight D/density */
        double r[2];
        orc_uniform_pair(cfg->seed, point, 0, 1, r);
        xu = pow(r[0], 1.0 / 0.5);
        xub = pow(r[1], 1.0 / 0.7);
        fpdf = pow(1.0 - xu, 3) / 0.5 * pow(1.0 - xub, 6) / 0.7;
        double shat = xu * xub * cfg->sqrt_s * cfg->sqrt_s;
        sqrt_shat = sqrt(shat);
        if (!(sqrt_shat >= cfg->sqrt_shat_lo)) {
            orc_cm_event(n, sqrt_shat > 0 ? sqrt_shat : 1.0, cfg->seed, point, p);
            return 0;
        }
    }
    orc_cm_event(n, sqrt_shat, cfg->seed, point, p);
    double shat = sqrt_shat * sqrt_shat;
    double base = partonic_factor(n, shat);
    if (cfg->mode != ORC_PP_TOY) {
        if (!orc_pass_cuts(n, p + 8, 0.0, cfg->pt_min, cfg->eta_max, cfg->dr_min)) return 0;
        *me2 = point_me2(n, cfg, p, 0, point);
        *w = base * *me2;
        return 1;
    }
    /* eq. (1): both assignments of u and ubar to the two beams.
     * A: u from beam 1 (moves along +z), x1 = xu, x2 = xub.
     * B: ubar from beam 1, u from beam 2; the CM event is the RAMBO event
     *    rotated by pi about the x axis, so u moves along -z. */
    double yA = 0.5 * log(xu / xub);
    double yB = 0.5 * log(xub / xu);
    *y = yA;
    double pB[4 * 10];
    for (int i = 0; i < n + 2; ++i) {
        pB[4 * i + 0] = p[4 * i + 0];
        pB[4 * i + 1] = p[4 * i + 1];
        pB[4 * i + 2] = -p[4 * i + 2];
        pB[4 * i + 3] = -p[4 * i + 3];
    }
    int passA = orc_pass_cuts(n, p + 8, yA, cfg->pt_min, cfg->eta_max, cfg->dr_min);
    int passB = orc_pass_cuts(n, pB + 8, yB, cfg->pt_min, cfg->eta_max, cfg->dr_min);
    double meA = passA ? point_me2(n, cfg, p, 0, point) : 0.0;
    double meB = passB ? point_me2(n, cfg, pB, 1, point) : 0.0;
    *me2 = passA ? meA : meB;
    *w = fpdf * base * (meA + meB);
    return passA || passB;
}

double orc_observable(int n, const double *k, int observable)
{
    if (observable == 0) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m = fmax(m, hypot(k[4 * i + 1], k[4 * i + 2]));
        return m;
    }
    double eta[8], phi[8], m = INFINITY;
    for (int i = 0; i < n; ++i) {
        const double *q = k + 4 * i;
        eta[i] = atanh(q[3] / sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]));
        phi[i] = atan2(q[2], q[1]);
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double dphi = fabs(phi[i] - phi[j]);
            if (dphi > M_PI) dphi = 2.0 * M_PI - dphi;
            m = fmin(m, hypot(eta[i] - eta[j], dphi));
        }
    return m;
}

int orc_hist(int n, const orc_config *cfg, int observable, int nbins, double lo, double hi,
             double *hist)
{
    init_gamma();
    const int64_t N = cfg->npoints;
    double *w = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *x = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    int threads = 1;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        threads = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < N; ++i) {
            double p[40], y, me2;
            orc_point(n, cfg, (uint64_t)(cfg->first_point + i), p, &y, &me2, &w[i]);
            x[i] = orc_observable(n, p + 8, observable);
        }
    }
    double *s = (double *)calloc((size_t)nbins + 2, sizeof(double));
    double *c = (double *)calloc((size_t)nbins + 2, sizeof(double));
    for (int64_t i = 0; i < N; ++i) {
        if (w[i] == 0.0) continue;
        int b;
        if (x[i] < lo) b = 0;
        else if (x[i] >= hi) b = nbins + 1;
        else {
            b = 1 + (int)((x[i] - lo) / (hi - lo) * nbins);
            if (b > nbins) b = nbins;
        }
        const double t = s[b] + w[i];
        if (fabs(s[b]) >= fabs(w[i])) c[b] += (s[b] - t) + w[i];
        else c[b] += (w[i] - t) + s[b];
        s[b] = t;
    }
    for (int b = 0; b < nbins + 2; ++b) hist[b] = N > 0 ? (s[b] + c[b]) / (double)N : 0.0;
    free(s);
    free(c);
    free(w);
    free(x);
    return threads;
}

int orc_xsec(int n, const orc_config *cfg, orc_result *out, double *w_out)
{
    init_gamma();
    int64_t N = cfg->npoints;
    double *w = w_out ? w_out : (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    char *acc = (char *)malloc((size_t)(N > 0 ? N : 1));
    int threads = 1;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        threads = omp_get_num_threads();
#endif
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < N; ++i) {
            double p[40], y, me2;
            acc[i] = (char)orc_point(n, cfg, (uint64_t)(cfg->first_point + i), p, &y, &me2,
                                     &w[i]);
        }
    }
    /* Neumaier summation in point order */
    double s = 0, c = 0, s2 = 0;
    int64_t nacc = 0;
    for (int64_t i = 0; i < N; ++i) {
        double t = s + w[i];
        if (fabs(s) >= fabs(w[i])) c += (s - t) + w[i];
        else c += (w[i] - t) + s;
        s = t;
        s2 += w[i] * w[i];
        nacc += acc[i];
    }
    out->sum_w = s + c;
    out->sum_w_comp = c;
    out->sum_w2 = s2;
    out->n_gen = N;
    out->n_acc = nacc;
    double sigma = N > 0 ? (s + c) / (double)N : 0.0;
    out->sigma_fb = sigma;
    out->err_fb = N > 1 ? sqrt(fmax(s2 / (double)N - sigma * sigma, 0.0) / (double)(N - 1)) : 0.0;
    free(acc);
    if (!w_out) free(w);
    return threads;
}
