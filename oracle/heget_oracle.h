/*
 * FP64 CPU oracle for the helicity-summed |M|^2 of u ubar -> n photons.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__.py
 * and the cpu_baseline leg of bench.py may load this library.  It shares no
 * code, header or constant with the HIP library under paper_0908_4403_amd/.
 *
 * Everything here is a plain, slow, literal restatement of the paper
 * (Hagiwara, Kanzaki, Okamura, Rainwater, Stelzer, "Fast calculation of HELAS
 * amplitudes using graphics processing unit (GPU)", arXiv:0908.4403):
 *   - eq. (1)-(4): pp factorisation, partonic cross section, phase space;
 *   - eq. (6)-(8): amplitude = sum over n! photon orderings of one chain;
 *   - eq. (9)-(10): photon cuts;
 *   - Appendix B: HELAS conventions of the wavefunction and FFV vertex
 *     functions (ixxxx1, oxxxx2, vxxxx0, iovxx0, fvoxx0, fvixx0), here written
 *     from their definitions with explicit 4x4 Dirac matrices;
 *   - Appendix A.2: amplitude = sum over orderings of a chain of fvoxx0
 *     currents closed by iovxx0.
 * Choices the paper leaves open (phase-space generator, random numbers,
 * alpha, toy parton densities) follow the published methods named where they
 * are used.  Parity of each function is pinned by the -m "not gpu" tests.
 *
 * Conventions: momenta are (E, px, py, pz) in GeV.  An event is an array
 * p[n+2][4]: p[0] = u quark (incoming), p[1] = ubar (incoming), p[2..n+1] =
 * photons (outgoing).
 */
#ifndef HEGET_ORACLE_H
#define HEGET_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- counter-based random numbers (Philox4x32-10, Salmon et al., SC'11) ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Counter = {lo32(point), hi32(point), block, stream}, key = {lo32(seed),
 * hi32(seed)}.  orc_uniform_quad: four uniforms in (0,1), one per word,
 * (w_j + 1/2) * 2^-32 (the photons).  orc_uniform_pair: two uniforms, u[0]
 * from words (1:0), u[1] from words (3:2), each (top 53 bits + 1/2) * 2^-53
 * (the partonic kinematics). */
void orc_uniform_quad(uint64_t seed, uint64_t point, uint32_t block, uint32_t stream,
                      double u[4]);
void orc_uniform_pair(uint64_t seed, uint64_t point, uint32_t block, uint32_t stream,
                      double u[2]);

/* ---- phase space (RAMBO, Kleiss, Stirling, Ellis, CPC 40 (1986) 359) ---- */
/* n massless momenta k[n][4] with sum (sqrt_s, 0,0,0) from 4n uniforms
 * (u[4i..4i+3] for photon i: cos theta, phi, and two for the energy). */
void orc_rambo(int n, double sqrt_s, const double *u, double *k);
/* constant RAMBO weight = volume of massless n-body phase space of eq. (4) */
double orc_rambo_weight(int n, double s);
/* CM event p[n+2][4] at sqrt_shat for point `point` of stream `seed`
 * (u along +z, ubar along -z, photons from RAMBO with stream-0 blocks 0..n-1). */
void orc_cm_event(int n, double sqrt_shat, uint64_t seed, uint64_t point, double *p);
/* points first .. first+np-1 into p_aos[np][n+2][4] (OpenMP) */
void orc_cm_events(int n, double sqrt_shat, uint64_t seed, uint64_t first, int64_t np,
                   double *p_aos);

/* ---- cuts of eq. (9)-(10) ---- */
/* 1 if every photon passes pT > pt_min, |eta + y| < eta_max and every pair
 * has Delta R > dr_min (a bound <= 0 disables that cut); photons k[n][4]
 * given in a frame boosted by rapidity y along z w.r.t. the lab. */
int orc_pass_cuts(int n, const double *k, double y, double pt_min, double eta_max,
                  double dr_min);

/* ---- amplitudes ---- */
/* Helicity amplitude of eq. (6)-(8) for quark helicities h1 (u), h2 (ubar)
 * and photon helicities lam[n] (each +-1), as the sum over all n! orderings
 * of chains built from the ubar end with fvoxx0 and closed with iovxx0
 * (Appendix A.2).  `u_along_minus_z` = 0: u moves along +z (p[0]), ubar
 * along -z; = 1: u along -z, ubar along +z.  g = coupling gal[0]=gal[1]. */
void orc_amp(int n, const double *p, int h1, int h2, const int *lam, double g,
             int u_along_minus_z, double *re, double *im);
/* The same amplitude built from the u end with fvixx0 currents. */
void orc_amp_from_u(int n, const double *p, int h1, int h2, const int *lam, double g,
                    double *re, double *im);
/* Amplitude with arbitrary complex polarisation 4-vectors eps[n][4] (re, im
 * interleaved: eps[(i*4+mu)*2+{0,1}]) in place of the photon wavefunctions;
 * used for the gauge-invariance check.  Also returns sum_orderings |diagram|. */
void orc_amp_custom_eps(int n, const double *p, int h1, int h2, const double *eps,
                        double g, double *re, double *im, double *sum_abs);
/* Two-sided schedule of Appendix A.1 (outgoing current from the ubar end
 * meets an incoming current from the u end); split < 0 varies the meeting
 * vertex with the ordering. */
void orc_amp_meet(int n, const double *p, int h1, int h2, const int *lam, double g,
                  int split, double *re, double *im);

/* Helicity-summed |M|^2 = sum over h1,h2 = +-1 and lam in {+-1}^n of |amp|^2
 * with g = -e*charge, e = sqrt(4 pi alpha) (units GeV^(4-2n)).
 * skip_zero = 1 skips h1 == h2, which vanish identically (chirality). */
double orc_me2(int n, const double *p, double alpha, double charge, int skip_zero,
               int u_along_minus_z);
/* OpenMP batch over points: p_aos[np][n+2][4] -> out[np]; returns threads used. */
/* OpenMP threads of the batch functions (k <= 0: the default); returns it. */
int orc_set_threads(int k);
int orc_me2_batch(int n, int64_t np, const double *p_aos, double alpha, double charge,
                  double *out);
/* Same |M|^2 by the subset (Berends-Giele) recursion of the same currents:
 * J(S) = sum_{j in S} fvoxx0(J(S\{j}), eps_j).  Cross-check only. */
double orc_me2_subsets(int n, const double *p, double alpha, double charge);
int orc_me2_subsets_batch(int n, int64_t np, const double *p_aos, double alpha,
                          double charge, double *out);

/* ---- cross section ---- */
enum { ORC_FIXED_SHAT = 0, ORC_UNIFORM_SQRTSHAT = 1, ORC_PP_TOY = 2 };
typedef struct {
    int mode;            /* ORC_* */
    uint64_t seed;
    int64_t npoints;     /* generated points */
    int64_t first_point; /* index of the first point (sub-samples of a stream) */
    double sqrt_s;       /* fixed sqrt(shat), or hadronic sqrt(s) for PP */
    double sqrt_shat_lo, sqrt_shat_hi; /* uniform range; PP: lo = min sqrt(shat) */
    double pt_min, eta_max, dr_min;
    double alpha, charge;
    int me2_method;      /* 0: sum over orderings (orc_me2); 1: subset recursion */
    int helicity_sampling; /* 1: one helicity configuration per point (see orc_point) */
} orc_config;

typedef struct {
    double sigma_fb, err_fb, sum_w, sum_w_comp, sum_w2;
    int64_t n_gen, n_acc;
} orc_result;

/* Per-point weight w (fb) of point `point` (0 if cut or below threshold),
 * and its event: p[n+2][4] in the partonic CM frame (u along +z), the boost
 * rapidity y to the lab and the |M|^2 used.  Returns 1 if accepted.
 * With helicity_sampling the |M|^2 used is the estimator 2^(n+1) |M_h|^2 of
 * the one configuration h drawn by orc_draw_helicity for the point. */
int orc_point(int n, const orc_config *cfg, uint64_t point, double *p, double *y,
              double *me2, double *w);
/* OpenMP over points, then a fixed-order Neumaier sum; returns threads used. */
int orc_xsec(int n, const orc_config *cfg, orc_result *out, double *w_out);

/* The helicity configuration point `point` draws in sampling mode (the
 * paper's per-event helicities, Section 3.1): word 0 of Philox4x32-10 at
 * counter {lo(point), hi(point), 0, 2}, key = seed.  Bit 0 picks the quark
 * pair (0: h_u = -1, h_ubar = +1; 1: h_u = +1, h_ubar = -1), bit 1 + i the
 * helicity of photon i (1: +1).  These are the 2^(n+1) configurations with a
 * non-vanishing amplitude, drawn uniformly. */
void orc_draw_helicity(int n, uint64_t seed, uint64_t point, int *h1, int *h2, int *lam);

/* Event observables of Fig. 2 (photons k[n][4]): 0 = largest photon pT
 * (GeV); 1 = smallest Delta R over photon pairs (Delta phi folded into
 * [0, pi]; both are unchanged by the longitudinal boost to the lab). */
double orc_observable(int n, const double *k, int observable);

/* Weighted histogram of an observable: hist[0] = underflow (< lo), hist[1 +
 * b] = bin b of nbins equal bins on [lo, hi), hist[nbins + 1] = overflow,
 * each the sum of w over the points in it divided by N (fb per bin; the
 * entries add up to sigma).  Same points and weights as orc_xsec; the sums
 * are Neumaier sums in point order.  Returns the threads used. */
int orc_hist(int n, const orc_config *cfg, int observable, int nbins, double lo, double hi,
             double *hist);

/* The massless HELAS set of Appendix B on one record, for the device
 * library's tests.  func: 0-2 ixxxx0/1/2, 3-5 oxxxx0/1/2, 6-8 vxxxx0/1/2 (in
 * = p[4], nhel, nsf or nsv; vxxxx1/2 give the incoming vector eps(p) with
 * momentum -p whatever nsv says), 9 iovxxx (in = fi, fo, vc, gal0, gal1; out = re,
 * im), 10 fvixx0 (fi, vc, gal0, gal1), 11 fvoxx0 (fo, vc, gal0, gal1),
 * 12 jioxx0 (fi, fo, gal0, gal1).  A wavefunction is 12 doubles: four complex
 * components (re, im) then the momentum along the flow.  Returns the number
 * of doubles written, or -1 for an unknown func. */
int orc_helas(int func, const double *in, double *out);

/* Helicity-summed |M|^2 of u(p1) ubar(p2) -> n photons for momenta in any
 * frame (p = p1, p2, k1..kn, (n+2)*4 doubles), built from ixxxx0, oxxxx0,
 * vxxxx0, fvoxx0 and iovxxx; all 2^(n+2) helicities summed. */
double orc_me2_frame(int n, const double *p, double alpha, double charge);

/* Helicity-summed |M|^2 of f(p1) fbar(p2) -> f'(p3) fbar'(p4) through one
 * photon (jioxx0 closed with iovxxx); charges q1, q2 in units of e. */
double orc_me2_ffff(const double *p, double alpha, double q1, double q2);

/* (hbar c)^2 in GeV^2 fb */
double orc_gev2_fb(void);

#ifdef __cplusplus
}
#endif

#endif
