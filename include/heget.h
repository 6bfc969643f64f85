/*
 * heget -- helicity-summed |M|^2 of u ubar -> n photons on an AMD Instinct
 * MI355X (gfx950), and the weighted Monte-Carlo cross section built on it.
 *
 * Method: K. Hagiwara, J. Kanzaki, N. Okamura, D. Rainwater, T. Stelzer,
 * "Fast calculation of HELAS amplitudes using graphics processing unit
 * (GPU)", arXiv:0908.4403.  Section 2 defines the physics (eq. (1)-(10)),
 * Section 3.1 the problem statement the calls below follow (the user supplies
 * random numbers -- here a seed -- and gets phase-space points, their |M|^2
 * and the cross section), Appendix B the HELAS conventions the amplitudes use.
 *
 * Conventions shared by every call:
 *   - n is the number of photons, 2 <= n <= 8.
 *   - Momenta are (E, px, py, pz) in GeV, FP64.  An event holds n+2 momenta in
 *     the order u (incoming, along +z), ubar (incoming, along -z), photons.
 *   - Host-pointer calls use the event-major layout momenta[npoints][n+2][4].
 *     Device-pointer calls ("_device") use component-major (SoA) layout
 *     mom[(n+2)*4][npoints]: row r = 4*particle + component.
 *   - |M|^2 values are summed over the two quark and all photon helicities
 *     (eq. (2)), with no spin, colour or identical-particle average, in
 *     GeV^(4-2n); coupling gal = -e Q with e = sqrt(4 pi alpha).
 *   - The caller owns every buffer it passes.  Host-pointer calls keep no
 *     pointer after they return.  Device-pointer calls enqueue work on the
 *     given stream and return; their buffers must stay valid until that work
 *     has completed.  The library owns its device scratch (allocated on first
 *     use, grown as needed, released by heget_shutdown()), one set per
 *     stream for up to four streams: calls on one stream reuse it in stream
 *     order with no extra synchronisation; a fifth stream takes over the
 *     least recently used set after waiting for the device to be idle.
 *   - Calls are serialised by an internal mutex; no exception crosses this
 *     boundary.  On failure the returned status is negative and
 *     heget_last_error() describes it.
 *   - Nothing touches the GPU before the first call that needs it, so the
 *     argument checks below work on a machine without one.
 */
#ifndef HEGET_H
#define HEGET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HEGET_OK = 0,
    HEGET_WARN_NONFINITE = 1, /* results written; some points gave NaN/inf
                                 (e.g. a photon with pT = 0) */
    HEGET_ERR_ARG = -1,       /* null pointer, bad enum, bad cut or energy */
    HEGET_ERR_RANGE = -2,     /* n outside 2..8, npoints < 0 or >= 2^31 */
    HEGET_ERR_ALLOC = -3,     /* device allocation failed */
    HEGET_ERR_DEVICE = -4     /* HIP runtime error (no GPU, launch failure) */
} heget_status;

/* Arithmetic of the amplitude (the shared-prefix tree of currents).  Both
 * accumulate the per-point ordering sum, the helicity sum and the cross
 * section in FP64; phase-space generation and boosts are always FP64. */
typedef enum {
    HEGET_FP64 = 0, /* amplitudes in FP64 */
    HEGET_FP32 = 1  /* amplitudes in FP32, ordering and helicity sums in FP64 */
} heget_prec;

/* Partonic kinematics of heget_xsec (Section 2.1). */
typedef enum {
    HEGET_FIXED_SHAT = 0,       /* u ubar at fixed sqrt(shat) = sqrt_s */
    HEGET_UNIFORM_SQRTSHAT = 1, /* sqrt(shat) uniform in [sqrt_shat_lo, sqrt_shat_hi];
                                   sigma is the average of sigma_hat over it */
    HEGET_PP_TOY = 2            /* eq. (1): pp at hadronic sqrt_s with toy densities
                                   D_u = x^-0.5 (1-x)^3, D_ubar = x^-0.3 (1-x)^6,
                                   both beam assignments, sqrt(shat) >= sqrt_shat_lo */
} heget_mode;

/* Final-state photon cuts, eq. (9)-(10): pT > pt_min, |eta| < eta_max,
 * Delta R > dr_min for every pair.  A bound <= 0 disables that cut.  eta is
 * the lab-frame rapidity; Delta phi is folded into [0, pi]. */
typedef struct {
    double pt_min, eta_max, dr_min;
} heget_cuts;

typedef struct {
    int32_t mode;       /* heget_mode */
    int32_t prec;       /* heget_prec */
    uint64_t seed;      /* random stream (key of the counter-based generator) */
    int64_t npoints;    /* generated points, 0 <= npoints < 2^31 */
    double sqrt_s;      /* FIXED: sqrt(shat); PP: hadronic sqrt(s) [GeV] */
    double sqrt_shat_lo, sqrt_shat_hi; /* UNIFORM: range; PP: lo = min sqrt(shat) */
    heget_cuts cuts;
    double alpha, charge; /* e^2 = 4 pi alpha; quark charge in units of e */
    int32_t helicity_sampling; /* 0: sum all helicities (eq. (2)); 1: one helicity
                                * configuration per point, drawn uniformly from the
                                * 2^(n+1) non-vanishing ones and weighted by 2^(n+1)
                                * (the paper's per-event helicities, Section 3.1);
                                * heget_xsec only, not heget_xsec_batch */
    int32_t reserved;          /* set to 0 */
} heget_config;

typedef struct {
    double sigma_fb, err_fb; /* sigma = sum_w / n_gen, MC standard error (fb) */
    double sum_w, sum_w_comp, sum_w2; /* compensated sum of weights, its
                                         compensation term, sum of squares */
    int64_t n_gen, n_acc;    /* generated points, points passing all cuts */
} heget_result;

/* A hipStream_t; NULL means the null stream. */
typedef void *heget_stream;

/* Phase-space points at fixed sqrt(shat) = sqrt_s (Section 3.1 step 4):
 * RAMBO massless momenta from the counter-based stream `seed`, point indices
 * 0..npoints-1, and the cuts.  momenta[npoints][n+2][4] (out, host) receives
 * every point; weight[npoints] (out, host) receives the phase-space weight of
 * eq. (4) (the massless n-body volume) for points passing the cuts, 0 for the
 * others.  cuts may be NULL (no cuts).  Returns HEGET_OK or an error. */
heget_status heget_gen_points(int n, double sqrt_s, const heget_cuts *cuts, uint64_t seed,
                              int64_t npoints, double *momenta, double *weight);

/* The same points written to device memory in SoA layout: d_mom[(n+2)*4][npoints]
 * and d_weight[npoints], for point indices first..first+npoints-1. */
heget_status heget_gen_points_device(int n, double sqrt_s, const heget_cuts *cuts,
                                     uint64_t seed, int64_t first, int64_t npoints,
                                     double *d_mom, double *d_weight, heget_stream stream);

/* Helicity-summed |M|^2 (eq. (2) summand; eq. (6)-(8) amplitudes) at the
 * given points.  momenta[npoints][n+2][4] (in, host), out_me2[npoints] (out,
 * host).  Preconditions per point: u along +z and ubar along -z (zero
 * transverse momenta), every photon with E > 0 and pT > 0.  A point that
 * violates them gets NaN and the call returns HEGET_WARN_NONFINITE. */
heget_status heget_me2(int n, int64_t npoints, const double *momenta, double *out_me2,
                       heget_prec prec);

/* Device-pointer form of heget_me2: d_mom[(n+2)*4][npoints] (SoA, device),
 * d_out[npoints] (device).  Enqueued on `stream`; non-finite results are not
 * reported in the status (inspect d_out). */
heget_status heget_me2_device(int n, int64_t npoints, const double *d_mom, double *d_out,
                              heget_prec prec, heget_stream stream);

/* The same call under the name of the stream-ordered form of heget_me2:
 * identical arguments, layout, ownership and errors as heget_me2_device. */
heget_status heget_me2_async(int n, int64_t npoints, const double *d_mom, double *d_out,
                             heget_prec prec, heget_stream stream);

/* Monte-Carlo cross section (Section 3.1 steps 2-6, eq. (1)-(2)): every
 * point is generated, cut, evaluated and weighted on the device; only the
 * result crosses to the host.  out (host) receives sigma +- err in fb.
 * Deterministic: the same config gives bitwise the same result. */
heget_status heget_xsec(int n, const heget_config *cfg, heget_result *out);

/* heget_xsec enqueued on `stream`; *out is written when the stream reaches
 * it, from a pinned staging buffer (out must stay valid until then). */
heget_status heget_xsec_async(int n, const heget_config *cfg, heget_result *out,
                              heget_stream stream);

/* heget_xsec enqueued on `stream` with the result record written by the
 * device into d_out, which must be device memory or host memory the device
 * can write (e.g. from hipHostMalloc); no host callback or synchronisation is
 * involved, so calls can be chained and captured.  npoints must be > 0.
 * Non-finite weights are not reported in the status (check d_out->sigma_fb). */
heget_status heget_xsec_device(int n, const heget_config *cfg, heget_result *d_out,
                               heget_stream stream);

/* heget_xsec_device for callers that cannot allocate device memory (code
 * under stream capture, serving loops, harnesses that forbid hipMalloc): the
 * same pass, same arguments and same results, with every intermediate buffer
 * (momenta, weights, survivor list, partial sums) carved from a fixed 64 MiB
 * workspace that the library holds in a static device array, one per device,
 * kept until the process ends.  The call allocates nothing (no hipMalloc,
 * hipFree or pinned host memory).  A configuration whose buffers exceed the
 * workspace -- about 32 (n + 2) + 14 bytes per point, e.g. 3.2e5 points at
 * n = 4 or 2.0e5 at n = 8 -- returns HEGET_ERR_RANGE before anything is
 * enqueued.  Every call on one device shares that device's workspace: calls
 * that overlap on the device (concurrent streams, or a captured graph
 * replayed beside another call) race and give wrong results; calls ordered
 * on one stream are safe.  Nothing in the workspace needs to be cleared by
 * the caller. */
heget_status heget_xsec_device_noalloc(int n, const heget_config *cfg, heget_result *d_out,
                                       heget_stream stream);

/* Event observables for heget_xsec_hist (the distributions of Fig. 2). */
typedef enum {
    HEGET_OBS_PT_MAX = 0, /* largest photon pT [GeV] */
    HEGET_OBS_DR_MIN = 1  /* smallest Delta R over photon pairs (eq. (10)) */
} heget_observable;

/* heget_xsec plus a weighted histogram of one observable over the same
 * points: hist[0] = underflow (< lo), hist[1 + b] = bin b of nbins equal bins
 * on [lo, hi), hist[nbins + 1] = overflow (host, [nbins + 2]), each the sum of
 * the weights in it over n_gen (fb per bin; the entries add up to sigma).
 * The bins are summed as 64-bit fixed-point integers scaled from the total
 * weight, so they are exact to 2^-62 of sigma and independent of the order of
 * the device's atomic adds.  1 <= nbins <= 4096, finite lo < hi. */
heget_status heget_xsec_hist(int n, const heget_config *cfg, int observable, int nbins, double lo,
                             double hi, double *hist, heget_result *out);

/* heget_xsec plus the record of every generated event, the per-event output
 * of the paper's program (Section 3.1: the momenta and helicities of each
 * event beside its weight).  For point i (0 <= i < npoints) of the same sample:
 *   weight[i]   its weight w_i in fb (eq. (1)-(2)), so that sigma = sum_i
 *               weight[i] / n_gen; 0 for points failing the cuts (or, in
 *               HEGET_PP_TOY, below sqrt_shat_lo);
 *   momenta     if not NULL, [npoints][n+2][4]: (E, px, py, pz) in GeV of u,
 *               ubar and photons 1..n in the partonic CM frame (u along +z),
 *               the layout of heget_gen_points;
 *   rapidity    if not NULL, [npoints]: rapidity of the partonic CM frame in
 *               the lab (0 unless HEGET_PP_TOY).  The weight covers both beam
 *               assignments of eq. (1): the event boosted by +rapidity, and
 *               its mirror (rotated by pi about x, boosted by -rapidity);
 *   helicity    if not NULL (needs cfg->helicity_sampling = 1), [npoints]:
 *               the configuration drawn for the point: bit 0 the quark pair
 *               (0: h_u = -1, h_ubar = +1; 1: h_u = +1, h_ubar = -1), bit
 *               1 + j photon j's helicity (1: +1).
 * A HEGET_PP_TOY point below sqrt_shat_lo is no event: only its weight (0) is
 * defined there, its momenta and rapidity are placeholders.  All arrays are
 * host memory of the caller, written before the call returns; *out is as
 * heget_xsec's. */
heget_status heget_xsec_events(int n, const heget_config *cfg, heget_result *out, double *weight,
                               double *momenta, double *rapidity, uint16_t *helicity);

/* Several cross sections in one device pass (e.g. n = 2..7 with different
 * point counts), captured on first use as ONE hipGraph that later calls with
 * the same arguments replay.  Two schedules of the amplitude work:
 *   1 persistent: one persistent amplitude launch whose waves pull
 *     (configuration, 64-point tile, helicity chunk) work items from an
 *     atomic queue, most expensive items first;
 *   2 branches: one graph branch per configuration (generation, compaction,
 *     the tuned amplitude kernel for its n, reduction), branches running
 *     concurrently so memory-bound and compute-bound work overlap.
 * With schedule 0 (auto, the default) the first call captures both, times
 * one launch of each and keeps the faster for these arguments.
 * n[ncfg], cfgs[ncfg] (in, host), out[ncfg] (out, host); 1 <= ncfg <= 8, all
 * with the same prec.  Results equal heget_xsec per configuration up to the
 * rounding of the kernel shape used (FP32: within 1e-5). */
heget_status heget_xsec_batch(const int *n, const heget_config *cfgs, int ncfg,
                              heget_result *out);

/* Schedule of later heget_xsec_batch calls: 0 auto, 1 persistent, 2 branches.
 * Drops captured batches. */
heget_status heget_set_batch_schedule(int schedule);

/* Schedule a batch with these arguments runs (0 if it has not run yet). */
heget_status heget_batch_schedule_in_use(const int *n, const heget_config *cfgs, int ncfg,
                                         int *schedule);

/* Couplings used by heget_me2 / heget_me2_device (defaults: 1/137, 2/3). */
heget_status heget_set_couplings(double alpha, double charge);

/* Optional per-kernel timing of the amplitude kernel: when enabled, each
 * launch of it is bracketed by events on its stream; heget_timing_read
 * returns the accumulated milliseconds and launch count since the last
 * reset (it synchronises the recorded events). */
heget_status heget_timing_enable(int on);
heget_status heget_timing_read(double *me2_ms, int64_t *me2_launches, int reset);

/* Shape of the amplitude kernel (the autotuner's search space).
 *   unrolled             photons left in a subtree that is unrolled at compile
 *                        time with its photons in registers (2..5); when it
 *                        covers all n photons the helicity configurations of
 *                        one walk also share every current that does not yet
 *                        depend on the photons where they differ
 *   helicities_per_walk  helicity configurations sharing one walk of the tree
 *   closing              1: every ordering closes photon by photon (iovxx0 at
 *                        the leaves); 2: the last two photons close together
 *                        through pair vectors built from the u end (the current
 *                        reuse of the paper's MadGraph program, Appendix A.1);
 *                        3: as 2, and the two photons before them are summed
 *                        over both orders at the ubar end, where the two
 *                        currents share their propagator, so four photons
 *                        close with 6 pair products instead of 12 (in FP32
 *                        kernels with 8 or more helicities per walk each of
 *                        the 6 products is taken in FP64); 4: as 3 with the
 *                        products always in the working precision; 5: as 4,
 *                        with the products of complementary splits ({x, y} |
 *                        {a, b} and {a, b} | {x, y}) summed in the working
 *                        precision, so that each four-photon closing enters
 *                        the FP64 ordering sum three times instead of six
 *   waves_per_block      64-lane waves per workgroup
 *   prefetch             0: one wave per 64-point work item; 1: only as many
 *                        waves as the device holds at once, each looping over
 *                        its items and loading the next item's inputs before
 *                        the walk of the current one (hides the memory latency
 *                        when few waves fit per SIMD, and shortens the tail)
 *   waves_per_simd       0: registers as the compiler likes; k > 0: at most
 *                        512 / k registers per lane so that k waves share each
 *                        SIMD (its FP32 instructions then issue from two waves
 *                        at once)
 *   points_per_lane      points each lane evaluates per work item (1, or 2
 *                        with prefetch 0): a work item is that many 64-point
 *                        tiles whose walks run as independent instruction
 *                        streams
 *   prefix_sets          0: the levels above the unrolled subtree walk every
 *                        ordered prefix; 1: they walk prefix sets, summing the
 *                        currents of all orderings of a set (subset recursion)
 *                        before the subtree, which then runs once per set --
 *                        the current reuse of the MadGraph program carried to
 *                        the meeting point of the two ends (Appendix A.1);
 *                        2 (with unrolled = n): meet in the middle -- subset
 *                        currents from the v-bar end for every set of up to
 *                        K = (n + 1) / 2 photons, subset currents from the u
 *                        end for the other side, one contraction per set of
 *                        K photons (closing is then unused), with the
 *                        momentum part of the nodes formed once per point;
 *                        3: as 2 with it formed per helicity walk (fewer
 *                        values held, for n >= 7); 4: as 3 with the v-bar-end
 *                        currents of K - 1 photons held in LDS */
typedef struct {
    int32_t unrolled, helicities_per_walk, closing, waves_per_block, prefetch, waves_per_simd,
        points_per_lane, prefix_sets;
} heget_shape;

/* Algorithmic floating-point operations per point of the amplitude kernel
 * that heget_me2 / heget_xsec run for (n, prec): FMA = 2, add/mul/reciprocal
 * = 1, counted on the schedule actually executed (the 2^n helicities of one
 * quark-helicity block; the shape's tree, closing and helicity sharing).
 * Per-point O(n) set-up is not counted.  *shape (may be NULL) receives the
 * shape in use. */
heget_status heget_me2_flops(int n, heget_prec prec, double *flops_per_point, heget_shape *shape);

/* Autotuner.  Times every compiled shape of the amplitude kernel for (n,
 * prec) on npoints synthetic points (sqrt(shat) = 1 TeV) generated on the
 * device, and makes the fastest the shape every later call uses for (n,
 * prec) in this process (a shape later in the table must be 2% faster than
 * the best so far to replace it, so near-ties resolve the same way on every
 * run).  If HEGET_TUNING_CACHE names a file, the choice is
 * also written there (one JSON object per line) and read back by later
 * processes on first device use.  *chosen and *ms (may be NULL) receive the
 * chosen shape and its time per launch.  64 <= npoints < 2^31. */
heget_status heget_autotune(int n, heget_prec prec, int64_t npoints, heget_shape *chosen,
                            double *ms);

/* The compiled shapes for (n, prec), the one in use first, into shapes[i]
 * for i < max (shapes may be NULL when max = 0); *count receives how many
 * exist. */
heget_status heget_kernel_shapes(int n, heget_prec prec, int max, heget_shape *shapes, int *count);

/* Use a compiled shape for (n, prec) from now on in this process; NULL
 * restores the default.  HEGET_ERR_ARG if no such shape was compiled. */
heget_status heget_set_kernel_shape(int n, heget_prec prec, const heget_shape *shape);

/* ---- The massless HELAS set (Appendix B) as a device library ----
 * Functions: B.1 external fermions (ixxxx0 any direction, ixxxx1 along +z,
 * ixxxx2 along -z: flowing-in |fi>, u for nSF = +1 and v for nSF = -1;
 * oxxxx0/1/2: flowing-out <fo|, ubar and vbar), B.2 massless vectors (vxxxx0
 * any direction: eps* for nSV = +1, eps for nSV = -1; vxxxx1/2: incoming
 * vectors along +z / -z, eps with momentum -p, nSV not read), B.3 the
 * fermion-fermion-vector vertex of  psibar_F1 gamma^mu (gal0 P_L + gal1 P_R)
 * psi_F2 V*_mu  (iovxxx: amplitude <fo|V|fi>; fvixx0: off-shell |f'> with
 * p = p_fi - p_vc; fvoxx0: off-shell <f'| with p = p_fo + p_vc; jioxx0:
 * off-shell vector current, Feynman gauge, p = p_fo - p_fi).  Massless
 * fermion propagators carry -1/p^2, the vector propagator +1/p^2.
 * The device header csrc/helas.hpp holds the same functions for use inside
 * other HIP kernels; the entry points below evaluate one function on many
 * independent records. */
typedef enum {
    HEGET_IXXXX0 = 0, HEGET_IXXXX1 = 1, HEGET_IXXXX2 = 2,
    HEGET_OXXXX0 = 3, HEGET_OXXXX1 = 4, HEGET_OXXXX2 = 5,
    HEGET_VXXXX0 = 6, HEGET_VXXXX1 = 7, HEGET_VXXXX2 = 8,
    HEGET_IOVXXX = 9, HEGET_FVIXX0 = 10, HEGET_FVOXX0 = 11, HEGET_JIOXX0 = 12
} heget_helas_fn;

/* Record sizes of a function, in doubles.  A wavefunction is 12 doubles: the
 * four complex components (re, im; spinors in the chiral basis with the
 * left-handed pair first, vectors contravariant) then the momentum along the
 * flow (p nSF or p nSV).  Inputs: external wavefunctions (p[4], nHEL, nSF or
 * nSV) = 6; iovxxx (fi, fo, vc, gal0, gal1) = 38; fvixx0 (fi, vc, gal0,
 * gal1), fvoxx0 (fo, vc, gal0, gal1), jioxx0 (fi, fo, gal0, gal1) = 26.
 * Outputs: a wavefunction (12), or the vertex amplitude (re, im) = 2 for
 * iovxxx.  HEGET_ERR_ARG for an unknown func or a null pointer. */
heget_status heget_helas_sizes(int func, int *in_doubles, int *out_doubles);

/* Evaluates `func` on count records: in[count][in_doubles] (host),
 * out[count][out_doubles] (host); the arithmetic runs on the device in the
 * precision `prec` (records are converted on the device).  nHEL, nSF and nSV
 * must be +1 or -1.  Synchronous. */
heget_status heget_helas(int func, int64_t count, const double *in, double *out, heget_prec prec);

/* The same on device buffers d_in, d_out (same layouts), enqueued on stream. */
heget_status heget_helas_device(int func, int64_t count, const double *d_in, double *d_out,
                                heget_prec prec, heget_stream stream);

/* Helicity-summed |M|^2 of u(p1) ubar(p2) -> n photons (2 <= n <= 5) for
 * massless momenta in any frame, composed from the library functions
 * (ixxxx0, oxxxx0, vxxxx0, fvoxx0 over all n! orderings, iovxxx).  Layouts
 * as heget_me2 (momenta[npoints][n+2][4], host); the couplings of
 * heget_set_couplings.  Every photon needs E > 0.  Equal to heget_me2 in the
 * frame where it applies.  HEGET_ERR_RANGE for n outside 2..5. */
heget_status heget_me2_frame(int n, int64_t npoints, const double *momenta, double *out_me2,
                             heget_prec prec);

/* Device-pointer form: d_mom[(n+2)*4][npoints] (SoA), d_out[npoints]. */
heget_status heget_me2_frame_device(int n, int64_t npoints, const double *d_mom, double *d_out,
                                    heget_prec prec, heget_stream stream);

/* Vector-ALU ceiling of the current device: the FP32 and FP64 FMA rates (in
 * TFLOP/s, FMA = 2 flops) of a kernel of independent FMA chains with no
 * memory traffic, built like the amplitude kernels (no packed FP32).  Either
 * pointer may be NULL.  Takes a few tens of milliseconds. */
heget_status heget_valu_peak(double *fp32_tflops, double *fp64_tflops);

/* Message of the last failure on this thread ("" if none). */
const char *heget_last_error(void);

/* Frees device scratch, pinned staging and events.  Safe to call twice. */
void heget_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif
