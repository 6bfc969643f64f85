// C ABI of libheget (include/heget.h): argument checks, the launch plan, the
// library-owned device scratch and the call sequences.  Host code only; all
// arithmetic of the path runs in the kernels of me2_kernels.hip and
// mc_kernels.hip.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "heget.h"
#include "kernels.hpp"

namespace {

std::mutex g_mu;
thread_local std::string g_err;

double g_alpha = 1.0 / 137.0;
double g_charge = 2.0 / 3.0;

constexpr double kGeV2fb = 0.3893793721e12;  // (hbar c)^2 in GeV^2 fb
constexpr int64_t kMaxPoints = (int64_t(1) << 31) - 1;

heget_status fail(heget_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define HG_HIP(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? HEGET_ERR_ALLOC : HEGET_ERR_DEVICE,        \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    } while (0)

#define HG_TRY(expr)                                                                          \
    do {                                                                                      \
        heget_status s_ = (expr);                                                             \
        if (s_ < 0) return s_;                                                                \
    } while (0)

// ---------------------------------------------------------------- device state

struct State {
    bool ready = false;
    int device = -1;
    hipStream_t stream = nullptr;     // library stream for the synchronous calls
    hipEvent_t ws_free = nullptr;     // recorded after every use of the scratch
    std::vector<void *> buf;          // scratch slots
    std::vector<size_t> cap;
    double *pinned = nullptr;         // staging ring for results (kRing slots of 8 doubles)
    std::atomic<unsigned> ring{0};
    // timing of the amplitude kernel
    bool timing = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    double ms_total = 0.0;
    int64_t launches = 0;
};
State g;
constexpr int kRing = 256;

enum Slot {
    S_MOM, S_WFAC, S_FLAG, S_BCOUNT, S_OFFS, S_COUNT, S_INDEX, S_PART, S_ME2, S_PARTIALS, S_RES,
    S_FLAGS, S_OUT, S_NSLOTS
};

heget_status ensure_device()
{
    if (g.ready) return HEGET_OK;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0)
        return fail(HEGET_ERR_DEVICE, "no HIP device available");
    HG_HIP(hipGetDevice(&g.device));
    HG_HIP(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
    HG_HIP(hipEventCreateWithFlags(&g.ws_free, hipEventDisableTiming));
    HG_HIP(hipHostMalloc(reinterpret_cast<void **>(&g.pinned), sizeof(double) * 8 * kRing,
                         hipHostMallocDefault));
    g.buf.assign(S_NSLOTS, nullptr);
    g.cap.assign(S_NSLOTS, 0);
    g.ready = true;
    return HEGET_OK;
}

// Scratch slot of at least `bytes`; grows (after the device is idle) when short.
heget_status scratch(int slot, size_t bytes, void **out)
{
    bytes = bytes < 256 ? 256 : bytes;
    if (g.cap[slot] < bytes) {
        HG_HIP(hipDeviceSynchronize());
        if (g.buf[slot]) HG_HIP(hipFree(g.buf[slot]));
        g.buf[slot] = nullptr;
        g.cap[slot] = 0;
        size_t want = bytes + bytes / 4;
        HG_HIP(hipMalloc(&g.buf[slot], want));
        g.cap[slot] = want;
    }
    *out = g.buf[slot];
    return HEGET_OK;
}

template <typename T>
heget_status scratch_t(int slot, size_t count, T **out)
{
    void *p = nullptr;
    HG_TRY(scratch(slot, count * sizeof(T), &p));
    *out = static_cast<T *>(p);
    return HEGET_OK;
}

// Scratch users on different streams are ordered through one event.
heget_status scratch_acquire(hipStream_t s)
{
    HG_HIP(hipStreamWaitEvent(s, g.ws_free, 0));
    return HEGET_OK;
}

heget_status scratch_release(hipStream_t s)
{
    HG_HIP(hipEventRecord(g.ws_free, s));
    return HEGET_OK;
}

// ---------------------------------------------------------------- checks

heget_status check_n(int n)
{
    if (n < 2 || n > 8) return fail(HEGET_ERR_RANGE, "n must be in 2..8, got " + std::to_string(n));
    return HEGET_OK;
}

heget_status check_np(int64_t np)
{
    if (np < 0 || np > kMaxPoints)
        return fail(HEGET_ERR_RANGE, "npoints must be in [0, 2^31), got " + std::to_string(np));
    return HEGET_OK;
}

heget_status check_prec(int prec)
{
    if (prec != HEGET_FP64 && prec != HEGET_FP32)
        return fail(HEGET_ERR_ARG, "prec must be HEGET_FP64 or HEGET_FP32");
    return HEGET_OK;
}

heget_status check_cuts(const heget_cuts *c)
{
    if (c && !(std::isfinite(c->pt_min) && std::isfinite(c->eta_max) && std::isfinite(c->dr_min)))
        return fail(HEGET_ERR_ARG, "cut values must be finite");
    return HEGET_OK;
}

heget_status check_energy(double v, const char *what)
{
    if (!(std::isfinite(v) && v > 0.0))
        return fail(HEGET_ERR_ARG, std::string(what) + " must be finite and > 0");
    return HEGET_OK;
}

// ---------------------------------------------------------------- plan

double factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

// Phi_n(s) = phase_volume_coef * s^(n-2): massless n-body volume of eq. (4).
double phase_volume_coef(int n)
{
    return std::pow(2.0 * M_PI, 4.0 - 3.0 * n) * std::pow(M_PI / 2.0, n - 1) /
           (factorial(n - 1) * factorial(n - 2));
}

// eq. (2) without |M|^2 as coef * shat^(n-3):
// 1/(2 shat) * 1/2^2 * 1/3^2 * 3 * 1/n! * Phi_n * (hbar c)^2
double partonic_coef(int n)
{
    return 0.5 * 0.25 * (3.0 / 9.0) / factorial(n) * phase_volume_coef(n) * kGeV2fb;
}

// 2 (eQ)^(2n): factor 2 from the parity image of the evaluated quark-helicity block
double me2_coef(int n, double alpha, double charge)
{
    const double e2q2 = 4.0 * M_PI * alpha * charge * charge;
    return 2.0 * std::pow(e2q2, n);
}

// Helicity chunks so that enough wave-sized work items exist for small batches.
int plan_chunks(const heget::Me2Variant &v, int64_t points_expected)
{
    const int passes = (1 << v.n) / v.h;
    const int64_t tiles = (points_expected + 63) / 64;
    const int64_t target = 8192;
    int c = 1;
    while (c < passes && tiles * c < target) c *= 2;
    return c;
}

const heget::Me2Variant *pick_variant(int prec, int n)
{
    return heget::me2_default(prec, n);
}

// ---------------------------------------------------------------- timing hooks

heget_status launch_me2_timed(const heget::Me2Variant &v, const heget::Me2Args &a, hipStream_t s)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g.timing) {
        while (g.ev.size() < g.ev_used + 2) {
            hipEvent_t e;
            HG_HIP(hipEventCreate(&e));
            g.ev.push_back(e);
        }
        e0 = g.ev[g.ev_used];
        e1 = g.ev[g.ev_used + 1];
        g.ev_used += 2;
        HG_HIP(hipEventRecord(e0, s));
    }
    HG_HIP(heget::launch_me2(v, a, s));
    if (g.timing) HG_HIP(hipEventRecord(e1, s));
    return HEGET_OK;
}

heget_status collect_timing()
{
    for (size_t i = 0; i + 1 < g.ev_used; i += 2) {
        HG_HIP(hipEventSynchronize(g.ev[i + 1]));
        float ms = 0.f;
        HG_HIP(hipEventElapsedTime(&ms, g.ev[i], g.ev[i + 1]));
        g.ms_total += ms;
        g.launches += 1;
    }
    g.ev_used = 0;
    return HEGET_OK;
}

// ---------------------------------------------------------------- call bodies

// |M|^2 of npoints SoA points on the device -> d_out, on stream s.
heget_status me2_on_device(int n, int64_t np, const double *d_mom, double *d_out, int prec,
                           hipStream_t s, unsigned *d_flags)
{
    const heget::Me2Variant *v = pick_variant(prec, n);
    if (!v) return fail(HEGET_ERR_ARG, "no compiled amplitude kernel for this n/precision");
    const int nchunks = plan_chunks(*v, np);
    double *part = d_out;
    if (nchunks > 1) HG_TRY(scratch_t<double>(S_PART, size_t(nchunks) * size_t(np), &part));
    heget::Me2Args a{d_mom, np, nullptr, nullptr, np, nchunks, me2_coef(n, g_alpha, g_charge),
                     part, np, d_flags};
    HG_TRY(launch_me2_timed(*v, a, s));
    if (nchunks > 1)
        HG_HIP(heget::launch_sum_chunks(part, nchunks, np, nullptr, np, d_out, d_flags, s));
    return HEGET_OK;
}

heget_status check_config(int n, const heget_config *cfg)
{
    HG_TRY(check_n(n));
    if (!cfg) return fail(HEGET_ERR_ARG, "cfg is NULL");
    HG_TRY(check_np(cfg->npoints));
    HG_TRY(check_prec(cfg->prec));
    HG_TRY(check_cuts(&cfg->cuts));
    if (!(std::isfinite(cfg->alpha) && cfg->alpha > 0.0 && std::isfinite(cfg->charge)))
        return fail(HEGET_ERR_ARG, "alpha must be > 0 and charge finite");
    switch (cfg->mode) {
    case HEGET_FIXED_SHAT: HG_TRY(check_energy(cfg->sqrt_s, "sqrt_s")); break;
    case HEGET_UNIFORM_SQRTSHAT:
        HG_TRY(check_energy(cfg->sqrt_shat_lo, "sqrt_shat_lo"));
        HG_TRY(check_energy(cfg->sqrt_shat_hi, "sqrt_shat_hi"));
        if (!(cfg->sqrt_shat_lo < cfg->sqrt_shat_hi))
            return fail(HEGET_ERR_ARG, "need sqrt_shat_lo < sqrt_shat_hi");
        break;
    case HEGET_PP_TOY:
        HG_TRY(check_energy(cfg->sqrt_s, "sqrt_s"));
        HG_TRY(check_energy(cfg->sqrt_shat_lo, "sqrt_shat_lo"));
        if (!(cfg->sqrt_shat_lo < cfg->sqrt_s))
            return fail(HEGET_ERR_ARG, "need sqrt_shat_lo < sqrt_s");
        break;
    default: return fail(HEGET_ERR_ARG, "unknown mode");
    }
    return HEGET_OK;
}

struct XsecTicket {
    heget_result *out;
    double *staged;
    int64_t n_gen;
};

void xsec_finish(void *p)
{
    XsecTicket *t = static_cast<XsecTicket *>(p);
    const double sum = t->staged[0], comp = t->staged[1], sum2 = t->staged[2];
    const int64_t N = t->n_gen;
    heget_result r{};
    r.sum_w = sum;
    r.sum_w_comp = comp;
    r.sum_w2 = sum2;
    r.n_gen = N;
    r.n_acc = static_cast<int64_t>(t->staged[3]);
    r.sigma_fb = N > 0 ? sum / double(N) : 0.0;
    const double var = N > 1 ? (sum2 / double(N) - r.sigma_fb * r.sigma_fb) / double(N - 1) : 0.0;
    r.err_fb = std::sqrt(var > 0.0 ? var : 0.0);
    *t->out = r;
    delete t;
}

heget_status xsec_enqueue(int n, const heget_config *cfg, heget_result *out, hipStream_t s,
                          unsigned **flags_out)
{
    const int64_t np = cfg->npoints;
    const int nb = static_cast<int>((np + 255) / 256);
    const heget::Me2Variant *v = pick_variant(cfg->prec, n);
    if (!v) return fail(HEGET_ERR_ARG, "no compiled amplitude kernel for this n/precision");
    const int nchunks = plan_chunks(*v, np / 2);

    double *mom, *wfac, *part, *me2, *partials, *res;
    uint8_t *flag;
    int32_t *bcount, *offs, *index;
    int64_t *d_count;
    unsigned *flags;
    HG_TRY(scratch_t<double>(S_MOM, size_t(n + 2) * 4 * size_t(np), &mom));
    HG_TRY(scratch_t<double>(S_WFAC, size_t(np), &wfac));
    HG_TRY(scratch_t<uint8_t>(S_FLAG, size_t(np), &flag));
    HG_TRY(scratch_t<int32_t>(S_BCOUNT, size_t(nb), &bcount));
    HG_TRY(scratch_t<int32_t>(S_OFFS, size_t(nb), &offs));
    HG_TRY(scratch_t<int64_t>(S_COUNT, 1, &d_count));
    HG_TRY(scratch_t<int32_t>(S_INDEX, size_t(np), &index));
    HG_TRY(scratch_t<double>(S_PART, size_t(nchunks) * size_t(np), &part));
    me2 = part;
    if (nchunks > 1) HG_TRY(scratch_t<double>(S_ME2, size_t(np), &me2));
    HG_TRY(scratch_t<double>(S_PARTIALS, size_t(3) * nb, &partials));
    HG_TRY(scratch_t<double>(S_RES, 8, &res));
    HG_TRY(scratch_t<unsigned>(S_FLAGS, 1, &flags));

    heget::GenParams gp{};
    gp.mode = cfg->mode;
    gp.seed = cfg->seed;
    gp.first = 0;
    gp.npoints = np;
    gp.sqrt_s = cfg->sqrt_s;
    gp.lo = cfg->sqrt_shat_lo;
    gp.hi = cfg->sqrt_shat_hi;
    gp.pt_min = cfg->cuts.pt_min;
    gp.eta_max = cfg->cuts.eta_max;
    gp.dr_min = cfg->cuts.dr_min;
    gp.partonic_coef = partonic_coef(n);
    gp.phase_volume_coef = phase_volume_coef(n);
    gp.weight_kind = 1;

    HG_TRY(scratch_acquire(s));
    HG_HIP(heget::launch_zero_u32(flags, 1, s));
    HG_HIP(heget::launch_gen(n, gp, mom, np, wfac, flag, bcount, s));
    HG_HIP(heget::launch_scan(bcount, nb, offs, d_count, s));
    HG_HIP(heget::launch_compact(flag, np, offs, index, s));
    heget::Me2Args a{mom, np, index, d_count, np, nchunks, me2_coef(n, cfg->alpha, cfg->charge),
                     part, np, flags};
    HG_TRY(launch_me2_timed(*v, a, s));
    if (nchunks > 1)
        HG_HIP(heget::launch_sum_chunks(part, nchunks, np, d_count, np, me2, flags, s));
    HG_HIP(heget::launch_weights(me2, index, wfac, d_count, np, partials, flags, s));
    HG_HIP(heget::launch_final(partials, nb, d_count, res, s));
    const unsigned slot = g.ring.fetch_add(1) % kRing;
    double *staged = g.pinned + 8 * slot;
    HG_HIP(hipMemcpyAsync(staged, res, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_TRY(scratch_release(s));
    XsecTicket *t = new XsecTicket{out, staged, np};
    HG_HIP(hipLaunchHostFunc(s, xsec_finish, t));
    if (flags_out) *flags_out = flags;
    return HEGET_OK;
}

}  // namespace

// ==================================================================== C ABI

extern "C" {

heget_status heget_gen_points(int n, double sqrt_s, const heget_cuts *cuts, uint64_t seed,
                              int64_t npoints, double *momenta, double *weight)
{
    g_err.clear();
    HG_TRY(check_n(n));
    HG_TRY(check_np(npoints));
    HG_TRY(check_energy(sqrt_s, "sqrt_s"));
    HG_TRY(check_cuts(cuts));
    if (npoints > 0 && (!momenta || !weight)) return fail(HEGET_ERR_ARG, "null output pointer");
    if (npoints == 0) return HEGET_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    double *d_mom, *d_w;
    const size_t rows = size_t(n + 2) * 4;
    HG_TRY(scratch_t<double>(S_MOM, rows * size_t(npoints), &d_mom));
    HG_TRY(scratch_t<double>(S_WFAC, size_t(npoints), &d_w));
    heget::GenParams gp{};
    gp.mode = HEGET_FIXED_SHAT;
    gp.seed = seed;
    gp.npoints = npoints;
    gp.sqrt_s = sqrt_s;
    gp.pt_min = cuts ? cuts->pt_min : 0.0;
    gp.eta_max = cuts ? cuts->eta_max : 0.0;
    gp.dr_min = cuts ? cuts->dr_min : 0.0;
    gp.phase_volume_coef = phase_volume_coef(n);
    gp.partonic_coef = partonic_coef(n);
    gp.weight_kind = 0;
    hipStream_t s = g.stream;
    HG_TRY(scratch_acquire(s));
    HG_HIP(heget::launch_gen(n, gp, d_mom, npoints, d_w, nullptr, nullptr, s));
    std::vector<double> soa(rows * size_t(npoints));
    HG_HIP(hipMemcpyAsync(soa.data(), d_mom, soa.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_HIP(hipMemcpyAsync(weight, d_w, size_t(npoints) * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_TRY(scratch_release(s));
    HG_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < npoints; ++i)
        for (size_t r = 0; r < rows; ++r) momenta[size_t(i) * rows + r] = soa[r * size_t(npoints) + size_t(i)];
    return HEGET_OK;
}

heget_status heget_gen_points_device(int n, double sqrt_s, const heget_cuts *cuts, uint64_t seed,
                                     int64_t first, int64_t npoints, double *d_mom,
                                     double *d_weight, heget_stream stream)
{
    g_err.clear();
    HG_TRY(check_n(n));
    HG_TRY(check_np(npoints));
    HG_TRY(check_energy(sqrt_s, "sqrt_s"));
    HG_TRY(check_cuts(cuts));
    if (first < 0) return fail(HEGET_ERR_RANGE, "first must be >= 0");
    if (npoints > 0 && (!d_mom || !d_weight)) return fail(HEGET_ERR_ARG, "null output pointer");
    if (npoints == 0) return HEGET_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    heget::GenParams gp{};
    gp.mode = HEGET_FIXED_SHAT;
    gp.seed = seed;
    gp.first = first;
    gp.npoints = npoints;
    gp.sqrt_s = sqrt_s;
    gp.pt_min = cuts ? cuts->pt_min : 0.0;
    gp.eta_max = cuts ? cuts->eta_max : 0.0;
    gp.dr_min = cuts ? cuts->dr_min : 0.0;
    gp.phase_volume_coef = phase_volume_coef(n);
    gp.partonic_coef = partonic_coef(n);
    gp.weight_kind = 0;
    HG_HIP(heget::launch_gen(n, gp, d_mom, npoints, d_weight, nullptr, nullptr,
                             static_cast<hipStream_t>(stream)));
    return HEGET_OK;
}

heget_status heget_me2(int n, int64_t npoints, const double *momenta, double *out_me2,
                       heget_prec prec)
{
    g_err.clear();
    HG_TRY(check_n(n));
    HG_TRY(check_np(npoints));
    HG_TRY(check_prec(prec));
    if (npoints > 0 && (!momenta || !out_me2)) return fail(HEGET_ERR_ARG, "null pointer");
    if (npoints == 0) return HEGET_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    const size_t rows = size_t(n + 2) * 4;
    std::vector<double> soa(rows * size_t(npoints));
    for (int64_t i = 0; i < npoints; ++i)
        for (size_t r = 0; r < rows; ++r) soa[r * size_t(npoints) + size_t(i)] = momenta[size_t(i) * rows + r];
    double *d_mom, *d_out;
    unsigned *d_flags;
    HG_TRY(scratch_t<double>(S_MOM, soa.size(), &d_mom));
    HG_TRY(scratch_t<double>(S_OUT, size_t(npoints), &d_out));
    HG_TRY(scratch_t<unsigned>(S_FLAGS, 1, &d_flags));
    hipStream_t s = g.stream;
    HG_TRY(scratch_acquire(s));
    HG_HIP(hipMemcpyAsync(d_mom, soa.data(), soa.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HG_HIP(heget::launch_zero_u32(d_flags, 1, s));
    HG_TRY(me2_on_device(n, npoints, d_mom, d_out, prec, s, d_flags));
    unsigned flags = 0;
    HG_HIP(hipMemcpyAsync(out_me2, d_out, size_t(npoints) * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_HIP(hipMemcpyAsync(&flags, d_flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HG_TRY(scratch_release(s));
    HG_HIP(hipStreamSynchronize(s));
    if (flags & 1u) {
        g_err = "some points gave a non-finite |M|^2 (check the preconditions)";
        return HEGET_WARN_NONFINITE;
    }
    return HEGET_OK;
}

heget_status heget_me2_device(int n, int64_t npoints, const double *d_mom, double *d_out,
                              heget_prec prec, heget_stream stream)
{
    g_err.clear();
    HG_TRY(check_n(n));
    HG_TRY(check_np(npoints));
    HG_TRY(check_prec(prec));
    if (npoints > 0 && (!d_mom || !d_out)) return fail(HEGET_ERR_ARG, "null pointer");
    if (npoints == 0) return HEGET_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned *d_flags;
    HG_TRY(scratch_t<unsigned>(S_FLAGS, 1, &d_flags));
    HG_TRY(scratch_acquire(s));
    HG_TRY(me2_on_device(n, npoints, d_mom, d_out, prec, s, d_flags));
    HG_TRY(scratch_release(s));
    return HEGET_OK;
}

heget_status heget_xsec_async(int n, const heget_config *cfg, heget_result *out,
                              heget_stream stream)
{
    g_err.clear();
    HG_TRY(check_config(n, cfg));
    if (!out) return fail(HEGET_ERR_ARG, "out is NULL");
    if (cfg->npoints == 0) {
        *out = heget_result{};
        return HEGET_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    return xsec_enqueue(n, cfg, out, static_cast<hipStream_t>(stream), nullptr);
}

heget_status heget_xsec(int n, const heget_config *cfg, heget_result *out)
{
    g_err.clear();
    HG_TRY(check_config(n, cfg));
    if (!out) return fail(HEGET_ERR_ARG, "out is NULL");
    if (cfg->npoints == 0) {
        *out = heget_result{};
        return HEGET_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    unsigned *d_flags = nullptr;
    HG_TRY(xsec_enqueue(n, cfg, out, g.stream, &d_flags));
    unsigned flags = 0;
    HG_HIP(hipMemcpyAsync(&flags, d_flags, sizeof(unsigned), hipMemcpyDeviceToHost, g.stream));
    HG_HIP(hipStreamSynchronize(g.stream));
    if (flags & 1u) {
        g_err = "some weights were not finite";
        return HEGET_WARN_NONFINITE;
    }
    return HEGET_OK;
}

heget_status heget_set_couplings(double alpha, double charge)
{
    g_err.clear();
    if (!(std::isfinite(alpha) && alpha > 0.0 && std::isfinite(charge)))
        return fail(HEGET_ERR_ARG, "alpha must be > 0 and charge finite");
    std::lock_guard<std::mutex> lk(g_mu);
    g_alpha = alpha;
    g_charge = charge;
    return HEGET_OK;
}

heget_status heget_timing_enable(int on)
{
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_mu);
    g.timing = on != 0;
    return HEGET_OK;
}

heget_status heget_timing_read(double *me2_ms, int64_t *me2_launches, int reset)
{
    g_err.clear();
    if (!me2_ms || !me2_launches) return fail(HEGET_ERR_ARG, "null pointer");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g.ready) HG_TRY(collect_timing());
    *me2_ms = g.ms_total;
    *me2_launches = g.launches;
    if (reset) {
        g.ms_total = 0.0;
        g.launches = 0;
    }
    return HEGET_OK;
}

heget_status heget_me2_flops(int n, heget_prec prec, double *flops_per_point, int *unrolled,
                             int *helicities_per_walk)
{
    g_err.clear();
    HG_TRY(check_n(n));
    HG_TRY(check_prec(prec));
    if (!flops_per_point) return fail(HEGET_ERR_ARG, "null pointer");
    const heget::Me2Variant *v = pick_variant(prec, n);
    if (!v) return fail(HEGET_ERR_ARG, "no compiled amplitude kernel for this n/precision");
    const double H = v->h;
    const double passes = double(1 << n) / H;
    const double nfact = factorial(n);
    double nodes = 0.0;  // sum_{j=1}^{n-1} n!/(n-j)!
    for (int j = 1; j <= n - 1; ++j) nodes += nfact / factorial(n - j);
    double builds = n;   // vertex blocks built per walk
    if (n > v->mb) {
        double top = 0.0;
        for (int j = 1; j <= n - v->mb; ++j) top += nfact / factorial(n - j);
        builds = top + nfact / factorial(v->mb) * v->mb;
    }
    // node: q update 4, q^2 5, 1/q^2 1, scale 4 (=14) + per helicity 8 complex
    // multiply-adds (=40); closing: 10 + 2 FP64 adds per helicity; vertex
    // build 3 + 4 per helicity; |amp|^2 in FP64 4 per helicity
    const double per_walk = nodes * (14.0 + 40.0 * H) + nfact * 12.0 * H + builds * (3.0 + 4.0 * H) +
                            4.0 * H;
    *flops_per_point = passes * per_walk;
    if (unrolled) *unrolled = v->mb;
    if (helicities_per_walk) *helicities_per_walk = v->h;
    return HEGET_OK;
}

const char *heget_last_error(void) { return g_err.c_str(); }

void heget_shutdown(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g.ready) return;
    (void)hipDeviceSynchronize();
    for (void *p : g.buf)
        if (p) (void)hipFree(p);
    g.buf.clear();
    g.cap.clear();
    for (hipEvent_t e : g.ev) (void)hipEventDestroy(e);
    g.ev.clear();
    g.ev_used = 0;
    if (g.pinned) (void)hipHostFree(g.pinned);
    g.pinned = nullptr;
    if (g.ws_free) (void)hipEventDestroy(g.ws_free);
    g.ws_free = nullptr;
    if (g.stream) (void)hipStreamDestroy(g.stream);
    g.stream = nullptr;
    g.ready = false;
}

}  // extern "C"
