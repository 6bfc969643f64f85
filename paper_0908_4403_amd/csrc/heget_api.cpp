// C ABI of libheget (include/heget.h): argument checks, the launch plan, the
// library-owned device scratch and the call sequences.  Host code only; all
// arithmetic of the path runs in the kernels of me2_kernels.hip and
// mc_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <exception>
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

// Host staging of `count` doubles; an allocation failure becomes
// HEGET_ERR_ALLOC instead of an exception crossing the C ABI.
heget_status host_buffer(std::vector<double> &v, size_t count)
{
    try {
        v.resize(count);
    } catch (const std::exception &) {
        return fail(HEGET_ERR_ALLOC, "host staging buffer: out of memory");
    }
    return HEGET_OK;
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

// Scratch memory of one stream.  Work on one stream is ordered, so calls on
// the same stream reuse their buffers with no synchronisation; each stream
// has its own set, so calls on different streams never share scratch.
constexpr int kContexts = 4;
struct Scratch {
    hipStream_t stream = nullptr;
    bool bound = false;
    uint64_t last_use = 0;
    std::vector<void *> buf;  // one per Slot
    std::vector<size_t> cap;
};

struct State {
    bool ready = false;
    int device = -1;
    hipStream_t stream = nullptr;     // library stream for the synchronous calls
    Scratch ctx[kContexts];           // ctx[0] belongs to `stream`
    Scratch *cur = nullptr;           // context of the call in progress
    uint64_t tick = 0;
    double *pinned = nullptr;         // staging ring for results (kRing slots of 8 doubles)
    std::atomic<unsigned> ring{0};
    // side streams and fork/join events of the parallel batch schedule
    hipStream_t side[8] = {};
    hipEvent_t fork = nullptr, join[8] = {};
    int batch_schedule = 0;  // 0 auto, 1 persistent kernel, 2 parallel branches
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
    S_MOM, S_WFAC, S_FLAG, S_BCOUNT, S_COUNT, S_INDEX, S_PART, S_PARTIALS, S_RES, S_FLAGS,
    S_OUT, S_BATCH, S_HEL, S_WOUT, S_BINS, S_HIST, S_EVW, S_EVY, S_EVH, S_NSLOTS
};

// Captured mixed-n batches, keyed by their configuration; replayed on repeat calls.
struct BatchGraph {
    std::string key;
    hipGraphExec_t exec = nullptr;  // the schedule in use for this key
    hipGraphExec_t other = nullptr; // kept only while "auto" compares the two
    double *staged = nullptr;       // pinned: 4 doubles per slice + flags
    int schedule = 0;               // 1 persistent, 2 branches
};
std::vector<BatchGraph> g_graphs;

void drop_graphs()
{
    for (BatchGraph &b : g_graphs) {
        if (b.exec) (void)hipGraphExecDestroy(b.exec);
        if (b.other) (void)hipGraphExecDestroy(b.other);
        if (b.staged) (void)hipHostFree(b.staged);
    }
    g_graphs.clear();
}

std::string g_arch;
void load_tuning_cache();

heget_status ensure_device()
{
    if (g.ready) return HEGET_OK;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0)
        return fail(HEGET_ERR_DEVICE, std::string("no HIP device available (hipGetDeviceCount: ") +
                                          hipGetErrorString(e) + ", " + std::to_string(ndev) +
                                          " devices)");
    HG_HIP(hipGetDevice(&g.device));
    HG_HIP(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
    HG_HIP(hipHostMalloc(reinterpret_cast<void **>(&g.pinned), sizeof(double) * 8 * kRing,
                         hipHostMallocDefault));
    for (Scratch &c : g.ctx) {
        c.buf.assign(S_NSLOTS, nullptr);
        c.cap.assign(S_NSLOTS, 0);
        c.bound = false;
    }
    g.ctx[0].stream = g.stream;
    g.ctx[0].bound = true;
    hipDeviceProp_t prop;
    HG_HIP(hipGetDeviceProperties(&prop, g.device));
    g_arch = prop.gcnArchName;
    g_arch = g_arch.substr(0, g_arch.find(':'));
    g.ready = true;
    load_tuning_cache();
    return HEGET_OK;
}

// Make the scratch set of stream s current (call before scratch()).  A stream
// seen for the first time takes a free set, else the least recently used set
// of another user stream once the device is idle (context 0 stays with the
// library stream, whose set also holds the captured batch graphs' memory).
heget_status scratch_bind(hipStream_t s)
{
    Scratch *hit = nullptr;
    for (Scratch &c : g.ctx)
        if (c.bound && c.stream == s) hit = &c;
    if (!hit) {
        for (int i = 1; i < kContexts && !hit; ++i)
            if (!g.ctx[i].bound) hit = &g.ctx[i];
        if (!hit) {
            hit = &g.ctx[1];
            for (int i = 2; i < kContexts; ++i)
                if (g.ctx[i].last_use < hit->last_use) hit = &g.ctx[i];
            HG_HIP(hipDeviceSynchronize());  // its buffers may still be in use on the old stream
        }
        hit->stream = s;
        hit->bound = true;
    }
    hit->last_use = ++g.tick;
    g.cur = hit;
    return HEGET_OK;
}

// Slot of the current scratch set with at least `bytes`; grows (after the
// device is idle) when short.
heget_status scratch(int slot, size_t bytes, void **out)
{
    if (!g.cur) return fail(HEGET_ERR_DEVICE, "internal: scratch used before scratch_bind");
    Scratch &c = *g.cur;
    bytes = bytes < 256 ? 256 : bytes;
    if (c.cap[slot] < bytes) {
        HG_HIP(hipDeviceSynchronize());
        if (slot == S_BATCH) drop_graphs();
        if (c.buf[slot]) HG_HIP(hipFree(c.buf[slot]));
        c.buf[slot] = nullptr;
        c.cap[slot] = 0;
        size_t want = bytes + bytes / 4;
        HG_HIP(hipMalloc(&c.buf[slot], want));
        c.cap[slot] = want;
    }
    *out = c.buf[slot];
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

double me2_flops_per_point(int n, int mb, int h, int cl, int ps = 0);

// Helicity chunks per work item: enough wave-sized items for small batches
// (>= 8192), and no item above ~2e8 flops so the tail of a launch stays short.
int plan_chunks_shape(int n, int mb, int h, int cl, int ps, int64_t points_expected)
{
    const int passes = (1 << n) / h;
    const int64_t tiles = (points_expected + 63) / 64;
    const double item_flops = 64.0 * me2_flops_per_point(n, mb, h, cl, ps);
    int c = 1;
    while (c < passes && (tiles * c < 8192 || item_flops / c > 2e8)) c *= 2;
    return c;
}

int plan_chunks(const heget::Me2Variant &v, int64_t points_expected)
{
    return plan_chunks_shape(v.n, v.mb, v.h, v.cl, v.ps, points_expected);
}

// Shape chosen by the autotuner (or loaded from the tuning cache) per (prec, n).
const heget::Me2Variant *g_tuned[2][9] = {};

const heget::Me2Variant *pick_variant(int prec, int n)
{
    if (prec >= 0 && prec < 2 && n >= 2 && n <= 8 && g_tuned[prec][n]) return g_tuned[prec][n];
    return heget::me2_default(prec, n);
}

const heget::Me2Variant *find_variant(int prec, int n, int mb, int h, int cl, int wpb, int pf, int wpe,
                                      int ppl, int ps)
{
    int cnt = 0;
    const heget::Me2Variant *v = heget::me2_variants(&cnt);
    for (int i = 0; i < cnt; ++i)
        if (v[i].prec == prec && v[i].n == n && v[i].mb == mb && v[i].h == h && v[i].cl == cl &&
            v[i].wpb == wpb && v[i].pf == pf && v[i].wpe == wpe && v[i].ppl == ppl && v[i].ps == ps)
            return &v[i];
    return nullptr;
}

heget_shape shape_of(const heget::Me2Variant &v)
{
    return heget_shape{v.mb, v.h, v.cl, v.wpb, v.pf, v.wpe, v.ppl, v.ps};
}

// Tuning cache: one JSON object per line,
// {"arch": "gfx950", "prec": 1, "n": 4, "mb": 4, "h": 2, "cl": 2, "wpb": 4, "pf": 0, "wpe": 2,
//  "ppl": 1, "ps": 0, "ms": 0.48, "points": 1048576}
void load_tuning_cache()
{
    const char *path = std::getenv("HEGET_TUNING_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char arch[64] = {0};
        int prec, n, mb, h, cl, wpb, pf, wpe, ppl, ps;
        if (std::sscanf(line, " {\"arch\": \"%63[^\"]\", \"prec\": %d, \"n\": %d, \"mb\": %d, \"h\": %d, \"cl\": %d, \"wpb\": %d, \"pf\": %d, \"wpe\": %d, \"ppl\": %d, \"ps\": %d",
                        arch, &prec, &n, &mb, &h, &cl, &wpb, &pf, &wpe, &ppl, &ps) == 11 &&
            g_arch == arch && prec >= 0 && prec < 2 && n >= 2 && n <= 8) {
            const heget::Me2Variant *v = find_variant(prec, n, mb, h, cl, wpb, pf, wpe, ppl, ps);
            if (v) g_tuned[prec][n] = v;
        }
    }
    std::fclose(f);
}

void save_tuning_cache(const heget::Me2Variant &v, double ms, int64_t points)
{
    const char *path = std::getenv("HEGET_TUNING_CACHE");
    if (!path) return;
    // keep other entries, replace this (arch, prec, n)
    std::vector<std::string> keep;
    if (FILE *f = std::fopen(path, "r")) {
        char line[512];
        char tag[128];
        std::snprintf(tag, sizeof tag, "{\"arch\": \"%s\", \"prec\": %d, \"n\": %d,", g_arch.c_str(), v.prec, v.n);
        while (std::fgets(line, sizeof line, f))
            if (std::strncmp(line, tag, std::strlen(tag)) != 0 && line[0] == '{') keep.push_back(line);
        std::fclose(f);
    }
    if (FILE *f = std::fopen(path, "w")) {
        for (const std::string &l : keep) std::fputs(l.c_str(), f);
        std::fprintf(f, "{\"arch\": \"%s\", \"prec\": %d, \"n\": %d, \"mb\": %d, \"h\": %d, \"cl\": %d, \"wpb\": %d, \"pf\": %d, \"wpe\": %d, \"ppl\": %d, \"ps\": %d, \"ms\": %.6f, \"points\": %lld}\n",
                     g_arch.c_str(), v.prec, v.n, v.mb, v.h, v.cl, v.wpb, v.pf, v.wpe, v.ppl, v.ps, ms,
                     static_cast<long long>(points));
        std::fclose(f);
    }
}

// Algorithmic flops per point of the schedule with unrolled depth mb, h
// helicities per walk and closing depth cl (FMA = 2; add, multiply,
// reciprocal = 1).  The h helicity configurations of one walk differ only in
// the helicities of photons 0 .. log2(h)-1 (the "variant" photons).  Where
// every index is a compile-time constant (n <= mb: the whole tree is one
// unrolled subtree) a value that does not depend on a variant photon is the
// same for all h configurations and is computed once: a current whose prefix
// holds k variant photons has 2^k distinct values, a vertex block or pair
// vector 2^(number of variant photons it involves).  Where the photons sit in
// run-time slots (n > mb) nothing is shared and every value is counted h
// times.  This is what the code computes when the compiler shares every
// such value, so the count is a lower bound of the work executed.  Vertex
// blocks are normalised to a unit diagonal, so a vertex product is four
// two-term fused multiply-adds on the current.
//   node update: q update 4, q^2 5, 1/q^2 1, scale by d 4 (= 14, once per node)
//                + 36 per distinct current (vertex half 16, propagator half 20)
//   cl = 1 leaf: closing 8 + 2 FP64 adds per helicity
//   cl = 2, node with two photons left: 2-vector product 14 + 2 FP64 adds per
//         helicity; per subtree: per slot r, p1 - k_r 2, q^2 5, 1/q^2 1,
//         scale 4 (= 12) and w_r 11 per distinct value, per ordered pair u_jr 16,
//         per unordered pair U 4, per distinct value
//   cl = 3, 4, node with four photons left: four node updates, then per split
//         the propagator of q + k_x + k_y 14, per distinct value a vertex half
//         16, a second vertex half added to it 20 and a propagator half 20,
//         and a pair closing (16 per helicity)
//   vertex block build: 4 per photon (kappa / k+-, shared by all helicities)
//   |ordering sum|^2 in FP64: 4 per helicity
namespace flops {

struct Walk {
    int n, b, H, cl;
    bool shared;
    double total = 0.0;

    int var_count(unsigned set) const  // distinct values over the walk's helicities
    {
        if (!shared) return H;
        return 1 << __builtin_popcount(set & ((1u << b) - 1u));
    }

    void subtree_pairs(unsigned slots)
    {
        for (int r = 0; r < n; ++r)
            if (slots >> r & 1u) total += 12.0 + 11.0 * var_count(1u << r);
        for (int j = 0; j < n; ++j)
            for (int r = 0; r < n; ++r)
                if (j != r && (slots >> j & 1u) && (slots >> r & 1u))
                    total += 16.0 * var_count((1u << j) | (1u << r));
        for (int j = 0; j < n; ++j)
            for (int r = j + 1; r < n; ++r)
                if ((slots >> j & 1u) && (slots >> r & 1u))
                    total += 4.0 * var_count((1u << j) | (1u << r));
    }

    // walk below a node whose prefix used the photons in `used`
    void below(unsigned used, int mb)
    {
        const unsigned all = (1u << n) - 1u;
        const unsigned left = all & ~used;
        const int nleft = __builtin_popcount(left);
        if (nleft == mb || (used == 0 && n <= mb)) {
            // subtree entry: vertex blocks of its slots, pair vectors
            for (int s = 0; s < n; ++s)
                if (left >> s & 1u) total += 4.0;
            if (cl >= 2) subtree_pairs(left);
        }
        if (cl == 1 && nleft == 1) {
            total += 10.0 * H;
            return;
        }
        if (cl >= 2 && nleft == 2) {
            total += 16.0 * H;
            return;
        }
        if (cl >= 3 && nleft == 4 && nleft <= mb) {
            // pair sums at both ends: four single-photon updates, then per
            // split {x, y} | {a, b}: the propagator of q + k_x + k_y, two vertex
            // halves and their sum, one propagator half and one pair closing
            for (int s = 0; s < n; ++s)
                if (left >> s & 1u) total += 14.0 + 36.0 * var_count(used | (1u << s));
            for (int x = 0; x < n; ++x)
                for (int y = x + 1; y < n; ++y)
                    if ((left >> x & 1u) && (left >> y & 1u))
                        total += 14.0 + 56.0 * var_count(used | (1u << x) | (1u << y)) + 16.0 * H;
            return;
        }
        for (int s = 0; s < n; ++s) {
            if (!(left >> s & 1u)) continue;
            if (nleft > mb) total += 4.0;  // top-level node builds its vertex block
            const unsigned u = used | (1u << s);
            total += 14.0 + 36.0 * var_count(u);
            below(u, mb);
        }
    }
};

}  // namespace flops

double me2_flops_per_point(int n, int mb, int h, int cl, int ps)
{
    flops::Walk w;
    w.n = n;
    w.H = h;
    w.b = 0;
    while ((1 << w.b) < h) ++w.b;
    w.cl = cl;
    w.shared = n <= mb;
    const int k = n - mb;
    if (ps >= 2) {
        // meeting in the middle (whole tree unrolled, so values that do not
        // depend on a variant photon are shared): v-bar-end currents of every
        // set of up to K = (n + 1) / 2 photons, u-end row vectors of every set
        // of up to n - K - 1, and per set A of K photons the row vector W of
        // the other n - K and one contraction.  A node: momentum 4 (its set's
        // sum is a subset's sum plus one photon, which the compiler shares) +
        // q^2 5 + 1/q^2 1 + scale 4; per distinct value one photon 11, else a
        // vertex half 16, L - 1 vertex halves added 20 each and a propagator
        // half 20 (L photons).  W: 16 + 20 (n - K - 1) per distinct value;
        // contraction 14 + 2 FP64 adds per helicity.  With ps = 2 the
        // momentum parts are formed once per point (the compiler takes them
        // out of the loop over walks), otherwise once per walk.
        const int K = (n + 1) / 2, ku = n - K;
        double momenta = 0.0;
        auto node = [&](unsigned set) {
            const int L = __builtin_popcount(set);
            const double per = L == 1 ? 11.0 : 36.0 + 20.0 * (L - 1);
            momenta += 14.0;
            return per * w.var_count(set);
        };
        w.total += 4.0 * n;
        for (unsigned set = 1; set < (1u << n); ++set) {
            const int L = __builtin_popcount(set);
            if (L <= K - 1) w.total += node(set);
            if (L <= ku - 1) w.total += node(set);
            if (L == K) {
                const unsigned rest = ((1u << n) - 1u) & ~set;
                w.total += node(set) + (16.0 + 20.0 * (ku - 1)) * w.var_count(rest) + 16.0 * h;
            }
        }
        w.total += 4.0 * h;
        const double walks = double(1 << n) / double(h);
        return w.total * walks + momenta * (ps == 2 ? 1.0 : walks);
    } else if (ps == 1 && k >= 2) {
        // prefix sets: per k-subset of the photons, its vertex blocks and the
        // subset recursion over its subsets Q (momentum part 14, a vertex half
        // 16, |Q| - 1 vertex halves added 20 each and a propagator half 20,
        // per helicity), then the subtree over the other photons
        for (unsigned set = 0; set < (1u << n); ++set) {
            if (__builtin_popcount(set) != k) continue;
            w.total += 4.0 * k;
            for (unsigned q = 1; q < (1u << k); ++q)
                w.total += 14.0 + (16.0 + 20.0 * (__builtin_popcount(q) - 1) + 20.0) * h;
            w.below(set, mb);
        }
    } else {
        w.below(0u, n <= mb ? n : mb);
    }
    w.total += 4.0 * h;
    return w.total * double(1 << n) / double(h);
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
    heget::Me2Args a{d_mom, np, nullptr, nullptr, nullptr, np, nchunks,
                     me2_coef(n, g_alpha, g_charge), part, np, nullptr, nullptr, nullptr, d_flags};
    HG_TRY(launch_me2_timed(*v, a, s));
    if (nchunks > 1)
        HG_HIP(heget::launch_sum_chunks(part, nchunks, np, nullptr, np, d_out, nullptr, nullptr,
                                        nullptr, nullptr, d_flags, s));
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
    if (cfg->helicity_sampling != 0 && cfg->helicity_sampling != 1)
        return fail(HEGET_ERR_ARG, "helicity_sampling must be 0 or 1");
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

heget_result make_result(const double *st, int64_t n_gen);

void xsec_finish(void *p)
{
    XsecTicket *t = static_cast<XsecTicket *>(p);
    *t->out = make_result(t->staged, t->n_gen);
    delete t;
}

// Device buffers of one Monte-Carlo configuration.
struct McBufs {
    double *mom, *wfac, *part, *partials, *res;
    uint8_t *flag;
    int32_t *bcount, *index;
    uint16_t *hel;  // sampled helicity configurations, or nullptr (helicity sum)
    double *wout;   // per-survivor weights (histograms), or nullptr
    int64_t *d_count;
    int nchunks;
};

// Status of a finished Monte-Carlo call from its device flags.
heget_status mc_flags_status(unsigned flags)
{
    if (flags & 1u) {
        g_err = "some weights were not finite";
        return HEGET_WARN_NONFINITE;
    }
    return HEGET_OK;
}

heget::GenParams slice_gen_params(int n, const heget_config &c)
{
    heget::GenParams gp{};
    gp.mode = c.mode;
    gp.seed = c.seed;
    gp.npoints = c.npoints;
    gp.sqrt_s = c.sqrt_s;
    gp.lo = c.sqrt_shat_lo;
    gp.hi = c.sqrt_shat_hi;
    gp.pt_min = c.cuts.pt_min;
    gp.eta_max = c.cuts.eta_max;
    gp.dr_min = c.cuts.dr_min;
    gp.partonic_coef = partonic_coef(n);
    gp.phase_volume_coef = phase_volume_coef(n);
    gp.weight_kind = 1;
    return gp;
}

// Generation and compaction: every point's momenta and weight factor, the
// survivor list (point order) and the survivor count in *d_count; `clear`
// (optional) is zeroed by the generation launch.
heget_status enqueue_generation(int n, const heget_config &c, const McBufs &b, hipStream_t s,
                                unsigned *clear = nullptr)
{
    const int64_t np = c.npoints;
    heget::GenParams gp = slice_gen_params(n, c);
    gp.clear_word = clear;
    gp.hel_out = b.hel;
    HG_HIP(heget::launch_gen(n, gp, b.mom, np, b.wfac, b.flag, b.bcount, s));
    HG_HIP(heget::launch_compact(b.bcount, b.flag, np, b.index, b.d_count, s));
    return HEGET_OK;
}

// Weighted sums after the amplitude pass: the weighted chunk sums when the
// amplitude pass wrote |M|^2 (split walks, or `weighted_in_me2` false), then
// the fixed-order reduction into b.res (and the result record if given).
heget_status enqueue_reduction(const heget_config &c, const McBufs &b, unsigned *flags, void *record,
                               hipStream_t s, bool weighted_in_me2 = true)
{
    const int64_t np = c.npoints;
    if (b.nchunks > 1 || !weighted_in_me2)
        HG_HIP(heget::launch_sum_chunks(b.part, b.nchunks, np, b.d_count, np, nullptr, b.index,
                                        b.wfac, b.partials, b.wout, flags, s));
    HG_HIP(heget::launch_final(b.partials, b.d_count, np, b.res, record, s));
    return HEGET_OK;
}

// Arguments of the amplitude pass of a Monte-Carlo call.  With helicity
// sampling the per-point value is the estimator 2^(n+1) |M_h|^2 of the drawn
// configuration: 2^n times the kernel's two-block coefficient.
heget::Me2Args mc_me2_args(int n, const heget_config &c, const McBufs &b, unsigned *flags)
{
    const double coef = me2_coef(n, c.alpha, c.charge) * (b.hel ? double(1 << n) : 1.0);
    const bool epi = b.nchunks == 1;
    return heget::Me2Args{b.mom,      c.npoints,  b.index,  b.hel,  b.d_count,
                          c.npoints,  b.nchunks,  coef,     b.part, c.npoints,
                          b.wfac,     epi ? b.partials : nullptr, epi ? b.wout : nullptr, flags};
}

// A weighted histogram to fill beside the cross section (heget_xsec_hist).
struct HistReq {
    int observable, nbins;
    double lo, hi;
    double *host;  // [nbins + 2], written by a copy enqueued on the stream
};

// Per-event records to copy out beside the cross section (heget_xsec_events):
// host arrays of npoints entries (momenta_soa: (n + 2) * 4 rows of npoints).
struct EventReq {
    double *weight, *momenta_soa, *rapidity;
    uint16_t *helicity;
};

// Enqueue the whole path.  The result goes to d_out (device-writable, filled by
// a kernel) when given, else to *out through the pinned ring and a host callback.
heget_status xsec_enqueue(int n, const heget_config *cfg, heget_result *out, heget_result *d_out,
                          hipStream_t s, unsigned **flags_out, const HistReq *hist = nullptr,
                          const EventReq *ev = nullptr)
{
    const int64_t np = cfg->npoints;
    const bool sampled = cfg->helicity_sampling != 0;
    const heget::Me2Variant *v =
        sampled ? heget::me2_sampled(cfg->prec, n) : pick_variant(cfg->prec, n);
    if (!v) return fail(HEGET_ERR_ARG, "no compiled amplitude kernel for this n/precision");

    const int64_t nb = (np + 255) / 256;
    McBufs b{};
    b.nchunks = sampled ? 1 : plan_chunks(*v, np / 2);
    unsigned *flags;
    HG_TRY(scratch_bind(s));
    HG_TRY(scratch_t<double>(S_MOM, size_t(n + 2) * 4 * size_t(np), &b.mom));
    HG_TRY(scratch_t<double>(S_WFAC, size_t(np), &b.wfac));
    HG_TRY(scratch_t<uint8_t>(S_FLAG, size_t(np), &b.flag));
    HG_TRY(scratch_t<int32_t>(S_BCOUNT, size_t(nb), &b.bcount));
    HG_TRY(scratch_t<int64_t>(S_COUNT, 1, &b.d_count));
    HG_TRY(scratch_t<int32_t>(S_INDEX, size_t(np), &b.index));
    b.hel = nullptr;
    if (sampled) HG_TRY(scratch_t<uint16_t>(S_HEL, size_t(np), &b.hel));
    b.wout = nullptr;
    unsigned long long *bins = nullptr;
    double *d_hist = nullptr;
    if (hist || ev) HG_TRY(scratch_t<double>(S_WOUT, size_t(np), &b.wout));
    double *ev_w = nullptr, *ev_y = nullptr;
    uint16_t *ev_h = nullptr;
    if (ev) {
        HG_TRY(scratch_t<double>(S_EVW, size_t(np), &ev_w));
        if (ev->rapidity) HG_TRY(scratch_t<double>(S_EVY, size_t(np), &ev_y));
        if (ev->helicity) HG_TRY(scratch_t<uint16_t>(S_EVH, size_t(np), &ev_h));
    }
    if (hist) {
        HG_TRY(scratch_t<unsigned long long>(S_BINS, size_t(hist->nbins) + 2, &bins));
        HG_TRY(scratch_t<double>(S_HIST, size_t(hist->nbins) + 2, &d_hist));
    }
    b.part = nullptr;
    if (b.nchunks > 1) HG_TRY(scratch_t<double>(S_PART, size_t(b.nchunks) * size_t(np), &b.part));
    // one spare tile slot: two-points-per-lane shapes write a zero sum there
    HG_TRY(scratch_t<double>(S_PARTIALS, size_t(3) * size_t((np + 63) / 64 + 1), &b.partials));
    HG_TRY(scratch_t<double>(S_RES, 8, &b.res));
    HG_TRY(scratch_t<unsigned>(S_FLAGS, 1, &flags));

    HG_TRY(enqueue_generation(n, *cfg, b, s, flags));  // also clears flags
    HG_TRY(launch_me2_timed(*v, mc_me2_args(n, *cfg, b, flags), s));
    HG_TRY(enqueue_reduction(*cfg, b, flags, d_out, s));
    if (hist) {
        HG_HIP(heget::launch_zero_u32(reinterpret_cast<unsigned *>(bins), 2 * (hist->nbins + 2), s));
        HG_HIP(heget::launch_hist(n, b.mom, np, b.index, b.wout, b.d_count, np, b.res,
                                  hist->observable, hist->nbins, hist->lo, hist->hi, bins, s));
        HG_HIP(heget::launch_hist_finish(bins, hist->nbins, b.res, np, d_hist, s));
        HG_HIP(hipMemcpyAsync(hist->host, d_hist, sizeof(double) * size_t(hist->nbins + 2),
                              hipMemcpyDeviceToHost, s));
    }
    if (ev) {
        const heget::GenParams gp = slice_gen_params(n, *cfg);
        HG_HIP(heget::launch_events(n, gp, ev_w, ev_y, ev_h, s));
        HG_HIP(heget::launch_event_scatter(b.index, b.wout, b.d_count, np, ev_w, s));
        HG_HIP(hipMemcpyAsync(ev->weight, ev_w, sizeof(double) * size_t(np), hipMemcpyDeviceToHost, s));
        if (ev_y)
            HG_HIP(hipMemcpyAsync(ev->rapidity, ev_y, sizeof(double) * size_t(np),
                                  hipMemcpyDeviceToHost, s));
        if (ev_h)
            HG_HIP(hipMemcpyAsync(ev->helicity, ev_h, sizeof(uint16_t) * size_t(np),
                                  hipMemcpyDeviceToHost, s));
        if (ev->momenta_soa)
            HG_HIP(hipMemcpyAsync(ev->momenta_soa, b.mom, sizeof(double) * size_t(n + 2) * 4 * size_t(np),
                                  hipMemcpyDeviceToHost, s));
    }
    if (!d_out) {
        const unsigned slot = g.ring.fetch_add(1) % kRing;
        double *staged = g.pinned + 8 * slot;
        HG_HIP(hipMemcpyAsync(staged, b.res, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        XsecTicket *t = new XsecTicket{out, staged, np};
        HG_HIP(hipLaunchHostFunc(s, xsec_finish, t));
    }
    if (flags_out) *flags_out = flags;
    return HEGET_OK;
}


// ---------------------------------------------------------------- mixed-n batch

// Bump allocator over one scratch slot (256-byte aligned pieces).
struct Arena {
    char *base = nullptr;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
};

struct SliceBufs {
    McBufs b;
    int mb, h, cl, ps;
};

void carve_batch(Arena &ar, int ncfg, const int *n, const heget_config *cfgs, int schedule,
                 SliceBufs *sb, unsigned **flags, unsigned long long **queue, int64_t **item_start)
{
    *flags = ar.take<unsigned>(1);
    *queue = ar.take<unsigned long long>(1);
    *item_start = ar.take<int64_t>(heget::kMaxSlices + 1);
    for (int s = 0; s < ncfg; ++s) {
        const int64_t np = cfgs[s].npoints;
        SliceBufs &sl = sb[s];
        if (schedule == 1) {
            heget::me2_batch_shape(cfgs[s].prec, n[s], &sl.mb, &sl.h, &sl.cl, &sl.ps);
        } else {
            const heget::Me2Variant *v = pick_variant(cfgs[s].prec, n[s]);
            sl.mb = v->mb;
            sl.h = v->h;
            sl.cl = v->cl;
            sl.ps = v->ps;
        }
        McBufs &b = sl.b;
        b.nchunks = plan_chunks_shape(n[s], sl.mb, sl.h, sl.cl, sl.ps, np / 2);
        b.mom = ar.take<double>(size_t(n[s] + 2) * 4 * size_t(np));
        b.wfac = ar.take<double>(size_t(np));
        b.flag = ar.take<uint8_t>(size_t(np));
        b.bcount = ar.take<int32_t>(size_t((np + 255) / 256));
        b.index = ar.take<int32_t>(size_t(np));
        b.hel = nullptr;
        b.wout = nullptr;
        b.d_count = ar.take<int64_t>(1);
        // the persistent kernel always writes |M|^2 per chunk
        const bool need_part = b.nchunks > 1 || schedule == 1;
        b.part = need_part ? ar.take<double>(size_t(b.nchunks) * size_t(np)) : nullptr;
        b.partials = ar.take<double>(size_t(3) * size_t((np + 63) / 64 + 1));  // + spare tile slot
        b.res = ar.take<double>(4);
    }
}

// Parallel schedule: one fork/join branch per configuration on the side
// streams, each with the tuned amplitude kernel for its n.
heget_status batch_enqueue_branches(int ncfg, const int *n, const heget_config *cfgs, SliceBufs *sb,
                                    unsigned *flags, double *staged, hipStream_t s)
{
    HG_HIP(heget::launch_zero_u32(flags, 1, s));
    HG_HIP(hipEventRecord(g.fork, s));
    for (int i = 0; i < ncfg; ++i) {
        hipStream_t si = g.side[i];
        const heget_config &c = cfgs[i];
        const McBufs &b = sb[i].b;
        HG_HIP(hipStreamWaitEvent(si, g.fork, 0));
        HG_TRY(enqueue_generation(n[i], c, b, si));
        HG_HIP(heget::launch_me2(*pick_variant(c.prec, n[i]), mc_me2_args(n[i], c, b, flags), si));
        HG_TRY(enqueue_reduction(c, b, flags, nullptr, si));
        HG_HIP(hipMemcpyAsync(staged + 4 * i, b.res, 4 * sizeof(double), hipMemcpyDeviceToHost, si));
        HG_HIP(hipEventRecord(g.join[i], si));
        HG_HIP(hipStreamWaitEvent(s, g.join[i], 0));
    }
    HG_HIP(hipMemcpyAsync(staged + 4 * heget::kMaxSlices, flags, sizeof(unsigned),
                          hipMemcpyDeviceToHost, s));
    return HEGET_OK;
}

heget_status batch_enqueue(int ncfg, const int *n, const heget_config *cfgs, SliceBufs *sb,
                           unsigned *flags, unsigned long long *queue, int64_t *item_start,
                           double *staged, hipStream_t s)
{
    HG_HIP(heget::launch_zero_u32(flags, 1, s));
    HG_HIP(heget::launch_zero_u32(reinterpret_cast<unsigned *>(queue), 2, s));
    for (int i = 0; i < ncfg; ++i) HG_TRY(enqueue_generation(n[i], cfgs[i], sb[i].b, s));
    // work items of the most expensive slices first (longest-processing-time order)
    std::vector<int> order(ncfg);
    for (int i = 0; i < ncfg; ++i) order[i] = i;
    auto cost = [&](int x) {
        return me2_flops_per_point(n[x], sb[x].mb, sb[x].h, sb[x].cl, sb[x].ps) / sb[x].b.nchunks;
    };
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        const double cx = cost(x), cy = cost(y);
        return cx > cy || (cx == cy && x < y);
    });
    heget::BatchDesc bd{};
    bd.nslices = ncfg;
    bd.item_start = item_start;
    bd.queue = queue;
    bd.flags = flags;
    for (int k = 0; k < ncfg; ++k) {
        const int i = order[k];
        const heget::Me2Args ma = mc_me2_args(n[i], cfgs[i], sb[i].b, flags);
        bd.s[k] = heget::SliceDesc{ma.mom, ma.ld, ma.index, ma.d_count, ma.out, ma.ld_out, ma.wfac,
                                   ma.partials, ma.coef, n[i], ma.nchunks};
    }
    HG_HIP(heget::launch_batch_plan(bd, s));
    int cus = 0;
    HG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g.device));
    const int grid = cus * heget::me2_batch_blocks_per_cu(cfgs[0].prec);
    HG_HIP(heget::launch_me2_batch(cfgs[0].prec, bd, grid, s));
    for (int i = 0; i < ncfg; ++i) {
        HG_TRY(enqueue_reduction(cfgs[i], sb[i].b, flags, nullptr, s, false));
        HG_HIP(hipMemcpyAsync(staged + 4 * i, sb[i].b.res, 4 * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    }
    HG_HIP(hipMemcpyAsync(staged + 4 * heget::kMaxSlices, flags, sizeof(unsigned),
                          hipMemcpyDeviceToHost, s));
    return HEGET_OK;
}

std::string batch_key(int ncfg, const int *n, const heget_config *cfgs)
{
    std::string k(reinterpret_cast<const char *>(n), sizeof(int) * size_t(ncfg));
    k.append(reinterpret_cast<const char *>(cfgs), sizeof(heget_config) * size_t(ncfg));
    return k;
}

heget_result make_result(const double *st, int64_t n_gen)
{
    heget_result r{};
    const double sum = st[0], sum2 = st[2];
    r.sum_w = sum;
    r.sum_w_comp = st[1];
    r.sum_w2 = sum2;
    r.n_gen = n_gen;
    r.n_acc = static_cast<int64_t>(st[3]);
    r.sigma_fb = n_gen > 0 ? sum / double(n_gen) : 0.0;
    const double var = n_gen > 1 ? (sum2 / double(n_gen) - r.sigma_fb * r.sigma_fb) / double(n_gen - 1) : 0.0;
    r.err_fb = std::sqrt(var > 0.0 ? var : 0.0);
    return r;
}

// Bytes of the S_BATCH slot that the batch needs under one schedule.
size_t batch_bytes(int schedule, int ncfg, const int *n, const heget_config *cfgs)
{
    SliceBufs sb[heget::kMaxSlices];
    unsigned *flags;
    unsigned long long *queue;
    int64_t *item_start;
    Arena sizing;
    carve_batch(sizing, ncfg, n, cfgs, schedule, sb, &flags, &queue, &item_start);
    return sizing.off;
}

// Capture the batch for one schedule into an executable graph, its buffers
// carved from `base` (the S_BATCH slot, already at least batch_bytes long).
// The graph keeps these addresses: the slot must not move while it lives.
heget_status capture_batch(int schedule, int ncfg, const int *n, const heget_config *cfgs,
                           void *base, double *staged, hipStream_t s, hipGraphExec_t *exec)
{
    SliceBufs sb[heget::kMaxSlices];
    unsigned *flags;
    unsigned long long *queue;
    int64_t *item_start;
    Arena ar;
    ar.base = static_cast<char *>(base);
    carve_batch(ar, ncfg, n, cfgs, schedule, sb, &flags, &queue, &item_start);
    HG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    heget_status st = schedule == 1
                          ? batch_enqueue(ncfg, n, cfgs, sb, flags, queue, item_start, staged, s)
                          : batch_enqueue_branches(ncfg, n, cfgs, sb, flags, staged, s);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st < 0) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    HG_HIP(e);
    e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HG_HIP(e);
    return HEGET_OK;
}

heget_status ensure_side_streams()
{
    if (g.fork) return HEGET_OK;
    HG_HIP(hipEventCreateWithFlags(&g.fork, hipEventDisableTiming));
    for (int i = 0; i < heget::kMaxSlices; ++i) {
        HG_HIP(hipStreamCreateWithFlags(&g.side[i], hipStreamNonBlocking));
        HG_HIP(hipEventCreateWithFlags(&g.join[i], hipEventDisableTiming));
    }
    return HEGET_OK;
}

heget_status time_graph(hipGraphExec_t exec, hipStream_t s, float *ms)
{
    hipEvent_t e0, e1;
    HG_HIP(hipEventCreate(&e0));
    HG_HIP(hipEventCreate(&e1));
    HG_HIP(hipEventRecord(e0, s));
    HG_HIP(hipGraphLaunch(exec, s));
    HG_HIP(hipEventRecord(e1, s));
    HG_HIP(hipEventSynchronize(e1));
    HG_HIP(hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return HEGET_OK;
}

// Buffers of one cross-section pass carved from `ar` (a dry run with a null
// base measures the bytes needed).
void carve_static(int n, const heget_config &c, const heget::Me2Variant &v, Arena &ar, McBufs &b,
                  unsigned **flags)
{
    const int64_t np = c.npoints;
    const bool sampled = c.helicity_sampling != 0;
    b = McBufs{};
    b.nchunks = sampled ? 1 : plan_chunks(v, np / 2);
    *flags = ar.take<unsigned>(1);
    b.d_count = ar.take<int64_t>(1);
    b.res = ar.take<double>(8);
    b.mom = ar.take<double>(size_t(n + 2) * 4 * size_t(np));
    b.wfac = ar.take<double>(size_t(np));
    b.flag = ar.take<uint8_t>(size_t(np));
    b.bcount = ar.take<int32_t>(size_t((np + 255) / 256));
    b.index = ar.take<int32_t>(size_t(np));
    b.hel = sampled ? ar.take<uint16_t>(size_t(np)) : nullptr;
    b.wout = nullptr;
    b.part = b.nchunks > 1 ? ar.take<double>(size_t(b.nchunks) * size_t(np)) : nullptr;
    b.partials = ar.take<double>(size_t(3) * size_t((np + 63) / 64 + 1));  // + spare tile slot
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
    hipStream_t s = g.stream;
    HG_TRY(scratch_bind(s));
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
    HG_HIP(heget::launch_gen(n, gp, d_mom, npoints, d_w, nullptr, nullptr, s));
    std::vector<double> soa;
    HG_TRY(host_buffer(soa, rows * size_t(npoints)));
    HG_HIP(hipMemcpyAsync(soa.data(), d_mom, soa.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_HIP(hipMemcpyAsync(weight, d_w, size_t(npoints) * sizeof(double), hipMemcpyDeviceToHost, s));
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
    std::vector<double> soa;
    HG_TRY(host_buffer(soa, rows * size_t(npoints)));
    for (int64_t i = 0; i < npoints; ++i)
        for (size_t r = 0; r < rows; ++r) soa[r * size_t(npoints) + size_t(i)] = momenta[size_t(i) * rows + r];
    double *d_mom, *d_out;
    unsigned *d_flags;
    hipStream_t s = g.stream;
    HG_TRY(scratch_bind(s));
    HG_TRY(scratch_t<double>(S_MOM, soa.size(), &d_mom));
    HG_TRY(scratch_t<double>(S_OUT, size_t(npoints), &d_out));
    HG_TRY(scratch_t<unsigned>(S_FLAGS, 1, &d_flags));
    HG_HIP(hipMemcpyAsync(d_mom, soa.data(), soa.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HG_HIP(heget::launch_zero_u32(d_flags, 1, s));
    HG_TRY(me2_on_device(n, npoints, d_mom, d_out, prec, s, d_flags));
    unsigned flags = 0;
    HG_HIP(hipMemcpyAsync(out_me2, d_out, size_t(npoints) * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_HIP(hipMemcpyAsync(&flags, d_flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
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
    HG_TRY(scratch_bind(s));
    HG_TRY(scratch_t<unsigned>(S_FLAGS, 1, &d_flags));
    HG_TRY(me2_on_device(n, npoints, d_mom, d_out, prec, s, d_flags));
    return HEGET_OK;
}

heget_status heget_me2_async(int n, int64_t npoints, const double *d_mom, double *d_out,
                             heget_prec prec, heget_stream stream)
{
    return heget_me2_device(n, npoints, d_mom, d_out, prec, stream);
}

heget_status heget_helas_sizes(int func, int *in_doubles, int *out_doubles)
{
    g_err.clear();
    if (func < 0 || func >= heget::kHelasFuncs)
        return fail(HEGET_ERR_ARG, "unknown HELAS function " + std::to_string(func));
    if (!in_doubles || !out_doubles) return fail(HEGET_ERR_ARG, "null pointer");
    *in_doubles = heget::helas_in_size(func);
    *out_doubles = heget::helas_out_size(func);
    return HEGET_OK;
}

heget_status heget_helas_device(int func, int64_t count, const double *d_in, double *d_out,
                                heget_prec prec, heget_stream stream)
{
    g_err.clear();
    if (func < 0 || func >= heget::kHelasFuncs)
        return fail(HEGET_ERR_ARG, "unknown HELAS function " + std::to_string(func));
    HG_TRY(check_np(count));
    HG_TRY(check_prec(prec));
    if (count > 0 && (!d_in || !d_out)) return fail(HEGET_ERR_ARG, "null pointer");
    if (count == 0) return HEGET_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    HG_HIP(heget::launch_helas(func, prec, count, d_in, d_out, static_cast<hipStream_t>(stream)));
    return HEGET_OK;
}

heget_status heget_helas(int func, int64_t count, const double *in, double *out, heget_prec prec)
{
    g_err.clear();
    if (func < 0 || func >= heget::kHelasFuncs)
        return fail(HEGET_ERR_ARG, "unknown HELAS function " + std::to_string(func));
    HG_TRY(check_np(count));
    HG_TRY(check_prec(prec));
    if (count > 0 && (!in || !out)) return fail(HEGET_ERR_ARG, "null pointer");
    if (count == 0) return HEGET_OK;
    const size_t ni = size_t(heget::helas_in_size(func)), no = size_t(heget::helas_out_size(func));
    if (func <= heget::kHelasVxxxx2)
        for (int64_t i = 0; i < count; ++i) {
            const double h = in[size_t(i) * ni + 4], f = in[size_t(i) * ni + 5];
            if (!((h == 1.0 || h == -1.0) && (f == 1.0 || f == -1.0)))
                return fail(HEGET_ERR_ARG, "record " + std::to_string(i) + ": nHEL and nSF/nSV must be +1 or -1");
        }
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    hipStream_t s = g.stream;
    double *d_in, *d_out;
    HG_TRY(scratch_bind(s));
    HG_TRY(scratch_t<double>(S_MOM, ni * size_t(count), &d_in));
    HG_TRY(scratch_t<double>(S_OUT, no * size_t(count), &d_out));
    HG_HIP(hipMemcpyAsync(d_in, in, ni * size_t(count) * sizeof(double), hipMemcpyHostToDevice, s));
    HG_HIP(heget::launch_helas(func, prec, count, d_in, d_out, s));
    HG_HIP(hipMemcpyAsync(out, d_out, no * size_t(count) * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_HIP(hipStreamSynchronize(s));
    return HEGET_OK;
}

heget_status heget_me2_frame_device(int n, int64_t npoints, const double *d_mom, double *d_out,
                                    heget_prec prec, heget_stream stream)
{
    g_err.clear();
    if (n < 2 || n > heget::kFrameMaxN)
        return fail(HEGET_ERR_RANGE, "n must be in 2.." + std::to_string(heget::kFrameMaxN) +
                                         " for the frame evaluator, got " + std::to_string(n));
    HG_TRY(check_np(npoints));
    HG_TRY(check_prec(prec));
    if (npoints > 0 && (!d_mom || !d_out)) return fail(HEGET_ERR_ARG, "null pointer");
    if (npoints == 0) return HEGET_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned *d_flags;
    HG_TRY(scratch_bind(s));
    HG_TRY(scratch_t<unsigned>(S_FLAGS, 1, &d_flags));
    const double coef = 0.5 * me2_coef(n, g_alpha, g_charge);  // (e Q)^(2n): both quark blocks are summed
    HG_HIP(heget::launch_me2_frame(n, prec, npoints, d_mom, npoints, coef, d_out, d_flags, s));
    return HEGET_OK;
}

heget_status heget_me2_frame(int n, int64_t npoints, const double *momenta, double *out_me2,
                             heget_prec prec)
{
    g_err.clear();
    if (n < 2 || n > heget::kFrameMaxN)
        return fail(HEGET_ERR_RANGE, "n must be in 2.." + std::to_string(heget::kFrameMaxN) +
                                         " for the frame evaluator, got " + std::to_string(n));
    HG_TRY(check_np(npoints));
    HG_TRY(check_prec(prec));
    if (npoints > 0 && (!momenta || !out_me2)) return fail(HEGET_ERR_ARG, "null pointer");
    if (npoints == 0) return HEGET_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    const size_t rows = size_t(n + 2) * 4;
    std::vector<double> soa;
    HG_TRY(host_buffer(soa, rows * size_t(npoints)));
    for (int64_t i = 0; i < npoints; ++i)
        for (size_t r = 0; r < rows; ++r) soa[r * size_t(npoints) + size_t(i)] = momenta[size_t(i) * rows + r];
    double *d_mom, *d_out;
    unsigned *d_flags;
    hipStream_t s = g.stream;
    HG_TRY(scratch_bind(s));
    HG_TRY(scratch_t<double>(S_MOM, soa.size(), &d_mom));
    HG_TRY(scratch_t<double>(S_OUT, size_t(npoints), &d_out));
    HG_TRY(scratch_t<unsigned>(S_FLAGS, 1, &d_flags));
    HG_HIP(hipMemcpyAsync(d_mom, soa.data(), soa.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HG_HIP(heget::launch_zero_u32(d_flags, 1, s));
    const double coef = 0.5 * me2_coef(n, g_alpha, g_charge);
    HG_HIP(heget::launch_me2_frame(n, prec, npoints, d_mom, npoints, coef, d_out, d_flags, s));
    unsigned flags = 0;
    HG_HIP(hipMemcpyAsync(out_me2, d_out, size_t(npoints) * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_HIP(hipMemcpyAsync(&flags, d_flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HG_HIP(hipStreamSynchronize(s));
    if (flags & 1u) {
        g_err = "some points gave a non-finite |M|^2 (check the preconditions)";
        return HEGET_WARN_NONFINITE;
    }
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
    return xsec_enqueue(n, cfg, out, nullptr, static_cast<hipStream_t>(stream), nullptr);
}

heget_status heget_xsec_device(int n, const heget_config *cfg, heget_result *d_out,
                               heget_stream stream)
{
    g_err.clear();
    HG_TRY(check_config(n, cfg));
    if (!d_out) return fail(HEGET_ERR_ARG, "d_out is NULL");
    if (cfg->npoints == 0) return fail(HEGET_ERR_RANGE, "heget_xsec_device needs npoints > 0");
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    return xsec_enqueue(n, cfg, nullptr, d_out, static_cast<hipStream_t>(stream), nullptr);
}

heget_status heget_xsec_device_noalloc(int n, const heget_config *cfg, heget_result *d_out,
                                       heget_stream stream)
{
    g_err.clear();
    HG_TRY(check_config(n, cfg));
    if (!d_out) return fail(HEGET_ERR_ARG, "d_out is NULL");
    if (cfg->npoints == 0) return fail(HEGET_ERR_RANGE, "heget_xsec_device_noalloc needs npoints > 0");
    const bool sampled = cfg->helicity_sampling != 0;
    std::lock_guard<std::mutex> lk(g_mu);
    const heget::Me2Variant *v =
        sampled ? heget::me2_sampled(cfg->prec, n) : pick_variant(cfg->prec, n);
    if (!v) return fail(HEGET_ERR_ARG, "no compiled amplitude kernel for this n/precision");
    McBufs b;
    unsigned *flags = nullptr;
    Arena dry;
    carve_static(n, *cfg, *v, dry, b, &flags);
    const size_t cap = heget::static_scratch_bytes();
    if (dry.off > cap)
        return fail(HEGET_ERR_RANGE, "heget_xsec_device_noalloc: n = " + std::to_string(n) + " with " +
                                         std::to_string(cfg->npoints) + " points needs " +
                                         std::to_string(dry.off) + " bytes of workspace, above its " +
                                         std::to_string(cap) + "-byte static workspace");
    void *base = nullptr;
    HG_HIP(heget::static_scratch_ptr(&base));
    Arena ar;
    ar.base = static_cast<char *>(base);
    carve_static(n, *cfg, *v, ar, b, &flags);
    hipStream_t s = static_cast<hipStream_t>(stream);
    HG_TRY(enqueue_generation(n, *cfg, b, s, flags));  // also clears flags
    HG_HIP(heget::launch_me2(*v, mc_me2_args(n, *cfg, b, flags), s));
    HG_TRY(enqueue_reduction(*cfg, b, flags, d_out, s));
    return HEGET_OK;
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
    HG_TRY(xsec_enqueue(n, cfg, out, nullptr, g.stream, &d_flags));
    unsigned flags = 0;
    HG_HIP(hipMemcpyAsync(&flags, d_flags, sizeof(unsigned), hipMemcpyDeviceToHost, g.stream));
    HG_HIP(hipStreamSynchronize(g.stream));
    return mc_flags_status(flags);
}

heget_status heget_xsec_hist(int n, const heget_config *cfg, int observable, int nbins, double lo,
                             double hi, double *hist, heget_result *out)
{
    g_err.clear();
    HG_TRY(check_config(n, cfg));
    if (!out || !hist) return fail(HEGET_ERR_ARG, "out and hist must not be NULL");
    if (observable != HEGET_OBS_PT_MAX && observable != HEGET_OBS_DR_MIN)
        return fail(HEGET_ERR_ARG, "unknown observable");
    if (nbins < 1 || nbins > heget::kHistMaxBins)
        return fail(HEGET_ERR_RANGE, "nbins must be in 1..4096");
    if (!(std::isfinite(lo) && std::isfinite(hi) && lo < hi))
        return fail(HEGET_ERR_ARG, "need finite lo < hi");
    if (cfg->npoints == 0) {
        *out = heget_result{};
        for (int b = 0; b < nbins + 2; ++b) hist[b] = 0.0;
        return HEGET_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    unsigned *d_flags = nullptr;
    const HistReq req{observable, nbins, lo, hi, hist};
    HG_TRY(xsec_enqueue(n, cfg, out, nullptr, g.stream, &d_flags, &req));
    unsigned flags = 0;
    HG_HIP(hipMemcpyAsync(&flags, d_flags, sizeof(unsigned), hipMemcpyDeviceToHost, g.stream));
    HG_HIP(hipStreamSynchronize(g.stream));
    return mc_flags_status(flags);
}

heget_status heget_xsec_events(int n, const heget_config *cfg, heget_result *out, double *weight,
                               double *momenta, double *rapidity, uint16_t *helicity)
{
    g_err.clear();
    HG_TRY(check_config(n, cfg));
    if (!out || !weight) return fail(HEGET_ERR_ARG, "out and weight must not be NULL");
    if (helicity && !cfg->helicity_sampling)
        return fail(HEGET_ERR_ARG, "helicities are drawn only with helicity_sampling = 1");
    const int64_t np = cfg->npoints;
    if (np == 0) {
        *out = heget_result{};
        return HEGET_OK;
    }
    std::vector<double> soa;
    if (momenta) HG_TRY(host_buffer(soa, size_t(n + 2) * 4 * size_t(np)));
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    unsigned *d_flags = nullptr;
    const EventReq req{weight, momenta ? soa.data() : nullptr, rapidity, helicity};
    HG_TRY(xsec_enqueue(n, cfg, out, nullptr, g.stream, &d_flags, nullptr, &req));
    unsigned flags = 0;
    HG_HIP(hipMemcpyAsync(&flags, d_flags, sizeof(unsigned), hipMemcpyDeviceToHost, g.stream));
    HG_HIP(hipStreamSynchronize(g.stream));
    if (momenta) {
        const size_t rows = size_t(n + 2) * 4;
        for (int64_t i = 0; i < np; ++i)
            for (size_t r = 0; r < rows; ++r) momenta[size_t(i) * rows + r] = soa[r * size_t(np) + size_t(i)];
    }
    return mc_flags_status(flags);
}

heget_status heget_set_batch_schedule(int schedule)
{
    g_err.clear();
    if (schedule < 0 || schedule > 2) return fail(HEGET_ERR_ARG, "schedule must be 0, 1 or 2");
    std::lock_guard<std::mutex> lk(g_mu);
    g.batch_schedule = schedule;
    drop_graphs();
    return HEGET_OK;
}

heget_status heget_xsec_batch(const int *n, const heget_config *cfgs, int ncfg,
                                         heget_result *out)
{
    g_err.clear();
    if (!n || !cfgs || !out) return fail(HEGET_ERR_ARG, "null pointer");
    if (ncfg < 1 || ncfg > heget::kMaxSlices)
        return fail(HEGET_ERR_RANGE, "ncfg must be in 1..8");
    for (int i = 0; i < ncfg; ++i) {
        HG_TRY(check_config(n[i], &cfgs[i]));
        if (cfgs[i].helicity_sampling)
            return fail(HEGET_ERR_ARG, "helicity sampling is not available in batches");
        if (cfgs[i].prec != cfgs[0].prec)
            return fail(HEGET_ERR_ARG, "all configurations of a batch need the same prec");
    }
    int64_t total = 0;
    for (int i = 0; i < ncfg; ++i) total += cfgs[i].npoints;
    if (total == 0) {
        for (int i = 0; i < ncfg; ++i) out[i] = heget_result{};
        return HEGET_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    HG_TRY(ensure_side_streams());
    hipStream_t s = g.stream;
    const std::string key = batch_key(ncfg, n, cfgs);
    BatchGraph *bg = nullptr;
    for (BatchGraph &b : g_graphs)
        if (b.key == key) bg = &b;
    HG_TRY(scratch_bind(s));
    if (!bg) {
        if (g_graphs.size() >= 8) drop_graphs();
        BatchGraph nb;
        nb.key = key;
        HG_HIP(hipHostMalloc(reinterpret_cast<void **>(&nb.staged),
                             sizeof(double) * 4 * (heget::kMaxSlices + 1), hipHostMallocDefault));
        // One S_BATCH slot of the size the largest schedule needs, obtained
        // before any capture: growing the slot frees the old memory, which a
        // graph captured earlier in this call would still address.
        size_t need = batch_bytes(g.batch_schedule == 0 ? 1 : g.batch_schedule, ncfg, n, cfgs);
        if (g.batch_schedule == 0) need = std::max(need, batch_bytes(2, ncfg, n, cfgs));
        void *base = nullptr;
        hipGraphExec_t a1 = nullptr, a2 = nullptr;
        heget_status st = scratch(S_BATCH, need, &base);
        if (st >= 0 && g.batch_schedule == 0) {
            // auto: capture both schedules, keep the faster (one timed run each)
            st = capture_batch(1, ncfg, n, cfgs, base, nb.staged, s, &a1);
            if (st >= 0) st = capture_batch(2, ncfg, n, cfgs, base, nb.staged, s, &a2);
            float t1 = 0.f, t2 = 0.f;
            if (st >= 0 && (hipGraphLaunch(a1, s) != hipSuccess || hipGraphLaunch(a2, s) != hipSuccess))
                st = fail(HEGET_ERR_DEVICE, "hipGraphLaunch failed");  // the launches warm both
            if (st >= 0) st = time_graph(a1, s, &t1);
            if (st >= 0) st = time_graph(a2, s, &t2);
            if (st >= 0) {
                nb.schedule = t1 <= t2 ? 1 : 2;
                nb.exec = t1 <= t2 ? a1 : a2;
                (t1 <= t2 ? a1 : a2) = nullptr;
            }
        } else if (st >= 0) {
            nb.schedule = g.batch_schedule;
            st = capture_batch(nb.schedule, ncfg, n, cfgs, base, nb.staged, s, &nb.exec);
        }
        if (st < 0) (void)hipStreamSynchronize(s);  // nothing of a failed call is left in flight
        if (a1) (void)hipGraphExecDestroy(a1);
        if (a2) (void)hipGraphExecDestroy(a2);
        if (st < 0) {
            if (nb.exec) (void)hipGraphExecDestroy(nb.exec);
            (void)hipHostFree(nb.staged);
            return st;
        }
        g_graphs.push_back(nb);
        bg = &g_graphs.back();
    }
    HG_HIP(hipGraphLaunch(bg->exec, s));
    HG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < ncfg; ++i) out[i] = make_result(bg->staged + 4 * i, cfgs[i].npoints);
    unsigned fl = 0;
    std::memcpy(&fl, bg->staged + 4 * heget::kMaxSlices, sizeof(unsigned));
    return mc_flags_status(fl);
}

heget_status heget_batch_schedule_in_use(const int *n, const heget_config *cfgs,
                                                    int ncfg, int *schedule)
{
    g_err.clear();
    if (!n || !cfgs || !schedule || ncfg < 1 || ncfg > heget::kMaxSlices)
        return fail(HEGET_ERR_ARG, "bad arguments");
    std::lock_guard<std::mutex> lk(g_mu);
    const std::string key = batch_key(ncfg, n, cfgs);
    *schedule = 0;
    for (BatchGraph &b : g_graphs)
        if (b.key == key) *schedule = b.schedule;
    return HEGET_OK;
}

heget_status heget_autotune(int n, heget_prec prec, int64_t npoints, heget_shape *chosen,
                            double *ms)
{
    g_err.clear();
    HG_TRY(check_n(n));
    HG_TRY(check_prec(prec));
    if (npoints < 64 || npoints > kMaxPoints)
        return fail(HEGET_ERR_RANGE, "autotune needs 64 <= npoints < 2^31");
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    hipStream_t s = g.stream;
    double *d_mom, *d_w, *d_out;
    unsigned *d_flags;
    HG_TRY(scratch_bind(s));
    HG_TRY(scratch_t<double>(S_MOM, size_t(n + 2) * 4 * size_t(npoints), &d_mom));
    HG_TRY(scratch_t<double>(S_WFAC, size_t(npoints), &d_w));
    HG_TRY(scratch_t<unsigned>(S_FLAGS, 1, &d_flags));
    // synthetic points: sqrt(shat) = 1 TeV, the paper's cuts applied to the
    // weights only (every generated point is a valid input)
    heget::GenParams gp{};
    gp.mode = HEGET_FIXED_SHAT;
    gp.seed = 0x5eed;
    gp.npoints = npoints;
    gp.sqrt_s = 1000.0;
    gp.pt_min = 20.0;
    gp.eta_max = 2.5;
    gp.dr_min = 0.4;
    gp.phase_volume_coef = phase_volume_coef(n);
    gp.weight_kind = 0;
    HG_HIP(heget::launch_gen(n, gp, d_mom, npoints, d_w, nullptr, nullptr, s));
    HG_HIP(heget::launch_zero_u32(d_flags, 1, s));
    hipEvent_t e0, e1;
    HG_HIP(hipEventCreate(&e0));
    HG_HIP(hipEventCreate(&e1));
    int cnt = 0;
    const heget::Me2Variant *all = heget::me2_variants(&cnt);
    const heget::Me2Variant *best = nullptr;
    double best_ms = 0.0;
    for (int i = 0; i < cnt; ++i) {
        const heget::Me2Variant &v = all[i];
        if (v.prec != prec || v.n != n) continue;
        const int nchunks = plan_chunks(v, npoints);
        double *out = nullptr;
        HG_TRY(scratch_t<double>(S_OUT, size_t(nchunks) * size_t(npoints), &out));
        heget::Me2Args a{d_mom, npoints, nullptr, nullptr, nullptr, npoints, nchunks,
                         me2_coef(n, g_alpha, g_charge), out, npoints, nullptr, nullptr, nullptr,
                         d_flags};
        HG_HIP(heget::launch_me2(v, a, s));  // warm-up
        HG_HIP(hipEventRecord(e0, s));
        const int reps = 3;
        for (int r = 0; r < reps; ++r) HG_HIP(heget::launch_me2(v, a, s));
        HG_HIP(hipEventRecord(e1, s));
        HG_HIP(hipEventSynchronize(e1));
        float t = 0.f;
        HG_HIP(hipEventElapsedTime(&t, e0, e1));
        const double per = double(t) / reps;
        // a later shape must be 2% faster to win, so near-ties keep the
        // earlier (default-first) table entry from run to run
        if (!best || per < 0.98 * best_ms) {
            best = &v;
            best_ms = per;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!best) return fail(HEGET_ERR_ARG, "no compiled amplitude kernel for this n/precision");
    g_tuned[prec][n] = best;
    save_tuning_cache(*best, best_ms, npoints);
    if (chosen) *chosen = shape_of(*best);
    if (ms) *ms = best_ms;
    return HEGET_OK;
}

heget_status heget_set_kernel_shape(int n, heget_prec prec, const heget_shape *shape)
{
    g_err.clear();
    HG_TRY(check_n(n));
    HG_TRY(check_prec(prec));
    std::lock_guard<std::mutex> lk(g_mu);
    if (!shape) {
        g_tuned[prec][n] = nullptr;
        return HEGET_OK;
    }
    const heget::Me2Variant *v =
        find_variant(prec, n, shape->unrolled, shape->helicities_per_walk, shape->closing,
                     shape->waves_per_block, shape->prefetch, shape->waves_per_simd,
                     shape->points_per_lane, shape->prefix_sets);
    if (!v) return fail(HEGET_ERR_ARG, "no compiled kernel shape with these parameters");
    g_tuned[prec][n] = v;
    return HEGET_OK;
}

heget_status heget_kernel_shapes(int n, heget_prec prec, int max, heget_shape *shapes, int *count)
{
    g_err.clear();
    HG_TRY(check_n(n));
    HG_TRY(check_prec(prec));
    if (!count || (max > 0 && !shapes)) return fail(HEGET_ERR_ARG, "null pointer");
    int cnt = 0, k = 0;
    const heget::Me2Variant *all = heget::me2_variants(&cnt);
    const heget::Me2Variant *cur = pick_variant(prec, n);
    if (cur) {  // the shape in use first
        if (k < max) shapes[k] = shape_of(*cur);
        ++k;
    }
    for (int i = 0; i < cnt; ++i) {
        if (all[i].prec != prec || all[i].n != n || &all[i] == cur) continue;
        if (k < max) shapes[k] = shape_of(all[i]);
        ++k;
    }
    *count = k;
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

heget_status heget_me2_flops(int n, heget_prec prec, double *flops_per_point, heget_shape *shape)
{
    g_err.clear();
    HG_TRY(check_n(n));
    HG_TRY(check_prec(prec));
    if (!flops_per_point) return fail(HEGET_ERR_ARG, "null pointer");
    const heget::Me2Variant *v = pick_variant(prec, n);
    if (!v) return fail(HEGET_ERR_ARG, "no compiled amplitude kernel for this n/precision");
    *flops_per_point = me2_flops_per_point(n, v->mb, v->h, v->cl, v->ps);
    if (shape) *shape = shape_of(*v);
    return HEGET_OK;
}

heget_status heget_valu_peak(double *fp32_tflops, double *fp64_tflops)
{
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_mu);
    HG_TRY(ensure_device());
    hipStream_t s = g.stream;
    int cus = 0;
    HG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g.device));
    const int blocks = cus * 16;  // 16 waves per CU
    const int iters = 512;
    HG_TRY(scratch_bind(s));
    void *out = nullptr;
    HG_TRY(scratch(S_OUT, size_t(blocks) * 256 * sizeof(double), &out));
    hipEvent_t e0, e1;
    HG_HIP(hipEventCreate(&e0));
    HG_HIP(hipEventCreate(&e1));
    double *res[2] = {fp64_tflops, fp32_tflops};
    for (int prec = 0; prec < 2; ++prec) {
        if (!res[prec]) continue;
        HG_HIP(heget::launch_fma_peak(prec, out, blocks, iters, s));  // warm-up
        float best = 0.f;
        for (int r = 0; r < 3; ++r) {
            HG_HIP(hipEventRecord(e0, s));
            HG_HIP(heget::launch_fma_peak(prec, out, blocks, iters, s));
            HG_HIP(hipEventRecord(e1, s));
            HG_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            HG_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (r == 0 || ms < best) best = ms;
        }
        *res[prec] = heget::fma_peak_flops(blocks, iters) / (double(best) * 1e-3) / 1e12;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return HEGET_OK;
}

const char *heget_last_error(void) { return g_err.c_str(); }

void heget_shutdown(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g.ready) return;
    (void)hipDeviceSynchronize();
    for (Scratch &c : g.ctx) {
        for (void *p : c.buf)
            if (p) (void)hipFree(p);
        c.buf.clear();
        c.cap.clear();
        c.bound = false;
    }
    g.cur = nullptr;
    for (hipEvent_t e : g.ev) (void)hipEventDestroy(e);
    g.ev.clear();
    g.ev_used = 0;
    drop_graphs();
    for (int i = 0; i < 8; ++i) {
        if (g.side[i]) (void)hipStreamDestroy(g.side[i]);
        if (g.join[i]) (void)hipEventDestroy(g.join[i]);
        g.side[i] = nullptr;
        g.join[i] = nullptr;
    }
    if (g.fork) (void)hipEventDestroy(g.fork);
    g.fork = nullptr;
    if (g.pinned) (void)hipHostFree(g.pinned);
    g.pinned = nullptr;
    if (g.stream) (void)hipStreamDestroy(g.stream);
    g.stream = nullptr;
    g.ready = false;
}

}  // extern "C"
