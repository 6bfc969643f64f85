// Registry of the compiled amplitude-kernel shapes and their launcher.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <vector>

#include "kernels.hpp"

namespace heget {

// Tables defined in the me2_shapes_*.hip translation units.
extern const Me2Variant kShapesF32Lo[], kShapesF32Mid[], kShapesF32Meet7[], kShapesF32Meet8[],
    kShapesF32Hi[];
extern const Me2Variant kShapesF64Lo[], kShapesF64Mid[], kShapesF64Hi[];
extern const int kShapesF32LoCount, kShapesF32MidCount, kShapesF32Meet7Count, kShapesF32Meet8Count,
    kShapesF32HiCount;
extern const int kShapesF64LoCount, kShapesF64MidCount, kShapesF64HiCount;
extern const Me2Variant kShapesSampled[], kShapesSampledMeet8[];
extern const int kShapesSampledCount, kShapesSampledMeet8Count;

static const std::vector<Me2Variant> &all_variants()
{
    static const std::vector<Me2Variant> v = [] {
        std::vector<Me2Variant> r;
        // the meeting-in-the-middle tables come before the other n = 7, 8
        // shapes: their first entries are the defaults
        const Me2Variant *tabs[] = {kShapesF32Lo, kShapesF32Mid, kShapesF32Meet7, kShapesF32Meet8,
                                    kShapesF32Hi, kShapesF64Lo, kShapesF64Mid, kShapesF64Hi};
        const int counts[] = {kShapesF32LoCount, kShapesF32MidCount, kShapesF32Meet7Count,
                              kShapesF32Meet8Count, kShapesF32HiCount, kShapesF64LoCount,
                              kShapesF64MidCount, kShapesF64HiCount};
        for (int t = 0; t < 8; ++t)
            for (int i = 0; i < counts[t]; ++i) r.push_back(tabs[t][i]);
        return r;
    }();
    return v;
}

const Me2Variant *me2_variants(int *count)
{
    *count = static_cast<int>(all_variants().size());
    return all_variants().data();
}

const Me2Variant *me2_default(int prec, int n)
{
    for (const Me2Variant &v : all_variants())
        if (v.prec == prec && v.n == n) return &v;
    return nullptr;
}

const Me2Variant *me2_sampled(int prec, int n)
{
    for (int i = 0; i < kShapesSampledCount; ++i)
        if (kShapesSampled[i].prec == prec && kShapesSampled[i].n == n) return &kShapesSampled[i];
    for (int i = 0; i < kShapesSampledMeet8Count; ++i)
        if (kShapesSampledMeet8[i].prec == prec && kShapesSampledMeet8[i].n == n) return &kShapesSampledMeet8[i];
    return nullptr;
}

// Blocks of a kernel that fit on the device at once (resident), per kernel.
static int64_t resident_blocks(const Me2Variant &v)
{
    static std::mutex mu;
    static std::map<const void *, int64_t> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(v.func);
    if (it != cache.end()) return it->second;
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, v.func, v.wpb * 64, 0) != hipSuccess ||
        per_cu <= 0 || cus <= 0)
        return 0;  // unknown: one wave per item
    const int64_t r = static_cast<int64_t>(per_cu) * cus;
    cache[v.func] = r;
    return r;
}

hipError_t launch_me2(const Me2Variant &v, const Me2Args &a, hipStream_t stream)
{
    const int64_t ntiles = (a.count + 63) / 64;
    const int64_t items = (ntiles + v.ppl - 1) / v.ppl * a.nchunks;
    if (items == 0) return hipSuccess;
    int64_t blocks = (items + v.wpb - 1) / v.wpb;
    if (v.pf) {
        const int64_t r = resident_blocks(v);
        if (r > 0 && r < blocks) blocks = r;
    }
    void *args[] = {const_cast<double **>(&a.mom), const_cast<int64_t *>(&a.ld),
                    const_cast<int32_t **>(&a.index), const_cast<uint16_t **>(&a.hel),
                    const_cast<int64_t **>(&a.d_count), const_cast<int64_t *>(&a.count),
                    const_cast<int *>(&a.nchunks), const_cast<double *>(&a.coef),
                    const_cast<double **>(&a.out), const_cast<int64_t *>(&a.ld_out),
                    const_cast<double **>(&a.wfac), const_cast<double **>(&a.partials),
                    const_cast<double **>(&a.wout), const_cast<unsigned **>(&a.flags)};
    return hipLaunchKernel(v.func, dim3(static_cast<unsigned>(blocks)), dim3(v.wpb * 64), args, 0,
                           stream);
}

}  // namespace heget
