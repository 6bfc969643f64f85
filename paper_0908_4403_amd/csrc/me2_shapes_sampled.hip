// Helicity-sampling kernels (helicities per walk 0: one configuration per
// lane, drawn per point), float and double, n = 2..8:
// variant<R, n, unrolled depth, 0, closing depth, waves per block, prefetch,
// waves per SIMD, points per lane, prefix sets>.  n >= 5 meet in the middle
// (prefix sets 2-4; FP64 n = 8 walks prefix sets); the float n = 8 kernel is in
// me2_shapes_sampled_meet8.hip.
#include "me2_item.hpp"

namespace heget {

extern const Me2Variant kShapesSampled[] = {
    variant<float, 2, 2, 0, 2, 4>(), variant<float, 3, 3, 0, 2, 4>(), variant<float, 4, 4, 0, 3, 4>(),
    variant<float, 5, 5, 0, 2, 1, 0, 0, 1, 2>(), variant<float, 6, 6, 0, 2, 1, 0, 0, 1, 2>(),
    variant<float, 7, 7, 0, 2, 1, 0, 0, 1, 3>(),
    variant<double, 2, 2, 0, 2, 4>(), variant<double, 3, 3, 0, 2, 4>(), variant<double, 4, 4, 0, 3, 4>(),
    variant<double, 5, 5, 0, 2, 1, 0, 0, 1, 2>(), variant<double, 6, 6, 0, 2, 1, 0, 0, 1, 4>(),
    variant<double, 7, 7, 0, 2, 1, 0, 0, 1, 3>(), variant<double, 8, 4, 0, 3, 4, 0, 0, 1, 1>(),
};
extern const int kShapesSampledCount = sizeof(kShapesSampled) / sizeof(Me2Variant);

}  // namespace heget
