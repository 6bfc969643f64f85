// Compiled amplitude-kernel shapes, double, n = 7, 8:
// variant<R, n, unrolled depth, helicities per walk, closing depth, waves per block,
// prefetch, waves per SIMD, points per lane, prefix sets> (the last four default to
// 0, 0, 1, 0; the fields of heget_shape).
// The first entry for each n is the default before tuning.
#include "me2_item.hpp"

namespace heget {

extern const Me2Variant kShapesF64Hi[] = {
    variant<double, 7, 7, 1, 2, 1, 0, 0, 1, 3>(), variant<double, 7, 4, 2, 3, 1, 1, 0, 1, 1>(), variant<double, 7, 4, 1, 3, 1, 0, 0, 1, 1>(), variant<double, 7, 4, 1, 3, 1, 1>(), variant<double, 7, 4, 1, 3, 1, 1, 0, 1, 1>(), variant<double, 7, 4, 1, 2, 4>(), variant<double, 7, 4, 1, 1, 4>(), variant<double, 7, 3, 1, 2, 4>(), variant<double, 7, 3, 2, 2, 4>(), variant<double, 7, 4, 1, 2, 1>(), variant<double, 7, 4, 1, 2, 1, 1>(),
    variant<double, 8, 4, 2, 3, 1, 1, 0, 1, 1>(), variant<double, 8, 4, 1, 3, 1, 0, 0, 1, 1>(), variant<double, 8, 4, 1, 3, 1, 1>(), variant<double, 8, 4, 1, 3, 1, 1, 0, 1, 1>(), variant<double, 8, 4, 1, 2, 4>(), variant<double, 8, 4, 1, 1, 4>(), variant<double, 8, 3, 1, 2, 4>(), variant<double, 8, 3, 2, 2, 4>(), variant<double, 8, 4, 1, 2, 1>(), variant<double, 8, 4, 1, 2, 1, 1>(),
};
extern const int kShapesF64HiCount = sizeof(kShapesF64Hi) / sizeof(Me2Variant);

}  // namespace heget
