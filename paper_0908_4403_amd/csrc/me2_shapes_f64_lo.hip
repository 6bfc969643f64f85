// Compiled amplitude-kernel shapes, double, n = 2, 3, 4:
// variant<R, n, unrolled depth, helicities per walk, closing depth, waves per block,
// prefetch, waves per SIMD, points per lane, prefix sets> (the last four default to
// 0, 0, 1, 0; the fields of heget_shape).
// The first entry for each n is the default before tuning.
#include "me2_item.hpp"

namespace heget {

extern const Me2Variant kShapesF64Lo[] = {
    variant<double, 2, 2, 2, 2, 4>(), variant<double, 2, 2, 2, 2, 4, 0, 0, 2>(), variant<double, 2, 2, 1, 1, 4>(), variant<double, 2, 2, 1, 2, 4>(), variant<double, 2, 2, 2, 2, 1, 1>(),
    variant<double, 3, 3, 4, 2, 1, 1>(), variant<double, 3, 3, 4, 2, 1, 0, 0, 2>(), variant<double, 3, 3, 4, 2, 1>(), variant<double, 3, 3, 2, 2, 4>(), variant<double, 3, 3, 1, 2, 4>(), variant<double, 3, 3, 1, 1, 4>(), variant<double, 3, 3, 2, 2, 1>(),
    variant<double, 4, 4, 4, 3, 1, 1>(), variant<double, 4, 4, 4, 3, 1, 0>(), variant<double, 4, 4, 2, 3, 1, 1>(), variant<double, 4, 4, 1, 2, 1, 1>(), variant<double, 4, 4, 1, 2, 1>(), variant<double, 4, 4, 1, 2, 4>(), variant<double, 4, 4, 1, 1, 4>(), variant<double, 4, 3, 1, 2, 4>(), variant<double, 4, 3, 2, 2, 4>(), variant<double, 4, 4, 1, 3, 1, 1>(),
};
extern const int kShapesF64LoCount = sizeof(kShapesF64Lo) / sizeof(Me2Variant);

}  // namespace heget
