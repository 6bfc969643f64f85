// Compiled amplitude-kernel shapes, double, n = 5, 6:
// variant<R, n, unrolled depth, helicities per walk, closing depth, waves per block,
// prefetch, waves per SIMD, points per lane, prefix sets> (the last four default to
// 0, 0, 1, 0; the fields of heget_shape).
// The first entry for each n is the default before tuning.
#include "me2_item.hpp"

namespace heget {

extern const Me2Variant kShapesF64Mid[] = {
    variant<double, 5, 5, 2, 2, 1, 0, 0, 1, 2>(), variant<double, 5, 5, 1, 2, 1, 0, 0, 1, 2>(), variant<double, 5, 4, 2, 3, 1, 1>(), variant<double, 5, 4, 1, 3, 1, 0>(), variant<double, 5, 4, 1, 3, 1, 1>(), variant<double, 5, 4, 1, 2, 1>(), variant<double, 5, 4, 1, 2, 4>(), variant<double, 5, 5, 1, 2, 4>(), variant<double, 5, 5, 1, 2, 1>(), variant<double, 5, 4, 1, 1, 4>(), variant<double, 5, 3, 1, 2, 4>(), variant<double, 5, 3, 2, 2, 4>(), variant<double, 5, 4, 1, 2, 1, 1>(),
    variant<double, 6, 6, 1, 2, 1, 0, 0, 1, 4>(), variant<double, 6, 6, 1, 2, 1, 0, 0, 1, 3>(), variant<double, 6, 4, 2, 3, 1, 0, 2, 1, 1>(), variant<double, 6, 4, 2, 3, 1, 1, 0, 1, 1>(), variant<double, 6, 4, 1, 3, 1, 0, 0, 1, 1>(), variant<double, 6, 4, 2, 3, 1, 1>(), variant<double, 6, 4, 1, 3, 1, 1, 0, 1, 1>(), variant<double, 6, 4, 1, 3, 1, 1>(), variant<double, 6, 4, 1, 2, 1>(), variant<double, 6, 4, 1, 2, 4>(), variant<double, 6, 4, 1, 1, 4>(), variant<double, 6, 3, 1, 2, 4>(), variant<double, 6, 3, 2, 2, 4>(), variant<double, 6, 4, 1, 2, 1, 1>(),
};
extern const int kShapesF64MidCount = sizeof(kShapesF64Mid) / sizeof(Me2Variant);

}  // namespace heget
