// Compiled amplitude-kernel shapes, float, n = 5, 6:
// variant<R, n, unrolled depth, helicities per walk, closing depth, waves per block,
// prefetch, waves per SIMD, points per lane, prefix sets> (the last four default to
// 0, 0, 1, 0; the fields of heget_shape).
// The first entry for each n is the default before tuning.
#include "me2_item.hpp"

namespace heget {

extern const Me2Variant kShapesF32Mid[] = {
    variant<float, 5, 5, 8, 2, 1, 0, 0, 1, 2>(), variant<float, 5, 5, 4, 2, 1, 0, 0, 1, 2>(), variant<float, 5, 5, 2, 2, 1, 0, 0, 1, 2>(), variant<float, 5, 5, 4, 5, 1, 0>(), variant<float, 5, 5, 4, 3, 1, 0>(), variant<float, 5, 5, 2, 3, 1, 0>(), variant<float, 5, 5, 2, 3, 1, 1>(), variant<float, 5, 4, 4, 3, 1, 0, 2>(), variant<float, 5, 5, 4, 2, 1>(), variant<float, 5, 4, 2, 2, 4>(), variant<float, 5, 5, 2, 2, 4>(), variant<float, 5, 5, 2, 2, 1>(), variant<float, 5, 5, 1, 2, 4>(), variant<float, 5, 4, 2, 1, 4>(), variant<float, 5, 3, 2, 2, 4>(), variant<float, 5, 4, 1, 2, 4>(), variant<float, 5, 4, 2, 2, 1>(), variant<float, 5, 4, 1, 2, 1>(), variant<float, 5, 5, 4, 2, 1, 1>(), variant<float, 5, 4, 2, 3, 1, 1>(),
    variant<float, 6, 6, 8, 2, 1, 0, 0, 1, 3>(), variant<float, 6, 6, 4, 2, 1, 0, 0, 1, 2>(), variant<float, 6, 6, 2, 2, 1, 0, 0, 1, 2>(), variant<float, 6, 6, 1, 2, 1, 0, 0, 1, 2>(), variant<float, 6, 4, 2, 3, 1, 0, 0, 1, 1>(), variant<float, 6, 4, 2, 5, 1, 0, 0, 1, 1>(), variant<float, 6, 4, 2, 3, 4, 0, 0, 1, 1>(), variant<float, 6, 4, 2, 3, 4>(), variant<float, 6, 4, 1, 3, 4, 0, 0, 1, 1>(), variant<float, 6, 4, 1, 3, 1, 0, 0, 1, 1>(), variant<float, 6, 4, 1, 3, 4>(), variant<float, 6, 4, 1, 3, 1>(), variant<float, 6, 4, 2, 2, 1>(), variant<float, 6, 4, 2, 2, 4>(), variant<float, 6, 4, 2, 1, 4>(), variant<float, 6, 3, 2, 2, 4>(), variant<float, 6, 4, 1, 2, 4>(), variant<float, 6, 4, 1, 2, 1>(), variant<float, 6, 4, 1, 2, 1, 1>(), variant<float, 6, 4, 1, 3, 1, 1>(), variant<float, 6, 4, 2, 3, 1>(),
};
extern const int kShapesF32MidCount = sizeof(kShapesF32Mid) / sizeof(Me2Variant);

}  // namespace heget
