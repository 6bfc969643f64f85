// Helicity-sampling kernels (helicities per walk 0: one configuration per
// lane, drawn per point), float and double, n = 2..8:
// variant<R, n, unrolled depth, 0, closing depth, waves per block, ...,
// prefix sets (n >= 6)>.
#include "me2_item.hpp"

namespace heget {

extern const Me2Variant kShapesSampled[] = {
    variant<float, 2, 2, 0, 2, 4>(), variant<float, 3, 3, 0, 2, 4>(), variant<float, 4, 4, 0, 3, 4>(),
    variant<float, 5, 4, 0, 3, 4>(), variant<float, 6, 4, 0, 3, 4, 0, 0, 1, 1>(),
    variant<float, 7, 4, 0, 3, 4, 0, 0, 1, 1>(), variant<float, 8, 4, 0, 3, 4, 0, 0, 1, 1>(),
    variant<double, 2, 2, 0, 2, 4>(), variant<double, 3, 3, 0, 2, 4>(), variant<double, 4, 4, 0, 3, 4>(),
    variant<double, 5, 4, 0, 3, 4>(), variant<double, 6, 4, 0, 3, 4, 0, 0, 1, 1>(),
    variant<double, 7, 4, 0, 3, 4, 0, 0, 1, 1>(), variant<double, 8, 4, 0, 3, 4, 0, 0, 1, 1>(),
};
extern const int kShapesSampledCount = sizeof(kShapesSampled) / sizeof(Me2Variant);

}  // namespace heget
