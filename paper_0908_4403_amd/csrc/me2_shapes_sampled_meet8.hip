// Helicity-sampling kernel, float, n = 8, meeting in the middle with the
// momentum part formed per walk (prefix sets field 3); in a translation unit
// of its own because its unrolled walk takes minutes to compile.
#include "me2_item.hpp"

namespace heget {

extern const Me2Variant kShapesSampledMeet8[] = {
    variant<float, 8, 8, 0, 2, 1, 0, 0, 1, 3>(),
};
extern const int kShapesSampledMeet8Count = sizeof(kShapesSampledMeet8) / sizeof(Me2Variant);

}  // namespace heget
