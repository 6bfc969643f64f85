// Compiled amplitude-kernel shape, float, n = 8, meeting in the middle with
// the momentum part formed per walk (prefix sets field 3); in a translation
// unit of its own because its single unrolled walk takes minutes to compile.
// The default before tuning.
#include "me2_item.hpp"

namespace heget {

extern const Me2Variant kShapesF32Meet8[] = {
    variant<float, 8, 8, 2, 2, 1, 0, 0, 1, 3>(),
};
extern const int kShapesF32Meet8Count = sizeof(kShapesF32Meet8) / sizeof(Me2Variant);

}  // namespace heget
