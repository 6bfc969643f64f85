// Compiled amplitude-kernel shapes, float, n = 7, meeting in the middle with
// the momentum part formed per walk (prefix sets field 3); in a translation
// unit of their own because their single unrolled walk takes a minute or more
// to compile.  The first entry is the default before tuning.
#include "me2_item.hpp"

namespace heget {

extern const Me2Variant kShapesF32Meet7[] = {
    variant<float, 7, 7, 4, 2, 1, 0, 0, 1, 3>(), variant<float, 7, 7, 2, 2, 1, 0, 0, 1, 3>(),
};
extern const int kShapesF32Meet7Count = sizeof(kShapesF32Meet7) / sizeof(Me2Variant);

}  // namespace heget
