// Narrow-schedule kernel instantiations: float, 4-wide loads.
// Ordered by capacity S*NG*VEC rows.
#include "gs_narrow.hpp"
#include "gs_registry.hpp"

namespace gs {
const NarrowEntry kNarrowF32V[] = {
    GS_NARROW_ENTRY(float, 4, 4, 2, false),
    GS_NARROW_ENTRY(float, 4, 4, 3, false),
    GS_NARROW_ENTRY(float, 4, 4, 4, false),
    GS_NARROW_ENTRY(float, 4, 4, 5, false),
    GS_NARROW_ENTRY(float, 4, 4, 6, false),
    GS_NARROW_ENTRY(float, 4, 4, 8, false),
    GS_NARROW_ENTRY(float, 4, 16, 3, false),
    GS_NARROW_ENTRY(float, 4, 16, 4, false),
    GS_NARROW_ENTRY(float, 4, 16, 6, false),
    GS_NARROW_ENTRY(float, 4, 16, 8, false),
    GS_NARROW_ENTRY(float, 4, 64, 3, false),
    GS_NARROW_ENTRY(float, 4, 64, 4, false),
    GS_NARROW_ENTRY(float, 4, 64, 6, false),
    GS_NARROW_ENTRY(float, 4, 64, 8, false)};
const int kNarrowF32VN = sizeof(kNarrowF32V) / sizeof(kNarrowF32V[0]);
}  // namespace gs
