// Narrow-schedule kernel instantiations: float, 1-wide loads.
// Ordered by capacity S*NG*VEC rows.
#include "gs_narrow.hpp"
#include "gs_registry.hpp"

namespace gs {
const NarrowEntry kNarrowF32S[] = {
    GS_NARROW_ENTRY(float, 1, 4, 8, false),
    GS_NARROW_ENTRY(float, 1, 4, 12, false),
    GS_NARROW_ENTRY(float, 1, 4, 16, false),
    GS_NARROW_ENTRY(float, 1, 4, 24, false),
    GS_NARROW_ENTRY(float, 1, 4, 32, false),
    GS_NARROW_ENTRY(float, 1, 16, 16, false),
    GS_NARROW_ENTRY(float, 1, 16, 32, false),
    GS_NARROW_ENTRY(float, 1, 64, 16, false),
    GS_NARROW_ENTRY(float, 1, 64, 32, false)};
const int kNarrowF32SN = sizeof(kNarrowF32S) / sizeof(kNarrowF32S[0]);
}  // namespace gs
