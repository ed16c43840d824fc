// Narrow-schedule kernel instantiations: float, 1-wide loads, row gather.
// Ordered by capacity S*NG*VEC rows.
#include "gs_narrow.hpp"
#include "gs_registry.hpp"

namespace gs {
const NarrowEntry kNarrowF32G[] = {
    GS_NARROW_ENTRY(float, 1, 4, 8, true),
    GS_NARROW_ENTRY(float, 1, 4, 9, true),
    GS_NARROW_ENTRY(float, 1, 4, 12, true),
    GS_NARROW_ENTRY(float, 1, 4, 16, true),
    GS_NARROW_ENTRY(float, 1, 4, 24, true),
    GS_NARROW_ENTRY(float, 1, 4, 32, true),
    GS_NARROW_ENTRY(float, 1, 16, 16, true),
    GS_NARROW_ENTRY(float, 1, 16, 32, true),
    GS_NARROW_ENTRY(float, 1, 64, 16, true),
    GS_NARROW_ENTRY(float, 1, 64, 32, true)};
const int kNarrowF32GN = sizeof(kNarrowF32G) / sizeof(kNarrowF32G[0]);
}  // namespace gs
