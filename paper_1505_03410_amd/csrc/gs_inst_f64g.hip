// Narrow-schedule kernel instantiations: double, 1-wide loads, row gather.
// Ordered by capacity S*NG*VEC rows.
#include "gs_narrow.hpp"
#include "gs_registry.hpp"

namespace gs {
const NarrowEntry kNarrowF64G[] = {
    GS_NARROW_ENTRY(double, 1, 4, 8, true),
    GS_NARROW_ENTRY(double, 1, 4, 16, true),
    GS_NARROW_ENTRY(double, 1, 4, 32, true),
    GS_NARROW_ENTRY(double, 1, 16, 16, true),
    GS_NARROW_ENTRY(double, 1, 16, 32, true),
    GS_NARROW_ENTRY(double, 1, 64, 16, true),
    GS_NARROW_ENTRY(double, 1, 64, 32, true)};
const int kNarrowF64GN = sizeof(kNarrowF64G) / sizeof(kNarrowF64G[0]);
}  // namespace gs
