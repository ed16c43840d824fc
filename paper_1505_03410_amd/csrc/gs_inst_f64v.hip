// Narrow-schedule kernel instantiations: double, 2-wide loads.
// Ordered by capacity S*NG*VEC rows.
#include "gs_narrow.hpp"
#include "gs_registry.hpp"

namespace gs {
const NarrowEntry kNarrowF64V[] = {
    GS_NARROW_ENTRY(double, 2, 4, 4, false),
    GS_NARROW_ENTRY(double, 2, 4, 6, false),
    GS_NARROW_ENTRY(double, 2, 4, 8, false),
    GS_NARROW_ENTRY(double, 2, 4, 12, false),
    GS_NARROW_ENTRY(double, 2, 16, 4, false),
    GS_NARROW_ENTRY(double, 2, 16, 8, false),
    GS_NARROW_ENTRY(double, 2, 64, 4, false),
    GS_NARROW_ENTRY(double, 2, 64, 8, false),
    GS_NARROW_ENTRY(double, 2, 64, 16, false)};
const int kNarrowF64VN = sizeof(kNarrowF64V) / sizeof(kNarrowF64V[0]);
}  // namespace gs
