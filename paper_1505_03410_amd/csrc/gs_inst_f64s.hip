// Narrow-schedule kernel instantiations: double, 1-wide loads.
// Ordered by capacity S*NG*VEC rows.
#include "gs_narrow.hpp"
#include "gs_registry.hpp"

namespace gs {
const NarrowEntry kNarrowF64S[] = {
    GS_NARROW_ENTRY(double, 1, 4, 8, false),
    GS_NARROW_ENTRY(double, 1, 4, 16, false),
    GS_NARROW_ENTRY(double, 1, 4, 32, false),
    GS_NARROW_ENTRY(double, 1, 16, 16, false),
    GS_NARROW_ENTRY(double, 1, 16, 32, false),
    GS_NARROW_ENTRY(double, 1, 64, 16, false),
    GS_NARROW_ENTRY(double, 1, 64, 32, false)};
const int kNarrowF64SN = sizeof(kNarrowF64S) / sizeof(kNarrowF64S[0]);
}  // namespace gs
