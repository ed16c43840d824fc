// Table of compiled kernel configurations (filled by the gs_inst_*.hip files).
#pragma once

#include "gs_internal.hpp"

namespace gs {

struct NarrowEntry {
  Cfg cfg;
  const void* path_kernel;  // k_path_narrow<...>
  size_t lds_bytes;
};

struct WideEntry {
  int dtype, vec, NG;       // sweep layout: 64 lanes over rows
  const void* pre_kernel;   // k_wide_pre<...>
  const void* sweep_kernel; // k_wide_sweep<..., 0>
  const void* sweep_nrm_kernel;  // k_wide_sweep<..., 1>: also ||x_j||^2
  const void* sweep_nxy_kernel;  // k_wide_sweep<..., 2>: also ||x_j||^2 and x_j^T y
  const void* csweep_kernel;     // k_wide_csweep<...>: c from the resume position
  const void* gstar_kernel;      // k_wide_gstar<...>: x_j^T x_{j*} (Dynamic ST3)
  const void* walk_kernel;       // k_wide_walk<...>: the CD epoch on one wave
  int nmax() const { return 64 * NG * vec; }
};

extern const NarrowEntry kNarrowF32V[];
extern const int kNarrowF32VN;
extern const NarrowEntry kNarrowF32S[];
extern const int kNarrowF32SN;
extern const NarrowEntry kNarrowF32G[];
extern const int kNarrowF32GN;
extern const NarrowEntry kNarrowF64V[];
extern const int kNarrowF64VN;
extern const NarrowEntry kNarrowF64S[];
extern const int kNarrowF64SN;
extern const NarrowEntry kNarrowF64G[];
extern const int kNarrowF64GN;
extern const WideEntry kWide[];
extern const int kWideN;

// Type-dependent single kernels (gs_wide.hip).
extern const void* const kWideInit[2];     // k_wide_init<float>, <double>
extern const void* const kWideRefresh[2];  // k_wide_refresh<...>
extern const void* const kWideGap[2];      // k_wide_gap<...>
extern const void* const kScreenPrep[2];   // k_screen_prep<...>
extern const void* const kWideTest;
extern const void* const kWideCompact;
extern const void* const kWideFin;
extern const void* const kWideLCount;
extern const void* const kWideLCompact;
extern const void* const kWideStats;
// Sparse (CSC) designs (gs_csc.hip).
extern const void* const kCscColStats[2];  // k_csc_colstats<float>, <double>
extern const void* const kPathCsc[2][2];   // k_path_csc<XT, residual in global memory>
extern const void* const kFillI32;

}  // namespace gs

#define GS_NARROW_ENTRY(XT, VEC, S, NG, G)                                                  \
  {                                                                                         \
    {0, sizeof(XT) == 8 ? 1 : 0, VEC, S, NG, G},                                            \
        reinterpret_cast<const void*>(&gs::k_path_narrow<XT, VEC, S, NG, G>),               \
        gs::narrow_lds_bytes<XT, VEC, S, NG, G>()                                           \
  }
