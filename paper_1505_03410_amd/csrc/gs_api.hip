// C ABI: argument checks, workspace layout, kernel selection and launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gapsafe.h"
#include "gs_registry.hpp"
#include "gs_wide.hpp"

using namespace gs;

// ---- static scratch of screen_noalloc (for callers that cannot allocate).
// In host code `scratch` only names the symbol: its device address comes from
// hipGetSymbolAddress, and only that address is handed to kernels.
static_assert(GS_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[GS_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail_hip(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return GS_EHIP;
}

#define HIPCHK(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return fail_hip(e_, #call);  \
  } while (0)

constexpr int kMaxN = 2048;
static_assert(kMaxN <= kMaxRowsDense, "the wide refresh keeps kMaxN rows per block");
#ifndef GS_SWEEP_BLOCKS
#define GS_SWEEP_BLOCKS 2048
#endif
constexpr int kWideSweepBlocks = GS_SWEEP_BLOCKS;
constexpr int kWidePreBlocks = 1024;
// n*p above which GS_SCHED_AUTO spreads one path over the whole GPU.
constexpr double kWideThreshold = 16.0 * 1024 * 1024;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves aligned sub-arrays from a workspace (or only measures when base is
// null).
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * std::max<size_t>(count, 1);
    return p;
  }
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

bool is_csc(const gs_problem* pr) { return pr->format == GS_CSC; }

int check_problem(const gs_problem* pr) {
  if (!pr) return GS_EINVAL;
  if (pr->n < 1 || pr->p < 1 || pr->T < 1) return GS_EINVAL;
  if (pr->dtype != GS_F32 && pr->dtype != GS_F64) return GS_EINVAL;
  if (pr->format != GS_DENSE && pr->format != GS_CSC) return GS_EINVAL;
  if (is_csc(pr)) {
    if (!pr->col_ptr || !pr->row_idx || pr->rows) return GS_EINVAL;
  } else {
    if (!pr->rows && pr->ldx < pr->n) return GS_EINVAL;
    if (pr->ldx < 1) return GS_EINVAL;
  }
  if (!pr->X || !pr->y || !pr->beta_out || !pr->gap_out || !pr->epochs_out ||
      !pr->nactive_out || !pr->status_out)
    return GS_EINVAL;
  if (pr->lambdas) {
    for (int t = 0; t < pr->T; ++t) {
      if (!finite_pos(pr->lambdas[t])) return GS_EINVAL;
      if (t > 0 && pr->lambdas[t] > pr->lambdas[t - 1]) return GS_EINVAL;
    }
  } else {
    if (!finite_pos(pr->lambda_min_ratio) || pr->lambda_min_ratio > 1.0) return GS_EINVAL;
  }
  if (!is_csc(pr) && pr->n > kMaxN) return GS_EUNSUPPORTED;
  return GS_OK;
}

int check_opts(const gs_opts* o) {
  if (!finite_pos(o->eps_rel)) return GS_EINVAL;
  if (o->screen_every < 1 || o->max_epochs < 0) return GS_EINVAL;
  if (o->schedule < GS_SCHED_AUTO || o->schedule > GS_SCHED_WIDE) return GS_EINVAL;
  if (o->cd_mode < GS_CD_AUTO || o->cd_mode > GS_CD_RESIDUAL) return GS_EINVAL;
  if (o->rule < GS_RULE_SPHERE || o->rule > GS_RULE_ST3) return GS_EINVAL;
  const double a = o->enet_alpha == 0.0 ? 1.0 : o->enet_alpha;
  if (!(a > 0.0 && a <= 1.0)) return GS_EINVAL;
  if (a < 1.0 && o->rule >= GS_RULE_STATIC) return GS_EINVAL;  // Lasso-only rules
  return GS_OK;
}

// 16-byte loads need an aligned X, aligned columns and n a multiple of the
// vector width (no load then straddles row n).
bool vec_ok(const gs_problem* pr) {
  const size_t es = pr->dtype == GS_F64 ? 8 : 4;
  const int vec = (int)(16 / es);
  return (reinterpret_cast<uintptr_t>(pr->X) % 16 == 0) && ((size_t)pr->ldx * es) % 16 == 0 &&
         pr->n % vec == 0;
}

const NarrowEntry* narrow_table(int dtype, bool gather, bool vec, int* count) {
  if (dtype == GS_F32) {
    if (gather) { *count = kNarrowF32GN; return kNarrowF32G; }
    if (vec) { *count = kNarrowF32VN; return kNarrowF32V; }
    *count = kNarrowF32SN;
    return kNarrowF32S;
  }
  if (gather) { *count = kNarrowF64GN; return kNarrowF64G; }
  if (vec) { *count = kNarrowF64VN; return kNarrowF64V; }
  *count = kNarrowF64SN;
  return kNarrowF64S;
}

// ---- tile choice.  A class of problems is (table, smallest entry that holds
// n); the autotuner may map a class to another entry of the same table that
// also holds n.  Keys: (table base pointer, smallest index).
std::mutex g_tune_mu;
std::map<std::pair<const NarrowEntry*, int>, int> g_tuned;
// Schedule autotuner: per dtype, the n*p above which lasso_path's "auto"
// schedule is wide, and the measured points (n*p, wide faster) it was set from.
double g_wide_thr[2] = {kWideThreshold, kWideThreshold};
std::vector<std::pair<double, bool>> g_sched_pts[2];

double wide_threshold(int dtype) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_wide_thr[dtype == GS_F64 ? 1 : 0];
}

// The problem cut to the first k lambdas of its grid: an explicit list keeps
// its first k entries; a generated grid lambda_max * ratio^(t/(T-1)) keeps
// its first k points through the ratio ratio^((k-1)/(T-1)).
void first_lambdas(gs_problem* q, int k) {
  if (k >= q->T) return;
  if (!q->lambdas && q->T > 1)
    q->lambda_min_ratio = k > 1 ? std::pow(q->lambda_min_ratio, (double)(k - 1) / (q->T - 1)) : 1.0;
  q->T = k;
}

// The cut between the measured sizes that misclassifies the fewest points
// (the geometric midpoint of the two sizes around it); the default when
// there are no points.
double fit_threshold(std::vector<std::pair<double, bool>> pts) {
  if (pts.empty()) return kWideThreshold;
  std::sort(pts.begin(), pts.end());
  const int m = (int)pts.size();
  int best_err = m + 1;
  double best = kWideThreshold;
  for (int k = 0; k <= m; ++k) {  // narrow for the first k points, wide for the rest
    int err = 0;
    for (int i = 0; i < m; ++i) err += (i < k) == pts[i].second ? 1 : 0;
    if (err < best_err) {
      best_err = err;
      if (k == 0) best = pts[0].first * 0.5;
      else if (k == m) best = pts[m - 1].first * 2.0;
      else best = std::sqrt(pts[k - 1].first * pts[k].first);
    }
  }
  return best;
}
// set while the autotuner times one candidate (this thread only)
thread_local const NarrowEntry* g_force = nullptr;

int smallest_fit(const NarrowEntry* tab, int cnt, int n) {
  for (int i = 0; i < cnt; ++i)
    if (tab[i].cfg.nmax() >= n) return i;
  return -1;
}

// The narrow configuration of a problem: the tuned one of its class, else the
// smallest compiled one that holds n rows.
const NarrowEntry* pick_narrow(const gs_problem* pr) {
  int cnt = 0;
  const NarrowEntry* tab = narrow_table(pr->dtype, pr->rows != nullptr, vec_ok(pr), &cnt);
  const int i0 = smallest_fit(tab, cnt, pr->n);
  if (i0 < 0) return nullptr;
  if (g_force) return g_force;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find({tab, i0});
  if (it != g_tuned.end() && it->second < cnt && tab[it->second].cfg.nmax() >= pr->n)
    return &tab[it->second];
  return &tab[i0];
}

const WideEntry* pick_wide(const gs_problem* pr) {
  const bool v = vec_ok(pr);
  const int want_vec = v ? (pr->dtype == GS_F64 ? 2 : 4) : 1;
  for (int i = 0; i < kWideN; ++i) {
    const WideEntry& w = kWide[i];
    if (w.dtype == pr->dtype && w.vec == want_vec && w.nmax() >= pr->n) return &w;
  }
  return nullptr;
}

bool use_wide(const gs_problem* pr, const gs_opts* o) {
  if (pr->rows) return false;  // the wide kernels read contiguous rows only
  if (o->schedule == GS_SCHED_WIDE) return true;
  if (o->rule >= GS_RULE_STATIC) return true;  // comparison rules: wide schedule only
  if (o->enet_alpha != 0.0 && o->enet_alpha < 1.0) return true;  // elastic net: likewise
  if (o->schedule == GS_SCHED_NARROW) return false;
  return (double)pr->n * (double)pr->p > wide_threshold(pr->dtype);
}

// Per-problem workspace arrays.
// Gram slots of the pattern mode: a Lasso solution has at most n nonzeros in
// general position; the margin covers transient supports.
int pattern_slots(const gs_problem* pr) {
  if (is_csc(pr)) return 1;  // the CSC path has no pattern mode
  const int want = (pr->n + 7) / 8 * 8 + 16;
  return std::max(1, std::min({kSlotsMax, pr->p, want}));
}

// Per-problem workspace arrays.  The pattern mode's arrays hold ldg entries
// (p rounded up to 256).
void carve_problem(Carver& cv, const gs_problem* pr, ProbDesc* d) {
  const int64_t ldg = (int64_t)align_up((size_t)pr->p, 256);
  const int ns = pattern_slots(pr);
  d->nrm2 = cv.take<double>(pr->p);
  d->xty = cv.take<double>(pr->p);
  d->gst = cv.take<double>(pr->p);
  d->inv = cv.take<double>(pr->p);
  d->beta = cv.take<double>(pr->p);
  d->c = cv.take<double>(ldg);
  d->act = cv.take<int32_t>(2 * (size_t)pr->p);
  d->lam = cv.take<double>(pr->T);
  d->lam_in = cv.take<double>(pr->T);
  d->rho = cv.take<double>(pr->n);
  d->gc = cv.take<float>((size_t)ns * ldg);
  d->ng = cv.take<float>(ldg);
  d->pslot = cv.take<int32_t>(ldg);
  d->pmem = cv.take<int32_t>(ldg);
  d->c2 = cv.take<double>(ldg);
  d->lst = cv.take<int32_t>(2 * (size_t)pr->p);
  d->lval = cv.take<double>(4 * (size_t)pr->p);
  d->ldg = ldg;
  d->ns = ns;
}

// LDS floats of the support's Gram block: up to ns columns (rounded up to 8)
// of stride 64 or 128.
int gs_floats(int ns) { return (ns + 7) / 8 * 8 * (ns > 64 ? 128 : 64); }

struct Shared {
  ProbDesc* descs;
  int32_t* queues;   // 64 counters
  WideState* st;
  WideBufs wb;
};

void carve_shared(Carver& cv, int B, int pmax, Shared* s) {
  s->descs = cv.take<ProbDesc>(B);
  s->queues = cv.take<int32_t>(64);
  s->st = cv.take<WideState>(1);
  s->wb.part = cv.take<double>(4 * (size_t)std::max(kWideSweepBlocks, kWidePreBlocks));
  s->wb.cnt = cv.take<int32_t>((pmax + kTestTile - 1) / kTestTile + 1);
  s->wb.nzidx = cv.take<int32_t>(pmax);
  s->wb.nzval = cv.take<double>(pmax);
}

void fill_desc(const gs_problem* pr, int orig, ProbDesc* d) {
  d->X = pr->X;
  d->y = pr->y;
  d->rows = pr->rows;
  d->format = pr->format;
  d->col_ptr = pr->col_ptr;
  d->row_idx = pr->row_idx;
  d->ldx = pr->ldx;
  d->n = pr->n;
  d->p = pr->p;
  d->T = pr->T;
  d->dtype = pr->dtype;
  d->lambda_relative = pr->lambda_relative ? 1 : 0;
  d->has_lambdas = pr->lambdas ? 1 : 0;
  d->lambda_min_ratio = pr->lambda_min_ratio;
  d->beta_init = pr->beta_init;
  d->beta_out = pr->beta_out;
  d->gap_out = pr->gap_out;
  d->epochs_out = pr->epochs_out;
  d->nactive_out = pr->nactive_out;
  d->status_out = pr->status_out;
  d->lambda_out = pr->lambda_out;
  d->orig = orig;
}

PathOpts path_opts(const gs_opts* o, bool batch) {
  PathOpts po;
  po.eps_rel = o->eps_rel;
  po.f = o->screen_every;
  po.K = o->max_epochs;
  po.lds_cap = 0;
  po.pattern = o->cd_mode == GS_CD_RESIDUAL ? 0 : 1;
  po.gs_cap = 0;
  po.rule = o->rule;
  po.enet = o->enet_alpha == 0.0 ? 1.0 : o->enet_alpha;
  po.select_counts = batch ? o->select_counts : nullptr;
  po.timestamps = batch ? reinterpret_cast<long long*>(o->timestamps) : nullptr;
  po.stats = reinterpret_cast<long long*>(o->stats);
  return po;
}

hipError_t launch(const void* k, dim3 g, dim3 b, void** args, size_t smem, hipStream_t s) {
  return hipLaunchKernel(k, g, b, args, smem, s);
}

// ---- optional event timing of selected kernels (gs_timing_*)
struct Timed {
  int slot;
  hipEvent_t a, b;
};
bool g_timing = false;
std::vector<Timed> g_pending;
double g_total_ms[3] = {0.0, 0.0, 0.0};
int64_t g_launches[3] = {0, 0, 0};
enum { kTimeSweep = 0, kTimePath = 1, kTimeCD = 2 };

hipError_t timed_launch(int slot, const void* k, dim3 g, dim3 b, void** args, size_t smem,
                        hipStream_t s) {
  if (!g_timing) return launch(k, g, b, args, smem, s);
  Timed t{slot, nullptr, nullptr};
  // device-scope events: no system-scope cache release around the kernel
  const unsigned fl = hipEventDisableSystemFence;
  hipError_t e = hipEventCreateWithFlags(&t.a, fl);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&t.b, fl);
  if (e == hipSuccess) e = hipEventRecord(t.a, s);
  if (e == hipSuccess) e = launch(k, g, b, args, smem, s);
  if (e == hipSuccess) e = hipEventRecord(t.b, s);
  if (e == hipSuccess) {
    g_pending.push_back(t);
  } else {
    if (t.a) (void)hipEventDestroy(t.a);
    if (t.b) (void)hipEventDestroy(t.b);
  }
  return e;
}

void resolve_timing() {
  for (const Timed& t : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      g_total_ms[t.slot] += ms;
      g_launches[t.slot] += 1;
    }
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  g_pending.clear();
}

hipError_t fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s) {
  int64_t cnt = count;
  void* args[] = {&p, &v, &cnt};
  unsigned g = (unsigned)std::min<int64_t>((count + 255) / 256, 1024);
  return launch(kFillI32, dim3(std::max(g, 1u)), dim3(256), args, 0, s);
}

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
  }
  return cus;
}

size_t device_lds_per_cu() {
  static int lds = 0;
  if (!lds) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess ||
        lds <= 0)
      lds = 64 * 1024;
  }
  return (size_t)lds;
}

// Number of concurrently resident wavefronts of a narrow kernel.
int narrow_slots(const NarrowEntry* e, size_t lds) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, e->path_kernel, 64, lds) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * device_cus();
}

// Size (floats) of the residual mode's LDS staging region for `count`
// problems of one configuration: the LDS of a CU is shared by the wavefronts
// that must run on it at once.
int lds_cap_for(const NarrowEntry* e, int count, int gs) {
  const size_t per_cu = device_lds_per_cu();
  const int cus = device_cus();
  const int waves = std::max(1, (count + cus - 1) / cus);
  const size_t budget = per_cu / waves;
  const size_t fixed = e->lds_bytes + sizeof(float) * (size_t)gs;
  if (budget <= fixed + 4096) return 0;
  size_t cap = (budget - fixed - 1024) / sizeof(float);
  cap = std::min<size_t>(cap, 1 << 20) & ~(size_t)63;
  return (int)cap;
}

// Upload the lambdas of each problem into its workspace copy.
int upload_lambdas(const gs_problem* pr, const ProbDesc* d, hipStream_t s) {
  if (pr->lambdas)
    HIPCHK(hipMemcpyAsync(d->lam_in, pr->lambdas, sizeof(double) * pr->T, hipMemcpyHostToDevice, s));
  return GS_OK;
}

// ---------------------------------------------------------------- wide path
int run_wide(const gs_problem* pr, const gs_opts* o, const Shared& sh, ProbDesc d,
             hipStream_t s) {
  const WideEntry* w = pick_wide(pr);
  if (!w) return GS_EUNSUPPORTED;
  PathOpts po = path_opts(o, false);
  WideState* st = sh.st;
  WideBufs wb = sh.wb;
  const int dt = pr->dtype;
  // precompute + init
  {
    void* a[] = {&d, &wb};
    HIPCHK(launch(w->pre_kernel, dim3(kWidePreBlocks), dim3(64 * kSweepWaves), a, 0, s));
    int npre = kWidePreBlocks;
    void* b[] = {&d, &st, &wb, &npre, &po};
    HIPCHK(launch(kWideInit[dt], dim3(1), dim3(256), b, 0, s));
    if (o->rule == GS_RULE_ST3) {
      void* g[] = {&d, &st};
      HIPCHK(launch(w->gstar_kernel, dim3(kWidePreBlocks), dim3(64 * kSweepWaves), g, 0, s));
    }
  }
  const int ntest = (pr->p + kTestTile - 1) / kTestTile;
  int nsweep = std::max(1, std::min(kWideSweepBlocks, (pr->p + kSweepWaves * kSweepU - 1) /
                                                                (kSweepWaves * kSweepU)));
  int zero = 0, one = 1;
  int32_t* nullq = nullptr;
  int32_t* nullo = nullptr;
  double* nd = nullptr;
  int nt = ntest;
  // One iteration enqueues a screening pass and f CD rounds; every kernel
  // checks the state machine, so a pass runs only when the previous f epochs
  // are done and a round only while an epoch is pending (a round that
  // re-anchors part of an epoch leaves the rest to the next iteration).
  const long long max_iter =
      4 * ((long long)pr->T * ((long long)o->max_epochs / o->screen_every + 3) + 16);
  long long enq = 0;
  int chunk = 4;
  for (;;) {
    for (int i = 0; i < chunk; ++i) {
      void* ar[] = {&d, &st, &wb, &zero};
      HIPCHK(launch(kWideRefresh[dt], dim3(1), dim3(kRefreshThreads), ar, 0, s));
      void* as[] = {&d, &st, &wb};
      HIPCHK(timed_launch(kTimeSweep, w->sweep_kernel, dim3(nsweep), dim3(64 * kSweepWaves), as,
                          0, s));
      void* ag[] = {&d, &st, &wb, &nsweep, &zero, &nd, &nd, &nd, &po};
      HIPCHK(launch(kWideGap[dt], dim3(1), dim3(256), ag, 0, s));
      void* at[] = {&d, &st, &wb};
      HIPCHK(launch(kWideTest, dim3(ntest), dim3(256), at, 0, s));
      void* ac[] = {&d, &st, &wb, &nullo};
      HIPCHK(launch(kWideCompact, dim3(ntest), dim3(256), ac, 0, s));
      void* af[] = {&d, &st, &wb, &nt, &nullq};
      HIPCHK(launch(kWideFin, dim3(1), dim3(64), af, 0, s));
      void* ar2[] = {&d, &st, &wb, &one};
      HIPCHK(launch(kWideRefresh[dt], dim3(1), dim3(kRefreshThreads), ar2, 0, s));
      for (int r = 0; r < o->screen_every; ++r) {
        void* a1[] = {&d, &st};
        HIPCHK(launch(w->csweep_kernel, dim3(nsweep), dim3(64 * kSweepWaves), a1, 0, s));
        void* a2[] = {&d, &st, &wb};
        HIPCHK(launch(kWideLCount, dim3(ntest), dim3(256), a2, 0, s));
        HIPCHK(launch(kWideLCompact, dim3(ntest), dim3(256), a2, 0, s));
        void* a3[] = {&d, &st, &wb, &nt, &po};
        HIPCHK(timed_launch(kTimeCD, w->walk_kernel, dim3(1), dim3(64), a3, 0, s));
      }
    }
    enq += chunk;
    WideState hs;
    HIPCHK(hipMemcpyAsync(&hs, st, sizeof(WideState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hs.done) {
      if (po.stats) {
        void* a[] = {&st, &po.stats};
        HIPCHK(launch(kWideStats, dim3(1), dim3(64), a, 0, s));
      }
      return hs.status_acc ? GS_NOT_CONVERGED : GS_OK;
    }
    if (enq > max_iter) {
      g_err = "wide schedule: pass budget exceeded";
      return GS_EHIP;
    }
    chunk = std::min(chunk * 2, 32);
  }
}

size_t path_ws(const gs_problem* probs, int B) {
  Carver cv{nullptr};
  int pmax = 1;
  for (int b = 0; b < B; ++b) pmax = std::max(pmax, probs[b].p);
  Shared sh;
  carve_shared(cv, B, pmax, &sh);
  for (int b = 0; b < B; ++b) {
    ProbDesc d;
    carve_problem(cv, &probs[b], &d);
  }
  cv.take<int64_t>(2 * ((size_t)B + 1));  // CSC: first column of every problem, per dtype
  return align_up(cv.off, 256);
}

// ---------------------------------------------------------- sparse (CSC)
// LDS of one CSC wavefront whose residual sits in LDS (n doubles).
constexpr size_t kCscLdsMax = 152 * 1024;

int run_csc(const gs_problem* probs, int B, const gs_opts* o, void* ws, size_t ws_bytes,
            hipStream_t s) {
  for (int b = 0; b < B; ++b)
    if (!is_csc(&probs[b])) return GS_EUNSUPPORTED;  // all CSC or all dense
  if (o->rule >= GS_RULE_STATIC || (o->enet_alpha != 0.0 && o->enet_alpha != 1.0))
    return GS_EUNSUPPORTED;
  if (!ws) return GS_EWORKSPACE;
  if (ws_bytes < path_ws(probs, B)) return GS_EWORKSPACE;
  Carver cv{static_cast<char*>(ws)};
  int pmax = 1;
  for (int b = 0; b < B; ++b) pmax = std::max(pmax, probs[b].p);
  Shared sh;
  carve_shared(cv, B, pmax, &sh);
  // groups by (dtype, residual in global memory); heaviest first inside
  std::vector<ProbDesc> descs(B);
  std::vector<int> key(B);
  for (int b = 0; b < B; ++b) {
    fill_desc(&probs[b], b, &descs[b]);
    carve_problem(cv, &probs[b], &descs[b]);
    int rc = upload_lambdas(&probs[b], &descs[b], s);
    if (rc) return rc;
    const bool grho = (size_t)probs[b].n * sizeof(double) > kCscLdsMax;
    key[b] = probs[b].dtype * 2 + (grho ? 1 : 0);
  }
  int64_t* first_col = cv.take<int64_t>(2 * ((size_t)B + 1));
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (key[a] != key[b]) return key[a] < key[b];
    return (double)probs[a].p * probs[a].T > (double)probs[b].p * probs[b].T;
  });
  std::vector<ProbDesc> sorted(B);
  for (int i = 0; i < B; ++i) sorted[i] = descs[order[i]];
  HIPCHK(hipMemcpyAsync(sh.descs, sorted.data(), sizeof(ProbDesc) * B, hipMemcpyHostToDevice, s));
  // the problems of each dtype are contiguous in `sorted`; per dtype, the
  // prefix of their column counts from 0 (first_col + dtype (B + 1))
  std::vector<int64_t> fcd(2 * ((size_t)B + 1), 0);
  int dfirst[2] = {-1, -1}, dcount[2] = {0, 0};
  for (int i = 0; i < B; ++i) {
    const int dt = sorted[i].dtype;
    if (dfirst[dt] < 0) dfirst[dt] = i;
    int64_t* f = fcd.data() + dt * (B + 1);
    f[dcount[dt] + 1] = f[dcount[dt]] + sorted[i].p;
    ++dcount[dt];
  }
  HIPCHK(fill_i32(sh.queues, 0, 64, s));
  HIPCHK(hipMemcpyAsync(first_col, fcd.data(), sizeof(int64_t) * fcd.size(), hipMemcpyHostToDevice,
                        s));
  PathOpts po = path_opts(o, B > 1);
  // column statistics of every problem (one pass over the nonzeros), per dtype
  for (int dt = 0; dt < 2; ++dt) {
    if (dfirst[dt] < 0) continue;
    const ProbDesc* dd = sh.descs + dfirst[dt];
    const int nb = dcount[dt];
    const int64_t* fcp = first_col + dt * ((int64_t)B + 1);
    const int64_t cols = fcd[dt * (B + 1) + nb];
    unsigned g = (unsigned)std::min<int64_t>((cols + 3) / 4, 8192);
    void* a[] = {(void*)&dd, (void*)&nb, (void*)&fcp};
    HIPCHK(launch(kCscColStats[dt], dim3(std::max(g, 1u)), dim3(256), a, 0, s));
  }
  // one persistent launch per group
  int gi = 0;
  for (int i = 0; i < B;) {
    int j = i;
    while (j < B && key[order[j]] == key[order[i]]) ++j;
    const int kk = key[order[i]];
    const int dt = kk / 2, grho = kk % 2;
    size_t lds = 0;
    if (!grho)
      for (int t = i; t < j; ++t) lds = std::max(lds, (size_t)sorted[t].n * sizeof(double));
    const void* kern = kPathCsc[dt][grho];
    HIPCHK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    const int grid = std::max(1, std::min(j - i, per_cu * device_cus()));
    const ProbDesc* dd = sh.descs + i;
    int cnt = j - i;
    int* q = sh.queues + gi;
    void* a[] = {(void*)&dd, &cnt, &q, &po};
    HIPCHK(timed_launch(kTimePath, kern, dim3(grid), dim3(64), a, lds, s));
    ++gi;
    i = j;
  }
  return GS_OK;
}

// Narrow launches of a (sorted) descriptor range grouped by configuration.
struct Group {
  const NarrowEntry* e;
  int first, count;
  int gs;       // LDS floats of the largest support Gram block in the group
  double cost;  // sum of n p T over the group's problems
};

int prepare_batch(const gs_problem* probs, int B, const gs_opts* o, void* ws, size_t ws_bytes,
                  hipStream_t s, Shared* sh, std::vector<Group>* groups) {
  if (!probs || B < 1 || !o) return GS_EINVAL;
  int rc = check_opts(o);
  if (rc) return rc;
  if (o->rule >= GS_RULE_STATIC) return GS_EUNSUPPORTED;  // wide schedule only
  if (o->enet_alpha != 0.0 && o->enet_alpha < 1.0) return GS_EUNSUPPORTED;
  for (int b = 0; b < B; ++b) {
    rc = check_problem(&probs[b]);
    if (rc) return rc;
    if (is_csc(&probs[b])) return GS_EUNSUPPORTED;  // CSC: lasso_path / lasso_solve_batch
    if (o->select_counts && (probs[b].p != probs[0].p || probs[b].T != probs[0].T))
      return GS_EINVAL;
  }
  if (!ws) return GS_EWORKSPACE;
  const size_t need = path_ws(probs, B);
  if (ws_bytes < need) return GS_EWORKSPACE;
  Carver cv{static_cast<char*>(ws)};
  int pmax = 1;
  for (int b = 0; b < B; ++b) pmax = std::max(pmax, probs[b].p);
  carve_shared(cv, B, pmax, sh);
  std::vector<ProbDesc> descs(B);
  std::vector<const NarrowEntry*> cfg(B);
  for (int b = 0; b < B; ++b) {
    fill_desc(&probs[b], b, &descs[b]);
    carve_problem(cv, &probs[b], &descs[b]);
    cfg[b] = pick_narrow(&probs[b]);
    if (!cfg[b]) return GS_EUNSUPPORTED;
    rc = upload_lambdas(&probs[b], &descs[b], s);
    if (rc) return rc;
  }
  // Group by configuration; inside a group, most expensive first.
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) order[b] = b;
  auto cost = [&](int b) { return (double)probs[b].n * probs[b].p * probs[b].T; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (cfg[a] != cfg[b]) return cfg[a] < cfg[b];
    return cost(a) > cost(b);
  });
  std::vector<ProbDesc> sorted(B);
  groups->clear();
  for (int i = 0; i < B; ++i) {
    sorted[i] = descs[order[i]];
    const NarrowEntry* e = cfg[order[i]];
    if (groups->empty() || groups->back().e != e) groups->push_back({e, i, 0, 0, 0.0});
    groups->back().count++;
    groups->back().cost += cost(order[i]);
    groups->back().gs = std::max(groups->back().gs, gs_floats(sorted[i].ns));
  }
  if ((int)groups->size() > 63) return GS_EUNSUPPORTED;
  HIPCHK(hipMemcpyAsync(sh->descs, sorted.data(), sizeof(ProbDesc) * B, hipMemcpyHostToDevice, s));
  return GS_OK;
}

// One persistent launch of a group: its kernel, grid, LDS and arguments.
struct Launch {
  const void* kernel;
  int grid;
  size_t lds;
  const ProbDesc* descs;
  int B;
  int* queue;
  PathOpts po;
  double cost;
};

// LDS split and grid of every group; sets the kernels' LDS limits (not a
// stream operation, so it stays outside graph capture).
int configure_groups(const Shared& sh, const std::vector<Group>& groups, PathOpts po,
                     std::vector<Launch>* out) {
  out->clear();
  for (size_t g = 0; g < groups.size(); ++g) {
    const Group& G = groups[g];
    Launch L;
    L.kernel = G.e->path_kernel;
    L.descs = sh.descs + G.first;
    L.B = G.count;
    L.queue = sh.queues + g;
    L.po = po;
    L.cost = G.cost;
    // the support's Gram block first (when the CU's share holds it), then
    // the residual mode's staging region
    const size_t per_wave = device_lds_per_cu() /
                            std::max(1, (G.count + device_cus() - 1) / device_cus());
    L.po.gs_cap =
        (po.pattern && G.e->lds_bytes + sizeof(float) * (size_t)G.gs + 1024 <= per_wave) ? G.gs
                                                                                           : 0;
    L.po.lds_cap = lds_cap_for(G.e, G.count, L.po.gs_cap);
    L.lds = G.e->lds_bytes + sizeof(float) * ((size_t)L.po.gs_cap + (size_t)L.po.lds_cap);
    HIPCHK(hipFuncSetAttribute(L.kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds));
    L.grid = std::max(1, std::min(G.count, narrow_slots(G.e, L.lds)));
    out->push_back(L);
  }
  return GS_OK;
}

// Side streams (default priority) and fork/join events of one device, made
// once and kept for the process: the group launches of a batch spread over
// the caller's stream and these, so that groups of different tile
// configurations run side by side instead of one after another.
constexpr int kSideStreams = 3;
struct SidePool {
  hipStream_t st[kSideStreams];
  hipEvent_t fork, join[kSideStreams];
};
std::mutex g_side_mu;
std::map<int, SidePool> g_side;

int side_pool(SidePool** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_side_mu);
  auto it = g_side.find(dev);
  if (it == g_side.end()) {
    SidePool p{};
    for (int i = 0; i < kSideStreams; ++i) {
      HIPCHK(hipStreamCreateWithFlags(&p.st[i], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&p.join[i], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&p.fork, hipEventDisableTiming));
    it = g_side.emplace(dev, p).first;
  }
  *out = &it->second;
  return GS_OK;
}

// Queue reset (a fill kernel, no memset node) and the group launches.  With
// several groups, the heaviest goes first onto the least loaded of the
// caller's stream and the side streams, which fork from the caller's stream
// after the reset and join it at the end (also under graph capture).
int enqueue_groups(const Shared& sh, std::vector<Launch>& launches, hipStream_t s, bool timed) {
  HIPCHK(fill_i32(sh.queues, 0, 64, s));
  const int nl = (int)launches.size();
  SidePool* sp = nullptr;
  const int nside = nl > 1 ? std::min(nl - 1, kSideStreams) : 0;
  if (nside > 0) {
    int rc = side_pool(&sp);
    if (rc) return rc;
    HIPCHK(hipEventRecord(sp->fork, s));
    for (int i = 0; i < nside; ++i) HIPCHK(hipStreamWaitEvent(sp->st[i], sp->fork, 0));
  }
  std::vector<int> order(nl);
  for (int i = 0; i < nl; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return launches[a].cost > launches[b].cost; });
  std::vector<double> load(nside + 1, 0.0);
  for (int i : order) {
    Launch& L = launches[i];
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[k] += L.cost;
    hipStream_t ls = k == 0 ? s : sp->st[k - 1];
    void* a[] = {&L.descs, &L.B, &L.queue, &L.po};
    if (timed)
      HIPCHK(timed_launch(kTimePath, L.kernel, dim3(L.grid), dim3(64), a, L.lds, ls));
    else
      HIPCHK(launch(L.kernel, dim3(L.grid), dim3(64), a, L.lds, ls));
  }
  for (int i = 0; i < nside; ++i) {
    HIPCHK(hipEventRecord(sp->join[i], sp->st[i]));
    HIPCHK(hipStreamWaitEvent(s, sp->join[i], 0));
  }
  return GS_OK;
}

int launch_groups(const Shared& sh, const std::vector<Group>& groups, PathOpts po,
                  hipStream_t s) {
  std::vector<Launch> launches;
  int rc = configure_groups(sh, groups, po, &launches);
  if (rc) return rc;
  return enqueue_groups(sh, launches, s, true);
}

// Arrays of one screen() pass: the state, the sweep partials, the test
// counts, the refresh's nonzero list, and per column ||x_j||^2, the FP64
// coefficients, c and the active list; rho per row.  The path arrays (Gram
// cache and the like) are not needed here.
void carve_screen(Carver& cv, int n, int p, Shared* s, ProbDesc* d) {
  s->descs = nullptr;
  s->queues = nullptr;
  s->st = cv.take<WideState>(1);
  s->wb.part = cv.take<double>(4 * (size_t)std::max(kWideSweepBlocks, kWidePreBlocks));
  s->wb.cnt = cv.take<int32_t>((p + kTestTile - 1) / kTestTile + 1);
  s->wb.nzidx = cv.take<int32_t>(p);
  s->wb.nzval = cv.take<double>(p);
  d->nrm2 = cv.take<double>(p);
  d->xty = cv.take<double>(p);
  d->beta = cv.take<double>(p);
  d->c = cv.take<double>(p);
  d->act = cv.take<int32_t>(p);
  d->lam = cv.take<double>(1);
  d->rho = cv.take<double>(n);
}

int check_screen(int32_t n, int32_t p, int64_t ldx, int32_t dtype, const void* X, const void* y,
                 const double* beta, double lambda, int32_t rule, const int32_t* active_in,
                 int32_t q_in,
                 int32_t* active_out, int32_t* q_out, double* gap_out, double* alpha_out,
                 double* radius_out) {
  if (n < 1 || p < 1 || ldx < n) return GS_EINVAL;
  if (dtype != GS_F32 && dtype != GS_F64) return GS_EINVAL;
  if (!X || !y || !beta || !active_out || !q_out || !gap_out || !alpha_out || !radius_out)
    return GS_EINVAL;
  if (!finite_pos(lambda)) return GS_EINVAL;
  if (rule >= GS_RULE_STATIC && rule <= GS_RULE_ST3) return GS_EUNSUPPORTED;
  if (rule != GS_RULE_SPHERE && rule != GS_RULE_DOME) return GS_EINVAL;
  if (active_in && (q_in < 0 || q_in > p)) return GS_EINVAL;
  if (n > kMaxN) return GS_EUNSUPPORTED;
  return GS_OK;
}

// The pass itself on the arrays carved from `base` (a workspace, or the
// static scratch of screen_noalloc).
int run_screen(int32_t n, int32_t p, int64_t ldx, int32_t dtype, const void* X, const void* y,
               const double* beta, double lambda, int32_t rule, const int32_t* active_in,
               int32_t q_in,
               int32_t* active_out, int32_t* q_out, double* gap_out, double* alpha_out,
               double* radius_out, double* c_out, char* base, hipStream_t s) {
  const int q = active_in ? q_in : p;
  gs_problem pr{};
  pr.n = n;
  pr.p = p;
  pr.ldx = ldx;
  pr.dtype = dtype;
  pr.X = X;
  pr.y = y;
  pr.T = 1;
  const WideEntry* w = pick_wide(&pr);
  if (!w) return GS_EUNSUPPORTED;
  Carver cv{base};
  Shared sh;
  ProbDesc d{};
  fill_desc(&pr, 0, &d);
  carve_screen(cv, n, p, &sh, &d);
  if (c_out) d.c = c_out;
  WideState* st = sh.st;
  WideBufs wb = sh.wb;
  PathOpts po{};
  po.eps_rel = 1.0;
  po.f = 1;
  po.K = 0;
  {
    int qi = q, ru = rule;  // all p positions when active_in is NULL (q_in is ignored)
    void* a[] = {&d, &st, (void*)&beta, (void*)&active_in, &qi, &lambda, &ru};
    const int nprep = std::max(1, std::min(1024, (p + 1023) / 1024));
    HIPCHK(launch(kScreenPrep[dtype], dim3(nprep), dim3(256), a, 0, s));
  }
  int zero = 0, one = 1;
  {
    void* a[] = {&d, &st, &wb, &zero};
    HIPCHK(launch(kWideRefresh[dtype], dim3(1), dim3(kRefreshThreads), a, 0, s));
  }
  int nsweep = std::max(1, std::min(kWideSweepBlocks, (q + kSweepWaves * kSweepU - 1) /
                                                          (kSweepWaves * kSweepU)));
  {
    void* a[] = {&d, &st, &wb};
    HIPCHK(timed_launch(kTimeSweep, rule == GS_RULE_DOME ? w->sweep_nxy_kernel : w->sweep_nrm_kernel,
                        dim3(nsweep), dim3(64 * kSweepWaves), a, 0, s));
  }
  {
    void* a[] = {&d, &st, &wb, &nsweep, &one, &gap_out, &alpha_out, &radius_out, &po};
    HIPCHK(launch(kWideGap[dtype], dim3(1), dim3(256), a, 0, s));
  }
  int ntest = std::max(1, (q + kTestTile - 1) / kTestTile);
  {
    void* a[] = {&d, &st, &wb};
    HIPCHK(launch(kWideTest, dim3(ntest), dim3(256), a, 0, s));
  }
  {
    void* a[] = {&d, &st, &wb, &active_out};
    HIPCHK(launch(kWideCompact, dim3(ntest), dim3(256), a, 0, s));
  }
  {
    void* a[] = {&d, &st, &wb, &ntest, &q_out};
    HIPCHK(launch(kWideFin, dim3(1), dim3(64), a, 0, s));
  }
  return GS_OK;
}

// Device address of the static scratch on the current device (looked up
// once per device: each GPU holds its own copy of the array).
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;

int scratch_base(char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      g_err = "hipGetSymbolAddress(scratch) returned a null address";
      return GS_EHIP;
    }
    it = g_scratch_ptr.emplace(dev, static_cast<char*>(ptr)).first;
  }
  *out = it->second;
  return GS_OK;
}

}  // namespace

int gs::set_hip_error(hipError_t e, const char* where) { return fail_hip(e, where); }

// ======================================================================= ABI

extern "C" {

void gs_opts_default(gs_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps_rel = 1e-8;
  o->screen_every = 10;
  o->max_epochs = 100000;
  o->schedule = GS_SCHED_AUTO;
  o->enet_alpha = 1.0;
}

double gs_wallclock_hz(void) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0.0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0.0;
  return 1000.0 * khz;
}

size_t lasso_workspace_size(const gs_problem* probs, int32_t B, const gs_opts* opts) {
  if (!probs || B < 1) return 0;
  gs_opts def;
  gs_opts_default(&def);
  if (!opts) opts = &def;
  if (check_opts(opts)) return 0;
  for (int b = 0; b < B; ++b)
    if (check_problem(&probs[b])) return 0;
  return path_ws(probs, B);
}

int lasso_path(const gs_problem* prob, const gs_opts* opts, void* workspace, size_t ws_bytes,
               void* stream) {
  gs_opts def;
  gs_opts_default(&def);
  if (!opts) opts = &def;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = check_opts(opts);
  if (rc) return rc;
  rc = check_problem(prob);
  if (rc) return rc;
  if (!workspace) return GS_EWORKSPACE;
  if (ws_bytes < path_ws(prob, 1)) return GS_EWORKSPACE;
  if (is_csc(prob)) {
    rc = run_csc(prob, 1, opts, workspace, ws_bytes, s);
    if (rc) return rc;
    std::vector<int32_t> st(prob->T);
    HIPCHK(hipMemcpyAsync(st.data(), prob->status_out, sizeof(int32_t) * prob->T,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int32_t v : st)
      if (v == GS_STATUS_NOT_CONVERGED) return GS_NOT_CONVERGED;
    return GS_OK;
  }
  if (use_wide(prob, opts)) {
    Carver cv{static_cast<char*>(workspace)};
    Shared sh;
    carve_shared(cv, 1, prob->p, &sh);
    ProbDesc d;
    fill_desc(prob, 0, &d);
    carve_problem(cv, prob, &d);
    rc = upload_lambdas(prob, &d, s);
    if (rc) return rc;
    return run_wide(prob, opts, sh, d, s);
  }
  Shared sh;
  std::vector<Group> groups;
  rc = prepare_batch(prob, 1, opts, workspace, ws_bytes, s, &sh, &groups);
  if (rc) return rc;
  rc = launch_groups(sh, groups, path_opts(opts, false), s);
  if (rc) return rc;
  // the path is done when its status words are on the host: a lambda that
  // reached max_epochs makes the call report GS_NOT_CONVERGED
  std::vector<int32_t> st(prob->T);
  HIPCHK(hipMemcpyAsync(st.data(), prob->status_out, sizeof(int32_t) * prob->T,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int32_t v : st)
    if (v == GS_STATUS_NOT_CONVERGED) return GS_NOT_CONVERGED;
  return GS_OK;
}

int lasso_solve_batch(const gs_problem* probs, int32_t B, const gs_opts* opts, void* workspace,
                      size_t ws_bytes, void* stream) {
  gs_opts def;
  gs_opts_default(&def);
  if (!opts) opts = &def;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (probs && B >= 1 && is_csc(&probs[0])) {
    int rc = check_opts(opts);
    if (rc) return rc;
    for (int b = 0; b < B; ++b) {
      rc = check_problem(&probs[b]);
      if (rc) return rc;
      if (opts->select_counts && (probs[b].p != probs[0].p || probs[b].T != probs[0].T))
        return GS_EINVAL;
    }
    return run_csc(probs, B, opts, workspace, ws_bytes, s);
  }
  Shared sh;
  std::vector<Group> groups;
  int rc = prepare_batch(probs, B, opts, workspace, ws_bytes, s, &sh, &groups);
  if (rc) return rc;
  return launch_groups(sh, groups, path_opts(opts, true), s);
}

size_t screen_workspace_size(int32_t n, int32_t p) {
  if (n < 1 || p < 1) return 0;
  Carver cv{nullptr};
  Shared sh;
  ProbDesc d{};
  carve_screen(cv, n, p, &sh, &d);
  return align_up(cv.off, 256);
}

int screen(int32_t n, int32_t p, int64_t ldx, int32_t dtype, const void* X, const void* y,
           const double* beta, double lambda, int32_t rule, const int32_t* active_in,
           int32_t q_in, int32_t* active_out, int32_t* q_out, double* gap_out,
           double* alpha_out, double* radius_out, double* c_out, void* workspace,
           size_t ws_bytes, void* stream) {
  const int rc = check_screen(n, p, ldx, dtype, X, y, beta, lambda, rule, active_in, q_in,
                              active_out, q_out, gap_out, alpha_out, radius_out);
  if (rc) return rc;
  if (!workspace) return GS_EWORKSPACE;
  if (ws_bytes < screen_workspace_size(n, p)) return GS_EWORKSPACE;
  return run_screen(n, p, ldx, dtype, X, y, beta, lambda, rule, active_in, q_in, active_out, q_out,
                    gap_out, alpha_out, radius_out, c_out, static_cast<char*>(workspace),
                    static_cast<hipStream_t>(stream));
}

int screen_noalloc(int32_t n, int32_t p, int64_t ldx, int32_t dtype, const void* X,
                   const void* y, const double* beta, double lambda, int32_t rule,
                   const int32_t* active_in, int32_t q_in, int32_t* active_out,
                   int32_t* q_out, double* gap_out, double* alpha_out, double* radius_out,
                   double* c_out, void* stream) {
  const int rc = check_screen(n, p, ldx, dtype, X, y, beta, lambda, rule, active_in, q_in,
                              active_out, q_out, gap_out, alpha_out, radius_out);
  if (rc) return rc;
  if (screen_workspace_size(n, p) > (size_t)GS_NOALLOC_SCRATCH_BYTES) return GS_ETOOLARGE;
  char* base = nullptr;
  const int r2 = scratch_base(&base);
  if (r2) return r2;
  return run_screen(n, p, ldx, dtype, X, y, beta, lambda, rule, active_in, q_in, active_out, q_out,
                    gap_out, alpha_out, radius_out, c_out, base,
                    static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------ batch plans

struct gs_batch_plan {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int lasso_batch_plan(const gs_problem* probs, int32_t B, const gs_opts* opts, void* workspace,
                     size_t ws_bytes, void* stream, gs_batch_plan** plan) {
  if (!plan) return GS_EINVAL;
  *plan = nullptr;
  gs_opts def;
  gs_opts_default(&def);
  if (!opts) opts = &def;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Shared sh;
  std::vector<Group> groups;
  int rc = prepare_batch(probs, B, opts, workspace, ws_bytes, s, &sh, &groups);
  if (rc) return rc;
  std::vector<Launch> launches;
  rc = configure_groups(sh, groups, path_opts(opts, true), &launches);
  if (rc) return rc;
  // the uploads above are ordered before every replay on `stream`; capture
  // the launches on a private stream
  HIPCHK(hipStreamSynchronize(s));
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  gs_batch_plan* p = new gs_batch_plan;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = enqueue_groups(sh, launches, cs, false);
    hipError_t e2 = hipStreamEndCapture(cs, &p->graph);
    if (rc == GS_OK && e2 != hipSuccess) rc = fail_hip(e2, "hipStreamEndCapture");
  } else {
    rc = fail_hip(e, "hipStreamBeginCapture");
  }
  if (rc == GS_OK) {
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = fail_hip(e, "hipGraphInstantiate");
  }
  (void)hipStreamDestroy(cs);
  if (rc != GS_OK) {
    lasso_batch_plan_free(p);
    return rc;
  }
  *plan = p;
  return GS_OK;
}

int lasso_batch_run(gs_batch_plan* plan, void* stream) {
  if (!plan || !plan->exec) return GS_EINVAL;
  HIPCHK(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
  return GS_OK;
}

void lasso_batch_plan_free(gs_batch_plan* plan) {
  if (!plan) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
}

// --------------------------------------------------------------- autotuner

int gs_autotune(const gs_problem* probs, int32_t B, const gs_opts* opts, void* workspace,
                size_t ws_bytes, void* stream, int32_t max_lambdas, int32_t sample,
                int32_t* choice_out) {
  gs_opts def;
  gs_opts_default(&def);
  if (!opts) opts = &def;
  if (!probs || B < 1 || max_lambdas < 1 || sample < 1) return GS_EINVAL;
  int rc = check_opts(opts);
  if (rc) return rc;
  for (int b = 0; b < B; ++b) {
    rc = check_problem(&probs[b]);
    if (rc) return rc;
  }
  if (!workspace) return GS_EWORKSPACE;
  if (ws_bytes < path_ws(probs, B)) return GS_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  gs_opts o = *opts;
  o.select_counts = nullptr;
  o.timestamps = nullptr;
  o.stats = nullptr;
  // classes present in the batch
  std::map<std::pair<const NarrowEntry*, int>, std::vector<int>> classes;
  for (int b = 0; b < B; ++b) {
    int cnt = 0;
    const NarrowEntry* tab = narrow_table(probs[b].dtype, probs[b].rows != nullptr,
                                          vec_ok(&probs[b]), &cnt);
    const int i0 = smallest_fit(tab, cnt, probs[b].n);
    if (i0 < 0) return GS_EUNSUPPORTED;
    classes[{tab, i0}].push_back(b);
  }
  hipEvent_t ea = nullptr, eb = nullptr;
  HIPCHK(hipEventCreate(&ea));
  HIPCHK(hipEventCreate(&eb));
  for (auto& kv : classes) {
    const NarrowEntry* tab = kv.first.first;
    const int i0 = kv.first.second;
    int cnt = 0;
    narrow_table(probs[kv.second[0]].dtype, probs[kv.second[0]].rows != nullptr,
                 vec_ok(&probs[kv.second[0]]), &cnt);
    std::vector<int> mem = kv.second;
    std::stable_sort(mem.begin(), mem.end(), [&](int a, int b) {
      return (double)probs[a].n * probs[a].p > (double)probs[b].n * probs[b].p;
    });
    if ((int)mem.size() > sample) mem.resize(sample);
    int nmax = 0;
    for (int b : mem) nmax = std::max(nmax, probs[b].n);
    std::vector<gs_problem> sp;
    for (int b : mem) {
      gs_problem q = probs[b];
      first_lambdas(&q, max_lambdas);
      sp.push_back(q);
    }
    // candidates: the smallest entry of each lane split S that holds the class
    std::vector<int> cand;
    std::vector<int> seenS;
    for (int i = i0; i < cnt; ++i) {
      if (tab[i].cfg.nmax() < nmax) continue;
      if (std::find(seenS.begin(), seenS.end(), tab[i].cfg.S) != seenS.end()) continue;
      seenS.push_back(tab[i].cfg.S);
      cand.push_back(i);
    }
    int best = i0;
    float best_ms = 1e30f;
    for (int c : cand) {
      g_force = &tab[c];
      float ms = 0.f;
      for (int rep = 0; rep < 2 && rc == GS_OK; ++rep) {  // the first run loads the code
        Shared sh;
        std::vector<Group> groups;
        rc = prepare_batch(sp.data(), (int)sp.size(), &o, workspace, ws_bytes, s, &sh, &groups);
        std::vector<Launch> launches;
        if (rc == GS_OK) rc = configure_groups(sh, groups, path_opts(&o, true), &launches);
        if (rc == GS_OK && hipEventRecord(ea, s) != hipSuccess) rc = GS_EHIP;
        if (rc == GS_OK) rc = enqueue_groups(sh, launches, s, false);
        if (rc == GS_OK && hipEventRecord(eb, s) != hipSuccess) rc = GS_EHIP;
        if (rc == GS_OK && hipEventSynchronize(eb) != hipSuccess) rc = GS_EHIP;
        if (rc == GS_OK && hipEventElapsedTime(&ms, ea, eb) != hipSuccess) rc = GS_EHIP;
      }
      g_force = nullptr;
      if (rc) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    if (rc) break;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tuned[kv.first] = best;
    }
    if (choice_out)
      for (int b : kv.second) {
        choice_out[2 * b] = tab[best].cfg.S;
        choice_out[2 * b + 1] = tab[best].cfg.NG;
      }
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  return rc;
}

int gs_autotune_schedule(const gs_problem* prob, const gs_opts* opts, void* workspace,
                         size_t ws_bytes, void* stream, int32_t max_lambdas,
                         int32_t* choice_out) {
  gs_opts def;
  gs_opts_default(&def);
  if (!opts) opts = &def;
  if (!prob || max_lambdas < 1) return GS_EINVAL;
  int rc = check_opts(opts);
  if (rc) return rc;
  rc = check_problem(prob);
  if (rc) return rc;
  if (prob->rows || is_csc(prob) || opts->rule >= GS_RULE_STATIC ||
      (opts->enet_alpha != 0.0 && opts->enet_alpha < 1.0))
    return GS_EUNSUPPORTED;  // one schedule only: nothing to choose
  if (!workspace) return GS_EWORKSPACE;
  if (ws_bytes < path_ws(prob, 1)) return GS_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  gs_problem q = *prob;
  first_lambdas(&q, max_lambdas);
  gs_opts o = *opts;
  o.select_counts = nullptr;
  o.timestamps = nullptr;
  o.stats = nullptr;
  float ms[2] = {0.f, 0.f};
  hipEvent_t ea = nullptr, eb = nullptr;
  HIPCHK(hipEventCreate(&ea));
  HIPCHK(hipEventCreate(&eb));
  for (int w = 0; w < 2 && rc >= 0; ++w) {
    o.schedule = w ? GS_SCHED_WIDE : GS_SCHED_NARROW;
    for (int rep = 0; rep < 2 && rc >= 0; ++rep) {  // the first run loads the code
      if (hipEventRecord(ea, s) != hipSuccess) rc = GS_EHIP;
      if (rc >= 0) rc = lasso_path(&q, &o, workspace, ws_bytes, stream);
      if (rc >= 0 && hipEventRecord(eb, s) != hipSuccess) rc = GS_EHIP;
      if (rc >= 0 && hipEventSynchronize(eb) != hipSuccess) rc = GS_EHIP;
      if (rc >= 0 && hipEventElapsedTime(&ms[w], ea, eb) != hipSuccess) rc = GS_EHIP;
    }
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  if (rc < 0) return rc;
  const bool wide = ms[1] < ms[0];
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int k = prob->dtype == GS_F64 ? 1 : 0;
    g_sched_pts[k].push_back({(double)prob->n * (double)prob->p, wide});
    g_wide_thr[k] = fit_threshold(g_sched_pts[k]);
  }
  if (choice_out) *choice_out = wide ? 1 : 0;
  return GS_OK;
}

double gs_wide_threshold(int32_t dtype) {
  if (dtype != GS_F32 && dtype != GS_F64) return -1.0;
  return wide_threshold(dtype);
}

void gs_tune_reset(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
  for (int k = 0; k < 2; ++k) {
    g_sched_pts[k].clear();
    g_wide_thr[k] = kWideThreshold;
  }
}

int gs_tune_save(const char* path) {
  if (!path) return GS_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) return GS_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::fprintf(f, "{\"tiles\": [");
  bool first = true;
  for (auto& kv : g_tuned) {
    const NarrowEntry& a = kv.first.first[kv.first.second];
    const NarrowEntry& c = kv.first.first[kv.second];
    std::fprintf(f, "%s\n  {\"dtype\": %d, \"vec\": %d, \"gather\": %d, \"S\": %d, \"NG\": %d, "
                 "\"to_S\": %d, \"to_NG\": %d}",
                 first ? "" : ",", a.cfg.dtype, a.cfg.vec, a.cfg.gather ? 1 : 0, a.cfg.S, a.cfg.NG,
                 c.cfg.S, c.cfg.NG);
    first = false;
  }
  std::fprintf(f, "\n], \"schedule\": [");
  for (int k = 0; k < 2; ++k)
    std::fprintf(f, "%s\n  {\"sched_dtype\": %d, \"wide_threshold\": %.17g}", k ? "," : "", k,
                 g_wide_thr[k]);
  std::fprintf(f, "\n]}\n");
  std::fclose(f);
  return GS_OK;
}

int gs_tune_load(const char* path) {
  if (!path) return GS_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return GS_EINVAL;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
  std::fclose(f);
  // one object per line of the form written by gs_tune_save
  int loaded = 0;
  size_t pos = 0;
  while ((pos = text.find("{\"dtype\"", pos)) != std::string::npos) {
    int dt, vec, ga, S, NG, tS, tNG;
    if (std::sscanf(text.c_str() + pos,
                    "{\"dtype\": %d, \"vec\": %d, \"gather\": %d, \"S\": %d, \"NG\": %d, "
                    "\"to_S\": %d, \"to_NG\": %d}",
                    &dt, &vec, &ga, &S, &NG, &tS, &tNG) == 7) {
      int cnt = 0;
      const bool vok = vec > 1;
      const NarrowEntry* tab = narrow_table(dt == 1 ? GS_F64 : GS_F32, ga != 0, vok, &cnt);
      int from = -1, to = -1;
      for (int i = 0; i < cnt; ++i) {
        if (tab[i].cfg.S == S && tab[i].cfg.NG == NG) from = i;
        if (tab[i].cfg.S == tS && tab[i].cfg.NG == tNG) to = i;
      }
      if (from >= 0 && to >= 0 && tab[to].cfg.nmax() >= tab[from].cfg.nmax()) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[{tab, from}] = to;
        ++loaded;
      }
    }
    pos += 8;
  }
  pos = 0;
  while ((pos = text.find("{\"sched_dtype\"", pos)) != std::string::npos) {
    int k;
    double thr;
    if (std::sscanf(text.c_str() + pos, "{\"sched_dtype\": %d, \"wide_threshold\": %lf}", &k,
                    &thr) == 2 &&
        (k == 0 || k == 1) && thr > 0.0 && std::isfinite(thr)) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_wide_thr[k] = thr;
      ++loaded;
    }
    pos += 14;
  }
  return loaded > 0 ? GS_OK : GS_EINVAL;
}

void gs_timing_enable(int on) { g_timing = on != 0; }

void gs_timing_reset(void) {
  resolve_timing();
  for (int i = 0; i < 3; ++i) {
    g_total_ms[i] = 0.0;
    g_launches[i] = 0;
  }
}

int gs_timing_query(const char* kernel, double* total_ms, int64_t* launches) {
  if (!kernel) return -1;
  int slot = -1;
  if (std::strcmp(kernel, "sweep") == 0) slot = kTimeSweep;
  if (std::strcmp(kernel, "path") == 0) slot = kTimePath;
  if (std::strcmp(kernel, "cd") == 0) slot = kTimeCD;
  if (slot < 0) return -1;
  resolve_timing();
  if (total_ms) *total_ms = g_total_ms[slot];
  if (launches) *launches = g_launches[slot];
  return 0;
}

const char* lasso_strerror(int code) {
  switch (code) {
    case GS_OK: return "ok";
    case GS_NOT_CONVERGED: return "not converged: max_epochs reached for some lambda";
    case GS_EINVAL: return "invalid argument";
    case GS_EHIP: return g_err.empty() ? "HIP runtime error" : g_err.c_str();
    case GS_EWORKSPACE: return "workspace missing or too small";
    case GS_EUNSUPPORTED: return "unsupported: n larger than 2048";
    case GS_ETOOLARGE:
      return "input larger than the static scratch of the allocation-free entry point "
             "(GS_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown error code";
  }
}

}  // extern "C"
