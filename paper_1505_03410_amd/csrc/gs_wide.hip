// Non-template kernels of the wide schedule and of screen(), plus the table
// of wide sweep instantiations.
#include "gs_registry.hpp"
#include "gs_wide.hpp"

namespace gs {

__device__ __forceinline__ GapInfo state_gap(const ProbDesc& d, const WideState* st) {
  GapInfo g;
  g.alpha = st->alpha_s;
  g.gap = st->gap;
  g.radius = st->radius_s;
  g.e_c = st->e_c;
  g.lambda = wide_l1(d, st);
  g.Rlo = st->Rlo;
  g.Rhi = st->Rhi;
  g.rc2lo = st->rc2lo;
  g.e_y = st->e_y;
  g.dome = st->rule == 1;
  g.rule = st->rule;
  g.shift = st->shift;
  g.rad_s = st->rad_s;
  g.e_shift = st->e_shift;
  g.nstar = st->nstar;
  return g;
}

// The GAP SAFE sphere test, and the dome test where it is on (each is safe
// alone); or one of the comparison rules of Table 1 in their place.
__device__ __forceinline__ bool wide_keep(const ProbDesc& d, const WideState* st,
                                          const GapInfo& g, int j, double c) {
  if (!(d.nrm2[j] > 0.0)) return false;
  const double nr = d.nrm2[j] + wide_mu2(d, st);  // ||x~_j||^2 (elastic net)
  const int nn = wide_nn(d, st);
  if (g.rule >= 2) return rule_keep(g, d.xty[j], g.rule == 4 ? d.gst[j] : 0.0, nr, nn);
  return sphere_keep(g, c, nr, nn) && (!g.dome || dome_keep(g, d.xty[j], c, nr, nn));
}

// Sphere test over one tile of A: kept count per block; screened nonzero
// coefficients are set to zero and flagged for a residual refresh.
__global__ __launch_bounds__(256) void k_wide_test(ProbDesc d, WideState* st, WideBufs wb) {
  __shared__ double sh[256];
  if (st->done || st->phase != 1) return;
  const int q = st->q;
  const bool full = st->full != 0;
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  const GapInfo g = state_gap(d, st);
  const int tile0 = blockIdx.x * kTestTile;
  int cnt = 0;
  bool dn = false;
  for (int e = threadIdx.x; e < kTestTile; e += 256) {
    const int k = tile0 + e;
    if (k >= q) break;
    const int j = full ? k : act[k];
    if (wide_keep(d, st, g, j, d.c[k])) {
      ++cnt;
    } else if (d.beta[j] != 0.0) {
      d.beta[j] = 0.0;
      dn = true;
    }
  }
  if (dn) st->need_refresh = 1;
  const double tot = block_sum<256>((double)cnt, sh);
  if (threadIdx.x == 0) wb.cnt[blockIdx.x] = (int)tot;
}

// Ordered compaction: block b writes its kept indices after those of blocks
// 0..b-1.  Thread t owns 8 consecutive positions of the tile.
__global__ __launch_bounds__(256) void k_wide_compact(ProbDesc d, WideState* st, WideBufs wb,
                                                      int32_t* out) {
  constexpr int PER = kTestTile / 256;
  __shared__ int scan[256];
  if (st->done || st->phase != 1) return;
  const int q = st->q;
  const bool full = st->full != 0;
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  int32_t* dst = out ? out : d.act + (int64_t)(st->cur ^ 1) * d.p;
  const GapInfo g = state_gap(d, st);
  int off = 0;
  for (int b = 0; b < (int)blockIdx.x; ++b) off += wb.cnt[b];
  const int k0 = blockIdx.x * kTestTile + threadIdx.x * PER;
  int js[PER];
  unsigned keep = 0;
  int c = 0;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int k = k0 + e;
    js[e] = -1;
    if (k < q) {
      const int j = full ? k : act[k];
      js[e] = j;
      if (wide_keep(d, st, g, j, d.c[k])) {
        keep |= 1u << e;
        ++c;
      }
    }
  }
  scan[threadIdx.x] = c;
  __syncthreads();
  // Hillis-Steele inclusive scan over 256 counts.
  for (int o = 1; o < 256; o <<= 1) {
    int v = (int)threadIdx.x >= o ? scan[threadIdx.x - o] : 0;
    __syncthreads();
    scan[threadIdx.x] += v;
    __syncthreads();
  }
  int pos = off + scan[threadIdx.x] - c;
#pragma unroll
  for (int e = 0; e < PER; ++e)
    if (keep & (1u << e)) dst[pos++] = js[e];
}

__global__ __launch_bounds__(256) void k_wide_lcount(ProbDesc d, WideState* st, WideBufs wb) {
  __shared__ double sh[256];
  if (st->done || st->phase != 2) return;
  const int q = st->q;
  const int tile0 = st->resume + blockIdx.x * kTestTile;
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  const double lambda = wide_l1(d, st);
  const double tau = st->tau;
  const double rn = sqrt(st->R2) * (1.0 + gam(wide_nn(d, st) + 2));
  int cnt = 0;
  for (int e = threadIdx.x; e < kTestTile; e += 256) {
    const int k = tile0 + e;
    if (k >= q) break;
    if (wide_listed(d, st, act[k], d.c[k], lambda, tau, rn)) ++cnt;
  }
  const double tot = block_sum<256>((double)cnt, sh);
  if (threadIdx.x == 0) wb.cnt[blockIdx.x] = (int)tot;
}

__global__ __launch_bounds__(256) void k_wide_lcompact(ProbDesc d, WideState* st, WideBufs wb) {
  constexpr int PER = kTestTile / 256;
  __shared__ int scan[256];
  if (st->done || st->phase != 2) return;
  const int q = st->q;
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  const double lambda = wide_l1(d, st);
  const double tau = st->tau;
  const double rn = sqrt(st->R2) * (1.0 + gam(wide_nn(d, st) + 2));
  int off = 0;
  for (int b = 0; b < (int)blockIdx.x; ++b) off += wb.cnt[b];
  const int k0 = st->resume + blockIdx.x * kTestTile + threadIdx.x * PER;
  unsigned keep = 0;
  int c = 0;
  int js[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int k = k0 + e;
    js[e] = k < q ? act[k] : 0;
    if (k < q && wide_listed(d, st, js[e], d.c[k], lambda, tau, rn)) {
      keep |= 1u << e;
      ++c;
    }
  }
  scan[threadIdx.x] = c;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int v = (int)threadIdx.x >= o ? scan[threadIdx.x - o] : 0;
    __syncthreads();
    scan[threadIdx.x] += v;
    __syncthreads();
  }
  int pos = off + scan[threadIdx.x] - c;
  const double mu2 = wide_mu2(d, st);
  // entry: position, feature, then (c_k, beta_j, 1/||x_j||^2, ||x_j||^2)
#pragma unroll
  for (int e = 0; e < PER; ++e)
    if (keep & (1u << e)) {
      const int j = js[e];
      d.lst[pos] = k0 + e;
      d.lst[d.p + pos] = j;
      double* v = d.lval + 4 * (int64_t)pos;
      v[0] = d.c[k0 + e];
      v[1] = d.beta[j];
      if (mu2 > 0.0) {  // elastic net: ||x~_j||^2
        const double nr = d.nrm2[j] + mu2;
        v[2] = 1.0 / nr;
        v[3] = nr;
      } else {
        v[2] = d.inv[j];
        v[3] = d.nrm2[j];
      }
      ++pos;
    }
}

__global__ __launch_bounds__(64) void k_wide_fin(ProbDesc d, WideState* st, WideBufs wb,
                                                 int ntest, int32_t* q_out) {
  if (st->done || st->phase != 1) return;
  int s = 0;
  for (int b = threadIdx.x; b < ntest; b += 64) s += wb.cnt[b];
  s = wave_sum_i(s);
  if (threadIdx.x == 0) {
    if (q_out) {
      *q_out = s;
      st->phase = 0;
    } else {
      st->q = s;
      st->cur ^= 1;
      st->full = 0;
      st->phase = 2;
      st->resume = 0;
      st->dmax2 = 0.0;
      if (st->first_epoch) st->tau = st->tau_first;
    }
  }
}

// Adds the wide path's counters to the caller's gs_opts.stats.
__global__ void k_wide_stats(const WideState* st, long long* stats) {
  if (threadIdx.x != 0 || !stats) return;
  unsigned long long* s = reinterpret_cast<unsigned long long*>(stats);
  atomicAdd(&s[kStatPasses], (unsigned long long)st->passes);
  atomicAdd(&s[kStatResidualEpochs], (unsigned long long)st->n_epochs);
  atomicAdd(&s[kStatWideVisits], (unsigned long long)st->n_visits);
  atomicAdd(&s[kStatWideRounds], (unsigned long long)st->n_rounds);
  atomicAdd(&s[kStatWideStops], (unsigned long long)st->n_stops);
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// screen(): beta to FP64, the active list, ||y||^2 and the state.
template <typename XT>
__global__ __launch_bounds__(256) void k_screen_prep(ProbDesc d, WideState* st,
                                                     const double* beta_in,
                                                     const int32_t* active_in, int q_in,
                                                     double lambda, int rule) {
  __shared__ double sh[256];
  for (int j = threadIdx.x; j < d.p; j += 256) d.beta[j] = beta_in[j];
  if (active_in)
    for (int k = threadIdx.x; k < q_in; k += 256) d.act[k] = active_in[k];
  const XT* Y = (const XT*)d.y;
  double yy = 0.0;
  for (int i = threadIdx.x; i < d.n; i += 256) {
    double v = (double)Y[i];
    yy = fma(v, v, yy);
  }
  yy = block_sum<256>(yy, sh);
  if (threadIdx.x == 0) {
    d.lam[0] = lambda;
    st->ynorm2 = yy;
    st->eps = 0.0;
    st->t = 0;
    st->k = 0;
    st->q = q_in;
    st->full = active_in ? 0 : 1;
    st->cur = 0;
    st->done = 0;
    st->phase = 0;
    st->need_refresh = 0;
    st->rule = rule;
    st->enet = 1.0;
  }
}

const void* const kWideInit[2] = {reinterpret_cast<const void*>(&k_wide_init<float>),
                                  reinterpret_cast<const void*>(&k_wide_init<double>)};
const void* const kWideRefresh[2] = {reinterpret_cast<const void*>(&k_wide_refresh<float>),
                                     reinterpret_cast<const void*>(&k_wide_refresh<double>)};
const void* const kWideGap[2] = {reinterpret_cast<const void*>(&k_wide_gap<float>),
                                 reinterpret_cast<const void*>(&k_wide_gap<double>)};
const void* const kScreenPrep[2] = {reinterpret_cast<const void*>(&k_screen_prep<float>),
                                    reinterpret_cast<const void*>(&k_screen_prep<double>)};
const void* const kWideTest = reinterpret_cast<const void*>(&k_wide_test);
const void* const kWideCompact = reinterpret_cast<const void*>(&k_wide_compact);
const void* const kWideFin = reinterpret_cast<const void*>(&k_wide_fin);
const void* const kFillI32 = reinterpret_cast<const void*>(&k_fill_i32);
const void* const kWideLCount = reinterpret_cast<const void*>(&k_wide_lcount);
const void* const kWideLCompact = reinterpret_cast<const void*>(&k_wide_lcompact);
const void* const kWideStats = reinterpret_cast<const void*>(&k_wide_stats);

#define GS_WIDE_ENTRY(XT, VEC, NG)                                              \
  {                                                                             \
    sizeof(XT) == 8 ? 1 : 0, VEC, NG,                                           \
        reinterpret_cast<const void*>(&k_wide_pre<XT, VEC, NG>),                \
        reinterpret_cast<const void*>(&k_wide_sweep<XT, VEC, NG, 0>),           \
        reinterpret_cast<const void*>(&k_wide_sweep<XT, VEC, NG, 1>),           \
        reinterpret_cast<const void*>(&k_wide_sweep<XT, VEC, NG, 2>),           \
        reinterpret_cast<const void*>(&k_wide_csweep<XT, VEC, NG>),             \
        reinterpret_cast<const void*>(&k_wide_gstar<XT, VEC, NG>),              \
        reinterpret_cast<const void*>(&k_wide_walk<XT, VEC, NG>)                \
  }

// Ordered by dtype, vector width, then capacity (64 * NG * VEC rows).
const WideEntry kWide[] = {
    GS_WIDE_ENTRY(float, 4, 2),  GS_WIDE_ENTRY(float, 4, 4),   GS_WIDE_ENTRY(float, 4, 8),
    GS_WIDE_ENTRY(float, 1, 8),  GS_WIDE_ENTRY(float, 1, 32),  GS_WIDE_ENTRY(double, 2, 4),
    GS_WIDE_ENTRY(double, 2, 16), GS_WIDE_ENTRY(double, 1, 8), GS_WIDE_ENTRY(double, 1, 32),
};
const int kWideN = sizeof(kWide) / sizeof(kWide[0]);

}  // namespace gs
