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
// Whether column j with c = x_j^T rho (norm^2 nrm2, x_j^T y xy, x_j^T x_{j*}
// gsv where the rule uses them) passes the active test.
__device__ __forceinline__ bool keep_vals(const ProbDesc& d, const WideState* st,
                                          const GapInfo& g, double nrm2, double c, double xy,
                                          double gsv) {
  if (!(nrm2 > 0.0)) return false;
  const double nr = nrm2 + wide_mu2(d, st);  // ||x~_j||^2 (elastic net)
  const int nn = wide_nn(d, st);
  if (g.rule >= 2) return rule_keep(g, xy, g.rule == 4 ? gsv : 0.0, nr, nn);
  return sphere_keep(g, c, nr, nn) && (!g.dome || dome_keep(g, xy, c, nr, nn));
}

// Keep bits of the PER consecutive positions k0.. of A (positions >= q are
// not kept) and their columns js.  Positions are clamped to q-1 so that
// every load is issued, without branches, before the first test; q >= 1.
template <int PER>
__device__ __forceinline__ unsigned keep_bits(const ProbDesc& d, const WideState* st,
                                              const GapInfo& g, const int32_t* act, bool full,
                                              int q, int k0, int (&js)[PER]) {
  double cs[PER], nr[PER], xy[PER], gv[PER];
  const bool need_xy = g.dome || g.rule >= 2;
  const bool need_g = g.rule == 4;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int k = max(0, min(k0 + e, q - 1));
    const int ak = act[k];
    js[e] = full ? k : ak;
    cs[e] = d.c[k];
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    nr[e] = d.nrm2[js[e]];
    xy[e] = need_xy ? d.xty[js[e]] : 0.0;
    gv[e] = need_g ? d.gst[js[e]] : 0.0;
  }
  unsigned keep = 0;
#pragma unroll
  for (int e = 0; e < PER; ++e)
    if (k0 + e < q && keep_vals(d, st, g, nr[e], cs[e], xy[e], gv[e])) keep |= 1u << e;
  return keep;
}

// Sphere test over one tile of A: kept count per block; screened nonzero
// coefficients are set to zero and flagged for a residual refresh.  Thread
// t owns 8 consecutive positions of the tile.
__global__ __launch_bounds__(256) void k_wide_test(ProbDesc d, WideState* st, WideBufs wb) {
  constexpr int PER = kTestTile / 256;
  __shared__ double sh[256];
  if (st->done || st->phase != 1) return;
  const int q = st->q;
  if (q <= 0) {  // an empty A: no entry of act is valid
    if (threadIdx.x == 0) wb.cnt[blockIdx.x] = 0;
    return;
  }
  const bool full = st->full != 0;
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  const GapInfo g = state_gap(d, st);
  const int k0 = blockIdx.x * kTestTile + threadIdx.x * PER;
  int js[PER];
  const unsigned keep = keep_bits<PER>(d, st, g, act, full, q, k0, js);
  double bz[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) bz[e] = d.beta[js[e]];
  bool dn = false;
#pragma unroll
  for (int e = 0; e < PER; ++e)
    if (k0 + e < q && !((keep >> e) & 1u) && bz[e] != 0.0) {
      d.beta[js[e]] = 0.0;
      dn = true;
    }
  if (dn) st->need_refresh = 1;
  const double tot = block_sum<256>((double)__popc(keep), sh);
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
  if (q <= 0) return;  // an empty A: nothing kept, no entry of act is valid
  const bool full = st->full != 0;
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  int32_t* dst = out ? out : d.act + (int64_t)(st->cur ^ 1) * d.p;
  const GapInfo g = state_gap(d, st);
  int off = 0;
  for (int b = 0; b < (int)blockIdx.x; ++b) off += wb.cnt[b];
  const int k0 = blockIdx.x * kTestTile + threadIdx.x * PER;
  int js[PER];
  const unsigned keep = keep_bits<PER>(d, st, g, act, full, q, k0, js);
  const int c = __popc(keep);
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

// List bits of the PER consecutive positions k0.. (positions >= q are not
// listed), their columns js, c_k, beta_j and ||x_j||^2; positions are clamped
// to q-1 so that every load is issued, without branches, before the first
// test; q >= 1.
template <int PER>
__device__ __forceinline__ unsigned listed_bits(const ProbDesc& d, const WideState* st,
                                                const int32_t* act, int q, int k0,
                                                int (&js)[PER], double (&cs)[PER],
                                                double (&bs)[PER], double (&ns)[PER]) {
  const double lambda = wide_l1(d, st);
  const double tau = st->tau;
  const double rn = sqrt(st->R2) * (1.0 + gam(wide_nn(d, st) + 2));
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int k = max(0, min(k0 + e, q - 1));
    js[e] = act[k];
    cs[e] = d.c[k];
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    ns[e] = d.nrm2[js[e]];
    bs[e] = d.beta[js[e]];
  }
  unsigned keep = 0;
#pragma unroll
  for (int e = 0; e < PER; ++e)
    if (k0 + e < q && wide_listed(d, st, ns[e], bs[e], cs[e], lambda, tau, rn)) keep |= 1u << e;
  return keep;
}

__global__ __launch_bounds__(256) void k_wide_lcount(ProbDesc d, WideState* st, WideBufs wb) {
  constexpr int PER = kTestTile / 256;
  __shared__ double sh[256];
  if (st->done || st->phase != 2) return;
  const int q = st->q;
  if (q <= 0) {  // an empty A: no entry of act is valid
    if (threadIdx.x == 0) wb.cnt[blockIdx.x] = 0;
    return;
  }
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  const int k0 = st->resume + blockIdx.x * kTestTile + threadIdx.x * PER;
  int js[PER];
  double cs[PER], bs[PER], ns[PER];
  const unsigned keep = listed_bits<PER>(d, st, act, q, k0, js, cs, bs, ns);
  const double tot = block_sum<256>((double)__popc(keep), sh);
  if (threadIdx.x == 0) wb.cnt[blockIdx.x] = (int)tot;
}

__global__ __launch_bounds__(256) void k_wide_lcompact(ProbDesc d, WideState* st, WideBufs wb) {
  constexpr int PER = kTestTile / 256;
  __shared__ int scan[256];
  if (st->done || st->phase != 2) return;
  const int q = st->q;
  if (q <= 0) return;  // an empty A lists nothing
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  int off = 0;
  for (int b = 0; b < (int)blockIdx.x; ++b) off += wb.cnt[b];
  const int k0 = st->resume + blockIdx.x * kTestTile + threadIdx.x * PER;
  int js[PER];
  double cs[PER], bs[PER], ns[PER];
  const unsigned keep = listed_bits<PER>(d, st, act, q, k0, js, cs, bs, ns);
  const int c = __popc(keep);
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
      v[0] = cs[e];
      v[1] = bs[e];
      if (mu2 > 0.0) {  // elastic net: ||x~_j||^2
        const double nr = ns[e] + mu2;
        v[2] = 1.0 / nr;
        v[3] = nr;
      } else {
        v[2] = d.inv[j];
        v[3] = ns[e];
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
  // all blocks copy beta and the active list; block 0 also sets the state
  const int g = blockIdx.x * 256 + threadIdx.x, G = gridDim.x * 256;
  for (int j = g; j < d.p; j += G) d.beta[j] = beta_in[j];
  if (active_in)
    for (int k = g; k < q_in; k += G) d.act[k] = active_in[k];
  if (blockIdx.x != 0) return;
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
