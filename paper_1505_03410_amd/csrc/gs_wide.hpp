// The wide schedule: one Lasso path whose screening passes use the whole GPU.
// A pass is a chain of kernels that read the state machine in the workspace
// (WideState), so the host only enqueues passes and polls `done`:
//
//   refresh (1 block)  rho = y - X_S beta_S, ||rho||^2, y^T rho
//   sweep   (grid)     c_k = x_{A[k]}^T rho, per-block max|c|, sums
//   gap     (1 block)  alpha, G, radius; stop test; record beta^{lambda_t}
//   test    (grid)     sphere test, per-block kept counts, zero dropped beta
//   compact (grid)     ordered compaction of A into the other buffer
//   fin     (1 block)  |A'|, swap buffers
//   refresh (1 block)  again only if a nonzero coefficient was screened
//   f CD rounds        csweep (grid), lcount + lcompact (grid), walk (1 wave):
//                      one epoch each, see the CD rounds below
//
// Every reduction goes through per-block partials reduced in a fixed order,
// so results are bitwise reproducible.
#pragma once

#include "gs_device.hpp"

namespace gs {

constexpr int kSweepWaves = 4;      // waves per sweep block
// Columns in flight per wave of the sweep.  Two keep the 1000-row FP32
// layout at 4 waves per SIMD without spills (about 110 VGPRs); four need
// about 150 VGPRs (3 waves per SIMD) and measured about 5% slower on the
// 1000 x 100000 sweep.
#ifndef GS_SWEEP_U
#define GS_SWEEP_U 2
#endif
constexpr int kSweepU = GS_SWEEP_U;
constexpr int kTestTile = 2048;     // entries per test/compact block
constexpr int kRefreshThreads = 1024;
constexpr int kRefreshBatch = 8;    // rows of 64 positions per refresh scan step
constexpr int kRefreshLoads = 32;   // column loads in flight per thread of the refresh
constexpr int kMaxRowsDense = 2048; // largest n of a dense design on these kernels

struct WideBufs {
  double* part;     // partial results, 4 per sweep block (or per pre block)
  int32_t* cnt;     // kept counts per test block
  int32_t* nzidx;   // p: nonzero coefficient list (refresh)
  double* nzval;    // p
};

// Elastic net (appendix): min 1/2||X b - y||^2 + a lambda ||b||_1 +
// (1-a) lambda/2 ||b||^2 is the Lasso with parameter a lambda on the
// augmented design X~ = [X; sqrt((1-a) lambda) I] and response y~ = [y; 0].
// X~ stays implicit: with mu2 = (1-a) lambda, ||x~_j||^2 = ||x_j||^2 + mu2,
// x~_j^T rho~ = x_j^T rho - mu2 b_j and ||rho~||^2 = ||rho||^2 + mu2 ||b||^2,
// y~^T rho~ = y^T rho; dot products get one more term.  a = 1 is the Lasso.
__device__ __forceinline__ double wide_l1(const ProbDesc& d, const WideState* st) {
  return st->enet * d.lam[st->t];
}
__device__ __forceinline__ double wide_mu2(const ProbDesc& d, const WideState* st) {
  return (1.0 - st->enet) * d.lam[st->t];
}
__device__ __forceinline__ int wide_nn(const ProbDesc& d, const WideState* st) {
  return st->enet < 1.0 ? d.n + 1 : d.n;
}

// Deterministic block reductions (256 or 1024 threads).
template <int NT>
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int o = NT / 2; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}
template <int NT>
__device__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int o = NT / 2; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// ---- precompute: ||x_j||^2, per-block max |x_j^T y| and a non-finite flag.
template <typename XT, int VEC, int NG>
__global__ __launch_bounds__(64 * kSweepWaves) void k_wide_pre(ProbDesc d, WideBufs wb) {
  using L = ColLayout<XT, VEC, 64, NG, false>;
  constexpr int RPL = L::RPL;
  __shared__ double sh[64 * kSweepWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const XT* X = (const XT*)d.X;
  const XT* Y = (const XT*)d.y;
  double yr[RPL];
#pragma unroll
  for (int m = 0; m < NG; ++m)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      int i = L::row(lane, m, e);
      yr[m * VEC + e] = (i < d.n) ? (double)Y[i] : 0.0;
    }
  const int W = gridDim.x * kSweepWaves;
  const int wid = blockIdx.x * kSweepWaves + w;
  const uint64_t mk = L::rowmask(lane, d.n);
  double mx = 0.0, bad = 0.0;
  int jm = 0x7fffffff;  // first column reaching mx
  for (int j = wid; j < d.p; j += W) {
    XT xv[RPL];
    L::load(X + (int64_t)j * d.ldx, d.n, lane, nullptr, mk, xv);
    double s2 = 0.0, sy = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      s2 = fma((double)xv[i], (double)xv[i], s2);
      sy = fma((double)xv[i], yr[i], sy);
    }
    s2 = wave_sum(s2);
    sy = wave_sum(sy);
    if (lane == 0) {
      d.nrm2[j] = s2;
      d.inv[j] = s2 > 0.0 ? 1.0 / s2 : 0.0;
      d.xty[j] = sy;
      if (fabs(sy) > mx || (fabs(sy) == mx && j < jm)) {
        mx = fabs(sy);
        jm = j;
      }
      if (!isfinite(s2) || !isfinite(sy)) bad = 1.0;
    }
  }
  const double bmx = block_max<64 * kSweepWaves>(mx, sh);
  bad = block_max<64 * kSweepWaves>(bad, sh);
  // first column of the block reaching its maximum
  const double jb = block_max<64 * kSweepWaves>(
      (lane == 0 && mx == bmx && jm != 0x7fffffff) ? -(double)jm : -INFINITY, sh);
  if (threadIdx.x == 0) {
    wb.part[4 * blockIdx.x + 0] = bmx;
    wb.part[4 * blockIdx.x + 1] = bad;
    wb.part[4 * blockIdx.x + 2] = -jb;
  }
}

// ---- x_j^T x_{j*} for every column (the Dynamic ST3 rule only).
template <typename XT, int VEC, int NG>
__global__ __launch_bounds__(64 * kSweepWaves) void k_wide_gstar(ProbDesc d, WideState* st) {
  using L = ColLayout<XT, VEC, 64, NG, false>;
  constexpr int RPL = L::RPL;
  if (st->rule != 4 || st->done) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const XT* X = (const XT*)d.X;
  const uint64_t mk = L::rowmask(lane, d.n);
  XT xs[RPL];
  L::load(X + (int64_t)st->jstar * d.ldx, d.n, lane, nullptr, mk, xs);
  const int W = gridDim.x * kSweepWaves;
  const int wid = blockIdx.x * kSweepWaves + w;
  for (int j = wid; j < d.p; j += W) {
    XT xv[RPL];
    L::load(X + (int64_t)j * d.ldx, d.n, lane, nullptr, mk, xv);
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) a = fma((double)xv[i], (double)xs[i], a);
    a = wave_sum(a);
    if (lane == 0) d.gst[j] = a;
  }
}

// ---- init: lambda_max, ||y||^2, the grid, beta, the state machine.
template <typename XT>
__global__ __launch_bounds__(256) void k_wide_init(ProbDesc d, WideState* st, WideBufs wb,
                                                   int npre, PathOpts opts) {
  __shared__ double sh[256];
  const XT* Y = (const XT*)d.y;
  double mx = 0.0, bad = 0.0, yy = 0.0;
  for (int b = threadIdx.x; b < npre; b += 256) {
    mx = fmax(mx, wb.part[4 * b]);
    bad = fmax(bad, wb.part[4 * b + 1]);
  }
  __shared__ double shj[256];
  const double gmx = block_max<256>(mx, shj);
  double jneg = -INFINITY;
  for (int b = threadIdx.x; b < npre; b += 256)
    if (wb.part[4 * b] == gmx) jneg = fmax(jneg, -wb.part[4 * b + 2]);
  const int jstar = (int)(-block_max<256>(jneg, shj));
  for (int i = threadIdx.x; i < d.n; i += 256) {
    double v = (double)Y[i];
    yy = fma(v, v, yy);
  }
  mx = block_max<256>(mx, sh);
  bad = block_max<256>(bad, sh);
  yy = block_sum<256>(yy, sh);
  if (!isfinite(yy)) bad = 1.0;
  const int T = d.T;
  // the smallest lambda with a zero solution: ||X^T y||_inf / a
  const double lmx = mx / opts.enet;
  for (int t = threadIdx.x; t < T; t += 256) {
    double lam;
    if (d.has_lambdas)
      lam = d.lam_in[t] * (d.lambda_relative ? lmx : 1.0);
    else
      lam = (T == 1) ? lmx : lmx * pow(d.lambda_min_ratio, (double)t / (double)(T - 1));
    d.lam[t] = lam;
    if (d.lambda_out) d.lambda_out[t] = lam;
  }
  for (int j = threadIdx.x; j < d.p; j += 256)
    d.beta[j] = (d.beta_init && bad == 0.0) ? d.beta_init[j] : 0.0;
  if (bad != 0.0) {
    for (int64_t e = threadIdx.x; e < (int64_t)d.p * T; e += 256) d.beta_out[e] = 0.0;
    for (int t = threadIdx.x; t < T; t += 256) {
      d.gap_out[t] = NAN;
      d.epochs_out[t] = 0;
      d.nactive_out[t] = 0;
      d.status_out[t] = 2;
    }
  }
  if (threadIdx.x == 0) {
    st->lambda_max = mx;
    st->ynorm2 = yy;
    st->eps = opts.eps_rel * yy;
    st->t = 0;
    st->k = 0;
    st->q = d.p;
    st->full = 1;
    st->cur = 0;
    st->done = (bad != 0.0) ? 1 : 0;
    st->phase = 0;
    st->need_refresh = 0;
    st->passes = 0;
    st->status_acc = 0;
    st->nonfinite = (bad != 0.0) ? 1 : 0;
    st->resume = 0;
    st->rule = opts.rule;
    st->enet = opts.enet;
    st->jstar = (jstar >= 0 && jstar < d.p) ? jstar : 0;
    st->sstar = d.xty[st->jstar] >= 0.0 ? 1.0 : -1.0;
    st->nstar = sqrt(d.nrm2[st->jstar]);
    st->first_epoch = 1;
    st->tau = INFINITY;
    st->tau_first = INFINITY;
    st->dmax2 = 0.0;
    st->n_visits = 0;
    st->n_rounds = 0;
    st->n_stops = 0;
    st->n_epochs = 0;
  }
}

// ---- residual refresh: ordered list of nonzero coefficients over A, then
// rho = y - sum beta_j x_j (ascending j) with one thread per row.
// mode 0: always; mode 1: only when a nonzero coefficient was screened.
template <typename XT>
__global__ __launch_bounds__(kRefreshThreads) void k_wide_refresh(ProbDesc d, WideState* st,
                                                                  WideBufs wb, int mode) {
  constexpr int NW = kRefreshThreads / 64;
  __shared__ int wcnt[NW];
  __shared__ double sh[kRefreshThreads];
  if (st->done) return;
  if (mode == 0 && st->phase != 0) return;
  if (mode == 1 && (st->phase != 2 || !st->need_refresh)) return;
  const int q = st->q;
  const bool full = st->full != 0;
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // Wave w scans positions [w*span, (w+1)*span) of A in order.
  const int span = (q + NW - 1) / NW;
  const int k0 = w * span, k1 = min(q, k0 + span);
  // The scans take kRefreshBatch rows of 64 positions at a time, all loads
  // of a batch issued before the first is used.
  constexpr int RB = kRefreshBatch;
  int cntw = 0;
  for (int base = k0; base < k1; base += 64 * RB) {
    int jr[RB];
    double br[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int k = min(base + 64 * r + lane, k1 - 1);  // clamped: loads need no branch
      const int ak = act[k];
      jr[r] = full ? k : ak;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const double b = d.beta[jr[r]];
      br[r] = base + 64 * r + lane < k1 ? b : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) cntw += __popcll(ballot(br[r] != 0.0));
  }
  if (lane == 0) wcnt[w] = cntw;
  __syncthreads();
  int off = 0, nnz = 0;
  for (int v = 0; v < NW; ++v) {
    if (v < w) off += wcnt[v];
    nnz += wcnt[v];
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int base = k0; base < k1; base += 64 * RB) {
    int jr[RB];
    double br[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int k = min(base + 64 * r + lane, k1 - 1);  // clamped: loads need no branch
      const int ak = act[k];
      jr[r] = full ? k : ak;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const double b = d.beta[jr[r]];
      br[r] = base + 64 * r + lane < k1 ? b : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const uint64_t m = ballot(br[r] != 0.0);
      if (br[r] != 0.0) {
        const int pos = off + __popcll(m & lt);
        wb.nzidx[pos] = jr[r];
        wb.nzval[pos] = br[r];
      }
      off += __popcll(m);
    }
  }
  __threadfence_block();
  // rho_i = y_i - sum_e beta_e x_{j_e, i} in ascending e, one thread per row;
  // the list passes through LDS a tile at a time and each thread keeps
  // kRefreshLoads column loads in flight (the one block's sum is a chain of
  // load latencies, nnz / kRefreshLoads of them).
  constexpr int RT = (kMaxRowsDense + kRefreshThreads - 1) / kRefreshThreads;
  constexpr int TILE = kRefreshThreads;
  __shared__ int s_ix[TILE];
  __shared__ double s_v[TILE];
  const XT* X = (const XT*)d.X;
  const XT* Y = (const XT*)d.y;
  double v[RT], yv[RT];
  int rr[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int i = threadIdx.x + t * kRefreshThreads;
    rr[t] = i < d.n ? (d.rows ? d.rows[i] : i) : 0;
    yv[t] = i < d.n ? (double)Y[rr[t]] : 0.0;
    v[t] = yv[t];
  }
  for (int e0 = 0; e0 < nnz; e0 += TILE) {
    const int ne = min(TILE, nnz - e0);
    __syncthreads();  // the previous tile is consumed (and the list is written)
    for (int e = threadIdx.x; e < ne; e += kRefreshThreads) {
      s_ix[e] = wb.nzidx[e0 + e];
      s_v[e] = wb.nzval[e0 + e];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      if (threadIdx.x + t * kRefreshThreads >= d.n) continue;
      const XT* Xr = X + rr[t];
      constexpr int NL = kRefreshLoads;
      int e = 0;
      for (; e + NL <= ne; e += NL) {
        XT xv[NL];
#pragma unroll
        for (int u = 0; u < NL; ++u) xv[u] = Xr[(int64_t)s_ix[e + u] * d.ldx];
#pragma unroll
        for (int u = 0; u < NL; ++u) v[t] = fma(-s_v[e + u], (double)xv[u], v[t]);
      }
      for (; e < ne; ++e) v[t] = fma(-s_v[e], (double)Xr[(int64_t)s_ix[e] * d.ldx], v[t]);
    }
  }
  double s2 = 0.0, sy = 0.0;
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int i = threadIdx.x + t * kRefreshThreads;
    if (i < d.n) {
      d.rho[i] = v[t];
      s2 = fma(v[t], v[t], s2);
      sy = fma(yv[t], v[t], sy);
    }
  }
  s2 = block_sum<kRefreshThreads>(s2, sh);
  sy = block_sum<kRefreshThreads>(sy, sh);
  const double mu2 = wide_mu2(d, st);
  if (mu2 > 0.0) {  // elastic net: ||rho~||^2 = ||rho||^2 + mu2 ||beta||^2
    double bb = 0.0;
    for (int e = threadIdx.x; e < nnz; e += kRefreshThreads) bb = fma(wb.nzval[e], wb.nzval[e], bb);
    s2 += mu2 * block_sum<kRefreshThreads>(bb, sh);
  }
  if (threadIdx.x == 0) {
    st->R2 = s2;
    st->Ry = sy;
    st->nnz = nnz;
    if (mode == 1) {
      // screened coefficients were zeroed: ||beta||_1 only fell
      st->pb2 = fmax(st->pb2, s2 + 2.0 * wide_l1(d, st) * st->l1);
      st->need_refresh = 0;
    }
  }
}

// ---- the sweep: c_k = x_{A[k]}^T rho for the k of A, per-block partials
// (max |c|, ||beta||_1, sum |beta_j| ||x_j||, max ||x_j||).  WN = 1: the
// column norms are computed here too (screen()); WN = 2: and x_j^T y (the
// dome test of screen()).
template <typename XT, int VEC, int NG, int WN>
__global__ __launch_bounds__(64 * kSweepWaves) void k_wide_sweep(ProbDesc d, WideState* st,
                                                                 WideBufs wb) {
  constexpr bool with_nrm2 = WN >= 1;
  constexpr bool with_xty = WN == 2;
  using L = ColLayout<XT, VEC, 64, NG, false>;
  constexpr int RPL = L::RPL;
  __shared__ double sh[4 * kSweepWaves];
  if (st->done || st->phase != 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = st->q;
  const bool full = st->full != 0;
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  const XT* X = (const XT*)d.X;
  double r[RPL];
  double yv[with_xty ? RPL : 1];
#pragma unroll
  for (int m = 0; m < NG; ++m)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      int i = L::row(lane, m, e);
      r[m * VEC + e] = (i < d.n) ? d.rho[i] : 0.0;
      if constexpr (with_xty) yv[m * VEC + e] = (i < d.n) ? (double)((const XT*)d.y)[i] : 0.0;
    }
  const int W = gridDim.x * kSweepWaves;
  const int wid = blockIdx.x * kSweepWaves + w;
  const int stride = W * kSweepU;
  const uint64_t mk = L::rowmask(lane, d.n);
  const double mu2 = WN == 0 ? wide_mu2(d, st) : 0.0;
  // Every lane carries the same wave-wide totals (the reductions below leave
  // the sum in all lanes); lane 0's copy is the wave's contribution.
  double Ml = 0.0, l1 = 0.0, sb = 0.0, xm = 0.0;
  // Positions past q-1 are clamped to q-1: that column is computed again
  // and its (identical) results stored again, so that the loop has no
  // data-dependent branches and its memory waits stay exact.
  // The wave's next step: clamped positions kn and their list entries an,
  // loaded a step ahead; the column indices jn are selected after the
  // step's arithmetic, when only the step's stores were issued after them.
  int kn[kSweepU], an[kSweepU], jn[kSweepU];
  int base = wid * kSweepU;
#pragma unroll
  for (int u = 0; u < kSweepU; ++u) {
    kn[u] = max(0, min(base + u, q - 1));
    an[u] = act[kn[u]];
    jn[u] = __builtin_amdgcn_readfirstlane(full ? kn[u] : an[u]);
  }
  for (; base < q; base += stride) {
    int jj[kSweepU];
    double nrv[kSweepU], bv[kSweepU];
    XT xv[kSweepU][RPL];
    // the per-column scalars are issued ahead of the columns, so waiting
    // for them leaves the columns in flight
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) {
      jj[u] = jn[u];
      nrv[u] = with_nrm2 ? 0.0 : d.nrm2[jj[u]];
      bv[u] = d.beta[jj[u]];
    }
#pragma unroll
    for (int u = 0; u < kSweepU; ++u)
      L::load_raw_nt(X + (int64_t)jj[u] * d.ldx, d.n, lane, xv[u]);
    const int nb = base + stride;
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) {
      kn[u] = max(0, min(nb + u, q - 1));
      an[u] = act[kn[u]];
    }
    // keep every load of the step issued before the first use
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) {
      const bool valid = base + u < q;
      const int kc = valid ? base + u : q - 1;
      double a = 0.0, s2 = 0.0, sy = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        a = fma((double)xv[u][i], r[i], a);  // r is zero at rows >= n
        if (with_nrm2) {
          const double xi = L::at(xv[u], mk, i);
          s2 = fma(xi, xi, s2);
        }
        if constexpr (with_xty) sy = fma((double)xv[u][i], yv[i], sy);
      }
      a = wave_sum(a);
      if (with_nrm2) s2 = wave_sum(s2);
      if constexpr (with_xty) sy = wave_sum(sy);
      const int j = jj[u];
      const double b = bv[u];
      a -= mu2 * b;  // mu2 is 0 but for the elastic net
      // every lane stores the same value
      d.c[kc] = a;
      if (with_nrm2) d.nrm2[j] = s2;
      if constexpr (with_xty) d.xty[j] = sy;
      const double nr = (with_nrm2 ? s2 : nrv[u]) + mu2;
      const double ab = valid ? fabs(b) : 0.0;
      const double xn = valid ? sqrt(nr) : 0.0;
      Ml = fmax(Ml, valid ? fabs(a) : 0.0);
      l1 += ab;
      sb += ab * xn;
      xm = fmax(xm, xn);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) jn[u] = __builtin_amdgcn_readfirstlane(full ? kn[u] : an[u]);
  }
  if (lane == 0) {
    sh[4 * w + 0] = Ml;
    sh[4 * w + 1] = l1;
    sh[4 * w + 2] = sb;
    sh[4 * w + 3] = xm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < kSweepWaves; ++v) {
      Ml = fmax(Ml, sh[4 * v + 0]);
      l1 += sh[4 * v + 1];
      sb += sh[4 * v + 2];
      xm = fmax(xm, sh[4 * v + 3]);
    }
    wb.part[4 * blockIdx.x + 0] = Ml;
    wb.part[4 * blockIdx.x + 1] = l1;
    wb.part[4 * blockIdx.x + 2] = sb;
    wb.part[4 * blockIdx.x + 3] = xm;
  }
}

// ---- gap, stop test and bookkeeping.  mode 0: path; mode 1: screen() (the
// gap is reported and the test always runs).
template <typename XT>
__global__ __launch_bounds__(256) void k_wide_gap(ProbDesc d, WideState* st, WideBufs wb,
                                                  int nsweep, int mode, double* gap_o,
                                                  double* alpha_o, double* radius_o,
                                                  PathOpts opts) {
  __shared__ double sh[256];
  if (st->done || st->phase != 0) return;
  double M = 0.0, l1 = 0.0, sb = 0.0, xm = 0.0;
  for (int b = threadIdx.x; b < nsweep; b += 256) {
    M = fmax(M, wb.part[4 * b]);
    l1 += wb.part[4 * b + 1];
    sb += wb.part[4 * b + 2];
    xm = fmax(xm, wb.part[4 * b + 3]);
  }
  M = block_max<256>(M, sh);
  l1 = block_sum<256>(l1, sh);
  sb = block_sum<256>(sb, sh);
  xm = block_max<256>(xm, sh);
  const int t = st->t;
  const double lambda = wide_l1(d, st);  // the Lasso parameter (a lambda_t for the elastic net)
  GapInfo g = gap_safe(st->R2, st->Ry, l1, sb, xm, M, st->nnz, wide_nn(d, st), lambda,
                       sqrt(st->ynorm2), st->q, st->rule == 1, st->rule >= 2);
  if (st->rule >= 2)
    rule_ball(g, st->rule, st->lambda_max, st->sstar, st->nstar, sqrt(st->ynorm2), d.n);
  if (threadIdx.x == 0) {
    st->Rlo = g.Rlo;
    st->Rhi = g.Rhi;
    st->rc2lo = g.rc2lo;
    st->e_y = g.e_y;
    st->shift = g.shift;
    st->rad_s = g.rad_s;
    st->e_shift = g.e_shift;
  }
  if (mode == 1) {
    if (threadIdx.x == 0) {
      *gap_o = g.gap;
      *alpha_o = g.alpha;
      *radius_o = g.radius;
      st->alpha_s = g.alpha;
      st->radius_s = g.radius;
      st->e_c = g.e_c;
      st->gap = g.gap;
      st->phase = 1;
    }
    return;
  }
  const bool conv = g.gap <= st->eps;
  const bool out_of_budget = st->k >= opts.K;
  if (conv || out_of_budget) {
    const int p = d.p;
    double* bo = d.beta_out + (int64_t)t * p;
    for (int j = threadIdx.x; j < p; j += 256) bo[j] = d.beta[j];
    if (threadIdx.x == 0) {
      d.gap_out[t] = g.gap;
      d.epochs_out[t] = st->k;
      d.nactive_out[t] = st->q;
      d.status_out[t] = conv ? 0 : 1;
      if (!conv) st->status_acc = 1;
      st->passes += 1;
      st->t = t + 1;
      st->k = 0;
      st->q = p;
      st->full = 1;
      st->cur = 0;
      st->phase = 0;
      st->need_refresh = 0;
      st->first_epoch = 1;
      if (t + 1 >= d.T) st->done = 1;
    }
  } else if (threadIdx.x == 0) {
    st->alpha_s = g.alpha;
    st->radius_s = g.radius;
    st->e_c = g.e_c;
    st->gap = g.gap;
    st->phase = 1;
    st->passes += 1;
    // 2 P(beta) at this pass bounds ||rho||^2 for every later CD iterate of
    // the interval (CD never increases P)
    st->l1 = l1;
    st->pb2 = st->R2 + 2.0 * lambda * l1;
  }
}

// ---- CD rounds of the wide schedule.
//
// An epoch of cyclic CD over A (Algorithm 1) visits every position in
// order.  A coordinate at zero stays at zero at its visit iff
// |x_k^T rho_visit| <= lambda.  With c_k = x_k^T rho_a at an anchor rho_a
// and D = rho_visit - rho_a, |x_k^T rho_visit| <= |c_k| + ||x_k|| ||D||, so
// while ||D|| <= tau every zero coordinate with |c_k| + ||x_k|| tau <= lambda
// (less the rounding of c_k) is left unchanged by its visit and need not be
// visited.  A round therefore
//   1. sweeps c_k for the positions from `resume` on (grid-wide, the anchor),
//   2. lists, in order, the positions that are nonzero or fail that test
//      (k_wide_lcount / k_wide_lcompact),
//   3. visits the listed positions exactly on one wavefront, tracking ||D||
//      from the scalars of each update:
//         ||D - delta x_m||^2 = ||D||^2 - 2 delta (d_m - c_m) + delta^2 ||x_m||^2
//      with d_m = x_m^T rho_visit, and stops right after an update that takes
//      ||D|| above tau: the next round re-anchors at the following position.
// The result is the cyclic epoch itself (up to the order of rounding).

// c_k = x_{A[k]}^T rho for the positions k >= resume (the anchor of a round).
template <typename XT, int VEC, int NG>
__global__ __launch_bounds__(64 * kSweepWaves) void k_wide_csweep(ProbDesc d, WideState* st) {
  using L = ColLayout<XT, VEC, 64, NG, false>;
  constexpr int RPL = L::RPL;
  if (st->done || st->phase != 2) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = st->q;
  const int k0 = st->resume;
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  const XT* X = (const XT*)d.X;
  double r[RPL];
#pragma unroll
  for (int m = 0; m < NG; ++m)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      int i = L::row(lane, m, e);
      r[m * VEC + e] = (i < d.n) ? d.rho[i] : 0.0;
    }
  const int W = gridDim.x * kSweepWaves;
  const int wid = blockIdx.x * kSweepWaves + w;
  const double mu2 = wide_mu2(d, st);
  const int stride = W * kSweepU;
  int base = k0 + wid * kSweepU;
  // Positions past q-1 are clamped to q-1 (the same value is stored
  // again).  The list entries an of the next step are loaded a step ahead
  // and taken into jn after the step's arithmetic.
  int an[kSweepU], jn[kSweepU];
#pragma unroll
  for (int u = 0; u < kSweepU; ++u) {
    an[u] = act[max(0, min(base + u, q - 1))];
    jn[u] = __builtin_amdgcn_readfirstlane(an[u]);
  }
  for (; base < q; base += stride) {
    XT xv[kSweepU][RPL];
    int jj[kSweepU];
    double bv[kSweepU];
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) {
      jj[u] = jn[u];
      bv[u] = d.beta[jj[u]];
    }
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) L::load_raw(X + (int64_t)jj[u] * d.ldx, d.n, lane, nullptr, xv[u]);
    const int nb = base + stride;
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) an[u] = act[max(0, min(nb + u, q - 1))];
    // keep every load of the step issued before the first use
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) {
      double a = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) a = fma((double)xv[u][i], r[i], a);  // r is zero at rows >= n
      a = wave_sum(a);
      d.c[base + u < q ? base + u : q - 1] = a - mu2 * bv[u];  // every lane stores the same value
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) jn[u] = __builtin_amdgcn_readfirstlane(an[u]);
  }
}

// Whether position k (>= resume) must be visited exactly in this round;
// nrm2 = ||x_j||^2 and b = beta_j of its column, ck its anchored correlation.
__device__ __forceinline__ bool wide_listed(const ProbDesc& d, const WideState* st, double nrm2,
                                            double b, double ck, double lambda, double tau,
                                            double rnorm) {
  const double nr = nrm2 + wide_mu2(d, st);
  if (!(nrm2 > 0.0)) return false;  // a zero column never moves
  if (b != 0.0) return true;
  const int nn = wide_nn(d, st);
  const double xn = sqrt(nr) * (1.0 + gam(nn + 2));
  // |c^_k - x_k^T rho_a| <= gamma_{n+1} ||x_k|| ||rho_a||
  const double thr = lambda * (1.0 - 4.0 * kU) - gam(nn + 1) * xn * rnorm;
  return fabs(ck) + xn * tau > thr;
}

// The CD walk of one round on one wavefront (layout of the sweep: all 64
// lanes split one column).  ntile: number of list tiles of the round.
template <typename XT, int VEC, int NG>
__global__ __launch_bounds__(64) void k_wide_walk(ProbDesc d, WideState* st, WideBufs wb,
                                                  int ntile, PathOpts opts) {
  using L = ColLayout<XT, VEC, 64, NG, false>;
  constexpr int RPL = L::RPL;
  constexpr int SEG = 1024;  // list entries staged in LDS at a time
  constexpr int RING = (RPL * sizeof(XT) <= 64) ? 6 : 3;
  __shared__ int s_j[SEG];
  __shared__ double s_c[SEG], s_b[SEG], s_inv[SEG], s_nr[SEG], s_xn[SEG];
  if (st->done || st->phase != 2) return;
  const int lane = threadIdx.x;
  const int q = st->q;
  const int32_t* act = d.act + (int64_t)st->cur * d.p;
  const double lambda = wide_l1(d, st);
  const double mu2 = wide_mu2(d, st);
  const int nn = wide_nn(d, st);
  const double tau = st->tau;
  const double tau2 = tau * tau;
  const gbl<XT>* X = gptr((const XT*)d.X);
  int nl = 0;
  for (int b = lane; b < ntile; b += 64) nl += wb.cnt[b];
  nl = wave_sum_i(nl);
  const uint64_t mk = L::rowmask(lane, d.n);
  double r[RPL];
#pragma unroll
  for (int m = 0; m < NG; ++m)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      int i = L::row(lane, m, e);
      r[m * VEC + e] = (i < d.n) ? d.rho[i] : 0.0;
    }
  // ||rho|| of every iterate of the round is at most sqrt(2 P) of the pass
  const double rb = sqrt(st->pb2) * (1.0 + 1e-9);
  const double erc = 4.0 * gam(nn + 1) * rb;
  double D2 = 0.0, De = 0.0, dmax2 = 0.0;
  int stop_k = -1;
  long long visits = 0;
  const gbl<int32_t>* lj = gptr(d.lst) + d.p;
  const gbl<double>* lv = gptr(d.lval);
  for (int s0 = 0; s0 < nl && stop_k < 0; s0 += SEG) {
    const int cnt = min(SEG, nl - s0);
    // the list holds each entry's feature and scalars contiguously, so the
    // staging loads are coalesced and independent (four entries per lane in
    // flight)
    for (int e0 = 0; e0 < cnt; e0 += 256) {
      int jv[4];
      double cv[4], bv[4], iv[4], nv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + 64 * u + lane;
        const int ee = s0 + (e < cnt ? e : cnt - 1);
        jv[u] = lj[ee];
        cv[u] = lv[4 * (int64_t)ee + 0];
        bv[u] = lv[4 * (int64_t)ee + 1];
        iv[u] = lv[4 * (int64_t)ee + 2];
        nv[u] = lv[4 * (int64_t)ee + 3];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + 64 * u + lane;
        if (e < cnt) {
          s_j[e] = jv[u];
          s_c[e] = cv[u];
          s_b[e] = bv[u];
          s_inv[e] = iv[u];
          s_nr[e] = nv[u];
          s_xn[e] = sqrt(nv[u]) * (1.0 + gam(nn + 2));
        }
      }
    }
    wave_lds_order();
    XT xs[RING][RPL];
    // the first RING-1 columns, issued in ring order: the scheduler must not
    // reorder them, or the wait for stage 0 would also wait for the others
#pragma unroll
    for (int i = 0; i + 1 < RING; ++i) {
      L::load_raw(X + (int64_t)s_j[i < cnt ? i : cnt - 1] * d.ldx, d.n, lane, nullptr, xs[i]);
      __builtin_amdgcn_sched_barrier(0);
    }
    int e_stop = -1;
    for (int e0 = 0; e0 < cnt; e0 += RING) {
#pragma unroll
      for (int i = 0; i < RING; ++i) {
        const int e = e0 + i;
        {
          const int en = e + RING - 1;
          L::load_raw(X + (int64_t)s_j[en < cnt ? en : cnt - 1] * d.ldx, d.n, lane, nullptr,
                      xs[(i + RING - 1) % RING]);
        }
        if (e < cnt && e_stop < 0) {
          const double b = s_b[e], inv = s_inv[e];
          // rows >= n hold copies of row 0: zero them once, in FP32
          double xd[RPL];
#pragma unroll
          for (int t = 0; t < RPL; ++t) xd[t] = (double)(((mk >> t) & 1ull) ? xs[i][t] : XT(0));
          double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
          for (int t = 0; t < RPL; t += 4) {
            a0 = fma(xd[t], r[t], a0);
            if (t + 1 < RPL) a1 = fma(xd[t + 1], r[t + 1], a1);
            if (t + 2 < RPL) a2 = fma(xd[t + 2], r[t + 2], a2);
            if (t + 3 < RPL) a3 = fma(xd[t + 3], r[t + 3], a3);
          }
          const double dm = wave_sum((a0 + a1) + (a2 + a3)) - mu2 * b;
          const double bn = soft_thr(lambda * inv, b + dm * inv);
          ++visits;
          if (bn != b) {
            const double delta = bn - b;
#pragma unroll
            for (int t = 0; t < RPL; ++t) r[t] = fma(-delta, xd[t], r[t]);
            if (lane == 0) s_b[e] = bn;
            const double nr = s_nr[e];
            const double dd = dm - s_c[e];
            const double t1 = -2.0 * delta * dd, t2 = delta * delta * nr;
            D2 = D2 + t1 + t2;
            // rounding of this update and of d_m - c_m taken as x_m^T D
            De += 4.0 * kU * (fabs(D2) + fabs(t1) + t2) + fabs(delta) * s_xn[e] * erc;
            dmax2 = fmax(dmax2, D2 + De);
            if (D2 + De > tau2) e_stop = e;
          }
        }
      }
      if (e_stop >= 0) break;
    }
    wave_lds_order();
    for (int e = lane; e < cnt; e += 64) d.beta[s_j[e]] = s_b[e];
    if (e_stop >= 0) stop_k = gptr(d.lst)[s0 + e_stop];
    wave_lds_order();
  }
  double r2 = 0.0;
#pragma unroll
  for (int m = 0; m < NG; ++m)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int i = L::row(lane, m, e);
      if (i < d.n) d.rho[i] = r[m * VEC + e];
      r2 = fma(r[m * VEC + e], r[m * VEC + e], r2);
    }
  r2 = wave_sum(r2);
  if (lane == 0) {
    st->R2 = r2;
    st->n_visits += visits;
    st->n_rounds += 1;
    st->dmax2 = fmax(st->dmax2, dmax2);
    if (stop_k >= 0 && stop_k + 1 < q) {
      // re-anchor after the listed position where ||D|| passed tau, with a
      // larger threshold
      st->resume = stop_k + 1;
      st->tau = fmax(4.0 * tau, 4.0 * sqrt(dmax2));
      st->n_stops += 1;
    } else {
      // the epoch is complete; the next one starts at position 0 with a
      // threshold from this epoch's largest residual move
      const int k = st->k + 1;
      st->k = k;
      st->n_epochs += 1;
      st->resume = 0;
      const double tn = 2.0 * sqrt(st->dmax2);
      if (st->first_epoch) st->tau_first = tn;
      st->first_epoch = 0;
      st->tau = tn;
      st->dmax2 = 0.0;
      if (k % opts.f == 0 || k >= opts.K) st->phase = 0;
    }
  }
}

// ---- sphere test: per-block kept counts; zero screened nonzero coefficients.
__global__ __launch_bounds__(256) void k_wide_test(ProbDesc d, WideState* st, WideBufs wb);
// ---- ordered compaction of the kept indices into `out` (or the other buffer).
__global__ __launch_bounds__(256) void k_wide_compact(ProbDesc d, WideState* st, WideBufs wb,
                                                      int32_t* out);
// ---- the list of positions a CD round visits exactly: per-tile counts, then
// the ordered compaction into d.lst (tiles of kTestTile positions from
// `resume`; tiles past q count zero).
__global__ __launch_bounds__(256) void k_wide_lcount(ProbDesc d, WideState* st, WideBufs wb);
__global__ __launch_bounds__(256) void k_wide_lcompact(ProbDesc d, WideState* st, WideBufs wb);
// ---- |A'| and buffer swap (path) or q_out (screen()).
__global__ __launch_bounds__(64) void k_wide_fin(ProbDesc d, WideState* st, WideBufs wb,
                                                 int ntest, int32_t* q_out);

}  // namespace gs
