// The per-problem ("narrow") schedule: one wavefront runs Algorithm 1 for one
// Lasso path, with the residual in LDS (canonical copy) and in registers
// (working copy in the column layout), and X streamed from L2/HBM.
//
// Column layout: lane = slot * S + seg.  Each of the C = 64/S slots works on
// its own column; the S lanes of a slot split that column's rows.  A column
// dot product is a per-lane FMA chain followed by a butterfly over S lanes.
//
// Cyclic CD over a chunk of C consecutive active coordinates: all C dot
// products x_j^T rho are formed at once against the current residual; the
// chunk is then resolved in ascending order: the first coordinate whose
// soft-threshold update changes beta is applied (rho -= delta x_j), the dot
// products of the later coordinates of the chunk are recomputed against the
// new residual, and the scan continues after it.  In exact arithmetic this is
// the same sequence of updates as one-coordinate-at-a-time cyclic CD.
#pragma once

#include "gs_device.hpp"

namespace gs {

template <typename XT, int VEC, int S, int NG, bool GATHER>
struct Narrow {
  using L = ColLayout<XT, VEC, S, NG, GATHER>;
  static constexpr int RPL = L::RPL;
  static constexpr int C = L::C;
  static constexpr int NMAX = L::NMAX;
  static constexpr int NT = (NMAX + 63) / 64;  // rows per lane, row-major layout

  // Per-wave context.
  struct Ctx {
    const XT* X;
    int64_t ldx;
    const int32_t* rows;
    int n, p;
    int lane, slot, seg;
    int ridx[GATHER ? NG : 1];  // gather: row of (seg, m) or -1
    int rrow[NT];               // row-major layout: source row of lane + 64 t
    double* y_l;                // LDS, n
    double* rho_l;              // LDS, n
    XT* tile;                   // LDS, 64 * RPL
    double* nrm2;
    double* beta;
    double* c;
    int32_t* act;
  };

  static __device__ __forceinline__ const XT* col(const Ctx& x, int j) {
    return x.X + (int64_t)j * x.ldx;
  }

  static __device__ void setup_rows(Ctx& x) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      int i = x.lane + 64 * t;
      x.rrow[t] = (i < x.n) ? (GATHER ? x.rows[i] : i) : -1;
    }
    if constexpr (GATHER) {
#pragma unroll
      for (int m = 0; m < NG; ++m) {
        int r = x.seg + S * m;
        x.ridx[m] = (r < x.n) ? x.rows[r] : -1;
      }
    }
  }

  static __device__ __forceinline__ void load_col(const Ctx& x, int j, bool valid, XT (&xv)[RPL]) {
    if (valid) {
      L::load(col(x, j), x.n, x.seg, x.ridx, xv);
    } else {
#pragma unroll
      for (int i = 0; i < RPL; ++i) xv[i] = XT(0);
    }
  }

  static __device__ __forceinline__ double dot(const XT (&xv)[RPL], const double (&r)[RPL]) {
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; i += 2) {
      a0 = fma((double)xv[i], r[i], a0);
      if (i + 1 < RPL) a1 = fma((double)xv[i + 1], r[i + 1], a1);
    }
    return seg_sum<S>(a0 + a1);
  }

  // Residual in the column layout, from the LDS copy.
  static __device__ void load_rho(const Ctx& x, double (&r)[RPL]) {
#pragma unroll
    for (int m = 0; m < NG; ++m)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        int i = L::row(x.seg, m, e);
        r[m * VEC + e] = (i < x.n) ? x.rho_l[i] : 0.0;
      }
  }

  // rho = y - sum_{j in A, beta_j != 0} beta_j x_j (ascending j), written to
  // LDS.  Returns nnz; R2 = ||rho||^2 and Ry = y^T rho.  (Sec. 2.3.)
  static __device__ int refresh(const Ctx& x, int q, bool full, double& R2, double& Ry) {
    double rr[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      int i = x.lane + 64 * t;
      rr[t] = (i < x.n) ? x.y_l[i] : 0.0;
    }
    int nnz = 0;
    for (int base = 0; base < q; base += 64) {
      int k = base + x.lane;
      int j = 0;
      double b = 0.0;
      if (k < q) {
        j = full ? k : x.act[k];
        b = x.beta[j];
      }
      uint64_t m = ballot(b != 0.0);
      nnz += __popcll(m);
      while (m) {
        int l = __builtin_ctzll(m);
        m &= m - 1;
        int jj = __builtin_amdgcn_readlane(j, l);
        double bb = readlane_d(b, l);
        const XT* cj = col(x, jj);
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (x.rrow[t] >= 0) rr[t] = fma(-bb, (double)cj[x.rrow[t]], rr[t]);
      }
    }
    double s2 = 0.0, sy = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      int i = x.lane + 64 * t;
      if (i < x.n) {
        x.rho_l[i] = rr[t];
        s2 = fma(rr[t], rr[t], s2);
        sy = fma(x.y_l[i], rr[t], sy);
      }
    }
    R2 = wave_sum(s2);
    Ry = wave_sum(sy);
    __syncthreads();
    return nnz;
  }

  // c_k = x_{A[k]}^T rho for every position k of A; M = max |c_k|,
  // l1 = ||beta||_1, sbx = sum |beta_j| ||x_j||, xmax = max ||x_j|| over A.
  static __device__ void sweep(const Ctx& x, int q, bool full, double& M, double& l1,
                               double& sbx, double& xmax) {
    double r[RPL];
    load_rho(x, r);
    double Ml = 0.0, l1l = 0.0, sbl = 0.0, xml = 0.0;
    int k = x.slot;
    bool v = k < q;
    int j = v ? (full ? k : x.act[k]) : 0;
    XT xv[RPL];
    load_col(x, j, v, xv);
    for (int base = 0; base < q; base += C) {
      int kn = base + C + x.slot;
      bool vn = kn < q;
      int jn = vn ? (full ? kn : x.act[kn]) : 0;
      XT xn[RPL];
      load_col(x, jn, vn, xn);
      double d = dot(xv, r);
      if (v && x.seg == 0) {
        x.c[k] = d;
        Ml = fmax(Ml, fabs(d));
        double b = x.beta[j], nr = sqrt(x.nrm2[j]);
        l1l += fabs(b);
        sbl += fabs(b) * nr;
        xml = fmax(xml, nr);
      }
      k = kn;
      v = vn;
      j = jn;
#pragma unroll
      for (int i = 0; i < RPL; ++i) xv[i] = xn[i];
    }
    M = wave_max(Ml);
    l1 = wave_sum(l1l);
    sbx = wave_sum(sbl);
    xmax = wave_max(xml);
    __threadfence_block();
  }

  // Sphere test over A with ordered in-place compaction; screened nonzero
  // coefficients are set to zero (dropped_nz is then set).  Returns |A'|.
  static __device__ int test_compact(const Ctx& x, const GapInfo& g, int q, bool full,
                                     bool& dropped_nz) {
    int q2 = 0;
    bool dn = false;
    const uint64_t lt = (x.lane == 0) ? 0ull : (~0ull >> (64 - x.lane));
    for (int base = 0; base < q; base += 64) {
      int k = base + x.lane;
      bool v = k < q;
      int j = v ? (full ? k : x.act[k]) : 0;
      bool keep = false;
      if (v) {
        keep = sphere_keep(g, x.c[k], x.nrm2[j], x.n);
        if (!keep && x.beta[j] != 0.0) {
          x.beta[j] = 0.0;
          dn = true;
        }
      }
      uint64_t m = ballot(keep);
      if (keep) x.act[q2 + __popcll(m & lt)] = j;
      q2 += __popcll(m);
    }
    dropped_nz = ballot(dn) != 0;
    __threadfence_block();
    return q2;
  }

  // One cyclic CD epoch over A (Algorithm 1):
  //   beta_j <- ST(lambda/||x_j||^2, beta_j + x_j^T rho / ||x_j||^2),
  //   rho    <- rho - (beta_j' - beta_j) x_j.
  static __device__ void cd_epoch(const Ctx& x, int q, bool full, double lambda,
                                  double (&r)[RPL]) {
    int k = x.slot;
    bool v = k < q;
    int j = v ? (full ? k : x.act[k]) : 0;
    XT xv[RPL];
    load_col(x, j, v, xv);
    XT* mytile = x.tile + x.lane * RPL;
    for (int base = 0; base < q; base += C) {
      int kn = base + C + x.slot;
      bool vn = kn < q;
      int jn = vn ? (full ? kn : x.act[kn]) : 0;
      XT xn[RPL];
      load_col(x, jn, vn, xn);
#pragma unroll
      for (int i = 0; i < RPL; ++i) mytile[i] = xv[i];
      double b = v ? x.beta[j] : 0.0;
      double nr = v ? x.nrm2[j] : 0.0;
      double d = dot(xv, r);
      __syncthreads();
      int start = 0;
      bool changed = false;
      for (;;) {
        bool chg = false;
        double bn = b;
        if (v && x.slot >= start && nr > 0.0) {
          bn = soft_thr(lambda / nr, b + d / nr);
          chg = (bn != b);
        }
        uint64_t mk = ballot(chg);
        if (!mk) break;
        int l0 = __builtin_ctzll(mk);
        int cs = l0 / S;
        double delta = readlane_d(bn - b, l0);
        if (x.slot == cs) {
          b = bn;
          changed = true;
        }
        const XT* tx = x.tile + (cs * S + x.seg) * RPL;
#pragma unroll
        for (int i = 0; i < RPL; ++i) r[i] = fma(-delta, (double)tx[i], r[i]);
        if (cs + 1 >= C) break;
        d = dot(xv, r);
        start = cs + 1;
      }
      if (changed && x.seg == 0) x.beta[j] = b;
      __syncthreads();
      k = kn;
      v = vn;
      j = jn;
#pragma unroll
      for (int i = 0; i < RPL; ++i) xv[i] = xn[i];
    }
    __threadfence_block();
  }
};

// LDS bytes the narrow kernel needs for problems with n <= nmax.
template <typename XT, int VEC, int S, int NG, bool GATHER>
constexpr size_t narrow_lds_bytes() {
  using N = Narrow<XT, VEC, S, NG, GATHER>;
  return 2 * sizeof(double) * N::NMAX + sizeof(XT) * 64 * N::RPL;
}

// Persistent kernel: each wavefront pops problems from a device queue and
// runs the whole path of each.
template <typename XT, int VEC, int S, int NG, bool GATHER>
__global__ __launch_bounds__(64) void k_path_narrow(const ProbDesc* __restrict__ descs, int B,
                                                    int* queue, PathOpts opts) {
  using N = Narrow<XT, VEC, S, NG, GATHER>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  for (;;) {
    int task = 0;
    if (lane == 0) task = atomicAdd(queue, 1);
    task = __builtin_amdgcn_readfirstlane(task);
    if (task >= B) break;
    const ProbDesc d = descs[task];
    long long t_start = wall_clock64();

    typename N::Ctx x;
    x.X = (const XT*)d.X;
    x.ldx = d.ldx;
    x.rows = d.rows;
    x.n = d.n;
    x.p = d.p;
    x.lane = lane;
    x.slot = lane / S;
    x.seg = lane % S;
    x.y_l = reinterpret_cast<double*>(smem);
    x.rho_l = x.y_l + N::NMAX;
    x.tile = reinterpret_cast<XT*>(x.rho_l + N::NMAX);
    x.nrm2 = d.nrm2;
    x.beta = d.beta;
    x.c = d.c;
    x.act = d.act;
    N::setup_rows(x);
    const int n = d.n, p = d.p, T = d.T;
    const XT* Y = (const XT*)d.y;

    // ---- y into LDS; precompute ||x_j||^2 and lambda_max = ||X^T y||_inf
    double yy = 0.0;
    for (int i = lane; i < n; i += 64) {
      double v = (double)Y[GATHER ? d.rows[i] : i];
      x.y_l[i] = v;
      yy = fma(v, v, yy);
    }
    __syncthreads();
    const double ynorm2 = wave_sum(yy);
    bool bad = !isfinite(ynorm2);
    double lmax_l = 0.0;
    {
      double yr[N::RPL];
#pragma unroll
      for (int m = 0; m < NG; ++m)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          int i = N::L::row(x.seg, m, e);
          yr[m * VEC + e] = (i < n) ? x.y_l[i] : 0.0;
        }
      for (int base = 0; base < p; base += N::C) {
        int j = base + x.slot;
        bool v = j < p;
        XT xv[N::RPL];
        N::load_col(x, j, v, xv);
        double s2 = 0.0, sy = 0.0;
#pragma unroll
        for (int i = 0; i < N::RPL; ++i) {
          s2 = fma((double)xv[i], (double)xv[i], s2);
          sy = fma((double)xv[i], yr[i], sy);
        }
        s2 = seg_sum<S>(s2);
        sy = seg_sum<S>(sy);
        if (v && x.seg == 0) {
          x.nrm2[j] = s2;
          lmax_l = fmax(lmax_l, fabs(sy));
          if (!isfinite(s2) || !isfinite(sy)) bad = true;
        }
      }
    }
    const double lmax = wave_max(lmax_l);
    bad = ballot(bad) != 0;

    // ---- the lambda grid (Sec. 3.3) and the warm start beta^{lambda_0}
    for (int t = lane; t < T; t += 64) {
      double lam;
      if (d.has_lambdas)
        lam = d.lam[t] * (d.lambda_relative ? lmax : 1.0);
      else
        lam = (T == 1) ? lmax : lmax * pow(d.lambda_min_ratio, (double)t / (double)(T - 1));
      d.lam[t] = lam;
      if (d.lambda_out) d.lambda_out[t] = lam;
    }
    for (int j = lane; j < p; j += 64)
      x.beta[j] = (d.beta_init && !bad) ? d.beta_init[j] : 0.0;
    __threadfence_block();

    if (bad) {
      for (int t = 0; t < T; ++t) {
        for (int j = lane; j < p; j += 64) d.beta_out[(int64_t)t * p + j] = 0.0;
        if (lane == 0) {
          d.gap_out[t] = NAN;
          d.epochs_out[t] = 0;
          d.nactive_out[t] = 0;
          d.status_out[t] = 2;
        }
      }
    } else {
      const double eps = opts.eps_rel * ynorm2;
      const double ynorm = sqrt(ynorm2);
      const int f = opts.f, K = opts.K;
      for (int t = 0; t < T; ++t) {
        const double lambda = d.lam[t];
        int q = p;
        bool full = true;
        int k = 0, status = 1;
        double G = 0.0;
        double r[N::RPL];
        for (;;) {
          if (k % f == 0 || k == K) {
            double R2, Ry, M, l1, sbx, xmax;
            int nnz = N::refresh(x, q, full, R2, Ry);
            N::sweep(x, q, full, M, l1, sbx, xmax);
            GapInfo g = gap_safe(R2, Ry, l1, sbx, xmax, M, nnz, n, lambda, ynorm);
            G = g.gap;
            if (G <= eps) {
              status = 0;
              break;
            }
            if (k == K) break;
            bool dropped;
            q = N::test_compact(x, g, q, full, dropped);
            full = false;
            if (dropped) N::refresh(x, q, full, R2, Ry);
            N::load_rho(x, r);
          }
          N::cd_epoch(x, q, full, lambda, r);
          ++k;
        }
        // beta^{lambda_t} and its certificate
        double* bo = d.beta_out + (int64_t)t * p;
        for (int j = lane; j < p; j += 64) {
          double b = x.beta[j];
          bo[j] = b;
          if (opts.select_counts && b != 0.0) atomicAdd(&opts.select_counts[(int64_t)t * p + j], 1);
        }
        if (lane == 0) {
          d.gap_out[t] = G;
          d.epochs_out[t] = k;
          d.nactive_out[t] = q;
          d.status_out[t] = status;
        }
      }
    }
    if (opts.timestamps && lane == 0) {
      opts.timestamps[2 * d.orig] = t_start;
      opts.timestamps[2 * d.orig + 1] = wall_clock64();
    }
    __syncthreads();
  }
}

// The CD part of the wide schedule: one wavefront runs min(f, K - k) epochs
// over the active set the wide kernels left in the workspace.
template <typename XT, int VEC, int S, int NG, bool GATHER>
__global__ __launch_bounds__(64) void k_wide_cd(ProbDesc d, WideState* st, PathOpts opts) {
  using N = Narrow<XT, VEC, S, NG, GATHER>;
  extern __shared__ __align__(16) unsigned char smem[];
  if (st->done || st->phase != 2) return;
  const int lane = threadIdx.x;
  typename N::Ctx x;
  x.X = (const XT*)d.X;
  x.ldx = d.ldx;
  x.rows = d.rows;
  x.n = d.n;
  x.p = d.p;
  x.lane = lane;
  x.slot = lane / S;
  x.seg = lane % S;
  x.y_l = reinterpret_cast<double*>(smem);
  x.rho_l = x.y_l + N::NMAX;
  x.tile = reinterpret_cast<XT*>(x.rho_l + N::NMAX);
  x.nrm2 = d.nrm2;
  x.beta = d.beta;
  x.c = d.c;
  x.act = d.act + (int64_t)st->cur * d.p;
  N::setup_rows(x);
  for (int i = lane; i < d.n; i += 64) x.rho_l[i] = d.rho[i];
  __syncthreads();
  const int q = st->q;
  const bool full = st->full != 0;
  const int k0 = st->k;
  const int ne = min(opts.f, opts.K - k0);
  const double lambda = d.lam[st->t];
  double r[N::RPL];
  N::load_rho(x, r);
  for (int e = 0; e < ne; ++e) N::cd_epoch(x, q, full, lambda, r);
  __syncthreads();
  if (lane == 0) {
    st->k = k0 + ne;
    st->phase = 0;
  }
}

}  // namespace gs
