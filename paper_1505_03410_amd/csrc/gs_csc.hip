// Sparse designs in compressed sparse column form (CSC): Algorithm 1 for one
// path per wavefront, like the dense narrow schedule, with the residual in
// LDS (or in global memory when n rows do not fit) and every column access a
// gather or scatter over its nonzeros.  The screening sweep c_j = x_j^T rho
// is a transposed sparse matrix-vector product over the active columns
// (8 bytes of index and value per nonzero, Sec. 4.1's O(nnz) pass), the CD
// update of coordinate j touches only the rows of column j.
//
// Lanes of the wavefront split one column's nonzeros (64 at a time); rows
// within a column are distinct, so a column's scatter into the residual has
// no conflicts, and consecutive columns are ordered by a wavefront fence.
#include "../../include/gapsafe.h"
#include "gs_registry.hpp"
#include "gs_wide.hpp"

namespace gs {

namespace {

// One column's nonzeros in registers (the first 64: lane e holds entry e).
template <typename XT>
struct CscCol {
  int64_t b0;  // first entry
  int len;     // number of entries
  int row;     // this lane's row (0 when the lane has no entry)
  double val;  // this lane's value (0 when the lane has no entry)
};

template <typename XT>
__device__ __forceinline__ void csc_load(const ProbDesc& d, int j, int lane, CscCol<XT>& c) {
  const gbl<int64_t>* cp = gptr(d.col_ptr);
  c.b0 = cp[j];
  c.len = (int)(cp[j + 1] - c.b0);
  const bool v = lane < c.len;
  c.row = v ? gptr(d.row_idx)[c.b0 + lane] : 0;
  c.val = v ? (double)gptr((const XT*)d.X)[c.b0 + lane] : 0.0;
}

// x_j^T v for a vector v indexed by row (LDS or global), all entries.
template <typename XT, typename V>
__device__ __forceinline__ double csc_dot(const ProbDesc& d, const CscCol<XT>& c, V v,
                                          int lane) {
  double a = c.val * v[c.row];
  for (int e = 64 + lane; e < c.len; e += 64) {
    const int64_t k = c.b0 + e;
    a = fma((double)gptr((const XT*)d.X)[k], v[gptr(d.row_idx)[k]], a);
  }
  return wave_sum(a);
}

// v[rows of x_j] -= delta * x_j.
template <typename XT, typename V>
__device__ __forceinline__ void csc_axpy(const ProbDesc& d, const CscCol<XT>& c, double delta,
                                         V v, int lane) {
  if (lane < c.len) v[c.row] = fma(-delta, c.val, v[c.row]);
  for (int e = 64 + lane; e < c.len; e += 64) {
    const int64_t k = c.b0 + e;
    const int r = gptr(d.row_idx)[k];
    v[r] = fma(-delta, (double)gptr((const XT*)d.X)[k], v[r]);
  }
}

// Orders one wavefront's residual accesses across columns.
template <bool GRHO>
__device__ __forceinline__ void rho_order() {
  if constexpr (GRHO) {
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  } else {
    wave_lds_order();
  }
}

}  // namespace

// ||x_j||^2, 1/||x_j||^2 and x_j^T y of every column of every CSC problem
// (one wavefront per column, grid-stride over all problems' columns).
template <typename XT>
__global__ __launch_bounds__(256) void k_csc_colstats(const ProbDesc* __restrict__ descs, int B,
                                                      const int64_t* __restrict__ first_col) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t W = (int64_t)gridDim.x * 4;
  const int64_t total = first_col[B];
  for (int64_t g = wid; g < total; g += W) {
    int b = 0;
    while (first_col[b + 1] <= g) ++b;  // B is small: linear search
    const ProbDesc& d = descs[b];
    const int j = (int)(g - first_col[b]);
    CscCol<XT> c;
    csc_load(d, j, lane, c);
    const XT* Y = (const XT*)d.y;
    double s2 = c.val * c.val;
    double sy = c.val * (double)Y[c.row];
    for (int e = 64 + lane; e < c.len; e += 64) {
      const int64_t k = c.b0 + e;
      const double v = (double)((const XT*)d.X)[k];
      s2 = fma(v, v, s2);
      sy = fma(v, (double)Y[d.row_idx[k]], sy);
    }
    s2 = wave_sum(s2);
    sy = wave_sum(sy);
    if (lane == 0) {
      d.nrm2[j] = s2;
      d.inv[j] = s2 > 0.0 ? 1.0 / s2 : 0.0;
      d.xty[j] = sy;
    }
  }
}

// Persistent kernel: each wavefront pops problems from the queue and runs
// the whole path of each (residual-mode cyclic CD, GAP SAFE sphere or dome
// screening every f epochs).  GRHO: the residual lives in the workspace
// (global memory) instead of LDS.
template <typename XT, bool GRHO>
__global__ __launch_bounds__(64) void k_path_csc(const ProbDesc* __restrict__ descs, int B,
                                                 int* queue, PathOpts opts) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  for (;;) {
    int task = 0;
    if (lane == 0) task = atomicAdd(queue, 1);
    task = __builtin_amdgcn_readfirstlane(task);
    if (task >= B) break;
    const ProbDesc d = descs[task];
    const long long t_start = wall_clock64();
    const int n = d.n, p = d.p, T = d.T;
    double* rho = GRHO ? d.rho : reinterpret_cast<double*>(smem);
    gbl<double>* nrm2 = gptr(d.nrm2);
    gbl<double>* inv = gptr(d.inv);
    gbl<double>* xty = gptr(d.xty);
    gbl<double>* beta = gptr(d.beta);
    gbl<double>* cc = gptr(d.c);
    gbl<int32_t>* act = gptr(d.act);
    gbl<double>* lam_g = gptr(d.lam);
    const XT* Y = (const XT*)d.y;
    // ||y||^2, lambda_max = ||X^T y||_inf (Sec. 1.2), finiteness
    double yy = 0.0;
    for (int i = lane; i < n; i += 64) {
      const double v = (double)Y[i];
      yy = fma(v, v, yy);
    }
    const double ynorm2 = wave_sum(yy);
    double lm = 0.0;
    bool bad = !isfinite(ynorm2);
    for (int j = lane; j < p; j += 64) {
      lm = fmax(lm, fabs(xty[j]));
      if (!isfinite(nrm2[j]) || !isfinite(xty[j])) bad = true;
    }
    const double lmax = wave_max(lm);
    bad = ballot(bad) != 0;
    for (int t = lane; t < T; t += 64) {
      double lam;
      if (d.has_lambdas)
        lam = gptr(d.lam_in)[t] * (d.lambda_relative ? lmax : 1.0);
      else
        lam = (T == 1) ? lmax : lmax * pow(d.lambda_min_ratio, (double)t / (double)(T - 1));
      lam_g[t] = lam;
      if (d.lambda_out) gptr(d.lambda_out)[t] = lam;
    }
    {
      const gbl<const double>* bi = gptr(d.beta_init);
      for (int j = lane; j < p; j += 64) beta[j] = (bi && !bad) ? bi[j] : 0.0;
    }
    __threadfence_block();
    gbl<double>* bout = gptr(d.beta_out);
    if (bad) {
      for (int t = 0; t < T; ++t) {
        for (int j = lane; j < p; j += 64) bout[(int64_t)t * p + j] = 0.0;
        if (lane == 0) {
          d.gap_out[t] = NAN;
          d.epochs_out[t] = 0;
          d.nactive_out[t] = 0;
          d.status_out[t] = GS_STATUS_NONFINITE;
        }
      }
    } else {
      const double eps = opts.eps_rel * ynorm2;
      const double ynorm = sqrt(ynorm2);
      const int f = opts.f, K = opts.K;
      long long passes = 0, epochs_all = 0;
      for (int t = 0; t < T; ++t) {
        const double lambda = lam_g[t];
        int q = p;
        bool full = true;
        int k = 0, status = 1;
        double G = 0.0;
        for (;;) {
          if (k % f == 0 || k == K) {
            // residual refresh rho = y - sum beta_j x_j (ascending j)
            for (int i = lane; i < n; i += 64) rho[i] = (double)Y[i];
            rho_order<GRHO>();
            int nnz = 0;
            for (int base = 0; base < q; base += 64) {
              const int kk = base + lane;
              const int j = kk < q ? (full ? kk : act[kk]) : 0;
              const double b = kk < q ? beta[j] : 0.0;
              uint64_t m = ballot(b != 0.0);
              nnz += __popcll(m);
              while (m) {
                const int l = __builtin_ctzll(m);
                m &= m - 1;
                const int jl = __builtin_amdgcn_readlane(j, l);
                const double bl = readlane_d(b, l);
                CscCol<XT> c;
                csc_load(d, jl, lane, c);
                csc_axpy(d, c, bl, rho, lane);
                rho_order<GRHO>();
              }
            }
            double r2 = 0.0, ry = 0.0;
            for (int i = lane; i < n; i += 64) {
              const double v = rho[i];
              r2 = fma(v, v, r2);
              ry = fma((double)Y[i], v, ry);
            }
            const double R2 = wave_sum(r2), Ry = wave_sum(ry);
            // sweep c = X_A^T rho, M, ||beta||_1, sum |beta_j| ||x_j||, max ||x_j||
            double Ml = 0.0, l1l = 0.0, sbl = 0.0, xml = 0.0;
            for (int kk = 0; kk < q; ++kk) {
              const int j = full ? kk : act[kk];
              CscCol<XT> c;
              csc_load(d, j, lane, c);
              const double cj = csc_dot(d, c, rho, lane);
              if (lane == 0) cc[kk] = cj;
              const double xn = sqrt(nrm2[j]);
              const double b = beta[j];
              Ml = fmax(Ml, fabs(cj));
              l1l += fabs(b);
              sbl += fabs(b) * xn;
              xml = fmax(xml, xn);
            }
            ++passes;
            const GapInfo g = gap_safe(R2, Ry, l1l, sbl, xml, Ml, nnz, n, lambda, ynorm, q,
                                       opts.rule == GS_RULE_DOME);
            G = g.gap;
            if (G <= eps) {
              status = 0;
              break;
            }
            if (k == K) break;
            // sphere (and dome) test; ordered in-place compaction of A and
            // c; screened nonzero coefficients set to zero
            int q2 = 0;
            bool dropped = false;
            const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
            __threadfence_block();
            for (int base = 0; base < q; base += 64) {
              const int kk = base + lane;
              const bool v = kk < q;
              const int j = v ? (full ? kk : act[kk]) : 0;
              const double cj = v ? cc[kk] : 0.0;
              const double nr = v ? nrm2[j] : 0.0;
              bool keep = v && sphere_keep(g, cj, nr, n);
              if (keep && g.dome) keep = dome_keep(g, xty[j], cj, nr, n);
              if (v && !keep && beta[j] != 0.0) {
                beta[j] = 0.0;
                dropped = true;
              }
              const uint64_t m = ballot(keep);
              __threadfence_block();  // reads of this chunk before the writes
              if (keep) {
                act[q2 + __popcll(m & lt)] = j;
                cc[q2 + __popcll(m & lt)] = cj;
              }
              q2 += __popcll(m);
            }
            q = q2;
            full = false;
            __threadfence_block();
            if (ballot(dropped) != 0) {
              // a screened coefficient moved: rebuild the residual
              for (int i = lane; i < n; i += 64) rho[i] = (double)Y[i];
              rho_order<GRHO>();
              for (int base = 0; base < q; base += 64) {
                const int kk = base + lane;
                const int j = kk < q ? act[kk] : 0;
                const double b = kk < q ? beta[j] : 0.0;
                uint64_t m = ballot(b != 0.0);
                while (m) {
                  const int l = __builtin_ctzll(m);
                  m &= m - 1;
                  CscCol<XT> c;
                  csc_load(d, __builtin_amdgcn_readlane(j, l), lane, c);
                  csc_axpy(d, c, readlane_d(b, l), rho, lane);
                  rho_order<GRHO>();
                }
              }
            }
          }
          // f cyclic CD epochs over A (Algorithm 1), the next column's
          // nonzeros loaded while the current one is resolved
          const int ne = min(f - k % f, K - k);
          for (int e = 0; e < ne; ++e) {
            CscCol<XT> nx;
            if (q > 0) csc_load(d, act[0], lane, nx);
            for (int kk = 0; kk < q; ++kk) {
              const CscCol<XT> c = nx;
              const int j = act[kk];
              if (kk + 1 < q) csc_load(d, act[kk + 1], lane, nx);
              const double iv = inv[j];
              if (!(iv > 0.0)) continue;
              const double b = beta[j];
              const double dm = csc_dot(d, c, rho, lane);
              const double bn = soft_thr(lambda * iv, b + dm * iv);
              if (bn != b) {
                csc_axpy(d, c, bn - b, rho, lane);
                if (lane == 0) beta[j] = bn;
                rho_order<GRHO>();
              }
            }
          }
          k += ne;
          epochs_all += ne;
        }
        gbl<double>* bo = bout + (int64_t)t * p;
        for (int j = lane; j < p; j += 64) {
          const double b = beta[j];
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
      if (opts.stats && lane == 0) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&opts.stats[kStatPasses]),
                  (unsigned long long)passes);
        atomicAdd(reinterpret_cast<unsigned long long*>(&opts.stats[kStatResidualEpochs]),
                  (unsigned long long)epochs_all);
      }
    }
    if (opts.timestamps && lane == 0) {
      opts.timestamps[2 * d.orig] = t_start;
      opts.timestamps[2 * d.orig + 1] = wall_clock64();
    }
    __syncthreads();
  }
}

const void* const kCscColStats[2] = {reinterpret_cast<const void*>(&k_csc_colstats<float>),
                                     reinterpret_cast<const void*>(&k_csc_colstats<double>)};
// [dtype][residual in global memory]
const void* const kPathCsc[2][2] = {
    {reinterpret_cast<const void*>(&k_path_csc<float, false>),
     reinterpret_cast<const void*>(&k_path_csc<float, true>)},
    {reinterpret_cast<const void*>(&k_path_csc<double, false>),
     reinterpret_cast<const void*>(&k_path_csc<double, true>)}};

}  // namespace gs
