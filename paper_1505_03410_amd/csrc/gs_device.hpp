// Device helpers for the gfx950 kernels: wavefront reductions, the
// soft-threshold, column loads and the GAP SAFE test with its rounding bound.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs_internal.hpp"

namespace gs {

constexpr double kU = 1.1102230246251565e-16;  // unit roundoff of FP64, 2^-53

// Higham's gamma_m = m u / (1 - m u): relative error bound of an m-term sum
// or dot product in FP64.
__device__ __forceinline__ double gam(double m) { return m * kU / (1.0 - m * kU); }

// ST(u, x) = sign(x) (|x| - u)_+   (Algorithm 1).
__device__ __forceinline__ double soft_thr(double u, double x) {
  return x > u ? x - u : (x < -u ? x + u : 0.0);
}

// ---- cross-lane reductions (wave64).  Butterflies give every lane of the
// group the bitwise-same result (FP addition is commutative).
template <int S>
__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
  for (int o = S / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) { return seg_sum<64>(v); }
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ uint64_t ballot(bool b) { return __ballot(b); }

// ---- vector types for 16-byte loads
template <typename XT, int VEC>
struct VecLoad;
template <>
struct VecLoad<float, 4> {
  __device__ static void go(const float* p, float* o) {
    float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <>
struct VecLoad<double, 2> {
  __device__ static void go(const double* p, double* o) {
    double2 v = *reinterpret_cast<const double2*>(p);
    o[0] = v.x; o[1] = v.y;
  }
};
template <typename XT>
struct VecLoad<XT, 1> {
  __device__ static void go(const XT* p, XT* o) { o[0] = p[0]; }
};

// Lane layout of one column: lane (slot, seg), seg in [0,S), owns the rows
// r = (seg + S*m)*VEC + e for m < NG, e < VEC.  With a row list (gather, VEC
// must be 1) the row index comes from ridx[m].
template <typename XT, int VEC, int S, int NG, bool GATHER>
struct ColLayout {
  static constexpr int RPL = NG * VEC;  // rows per lane
  static constexpr int C = 64 / S;      // columns per wavefront step
  static constexpr int NMAX = S * NG * VEC;

  __device__ static __forceinline__ int row(int seg, int m, int e) {
    return (seg + S * m) * VEC + e;
  }

  // Loads the lane's rows of column `col` (pointer to its first entry).
  // Entries at rows >= n are 0; no entry beyond row n-1 is read.
  __device__ static __forceinline__ void load(const XT* __restrict__ col, int n, int seg,
                                              const int* ridx, XT (&xv)[RPL]) {
#pragma unroll
    for (int m = 0; m < NG; ++m) {
      if constexpr (GATHER) {
        int r = ridx[m];
        xv[m] = (r >= 0) ? col[r] : XT(0);
      } else {
        const int r0 = (seg + S * m) * VEC;
        if (r0 + VEC <= n) {
          VecLoad<XT, VEC>::go(col + r0, &xv[m * VEC]);
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) xv[m * VEC + e] = (r0 + e < n) ? col[r0 + e] : XT(0);
        }
      }
    }
  }
};

// ---- GAP SAFE sphere with the stated rounding bound -------------------------
//
// Inputs are the FP64 reductions of one screening pass on the refreshed
// residual rho~ of beta: R2 = ||rho~||^2, Ry = y^T rho~, l1 = ||beta||_1,
// sbx = sum_j |beta_j| ||x_j||, xmax = max_{j in A} ||x_j||, M = max_{j in A}
// |x_j^T rho~| (computed), nnz = #nonzeros of beta.
//   e_c   bounds |c^_j - x_j^T rho~| / ||x_j||             (gamma_{n+1} ||rho~||)
//   M+    = (M + e_c xmax+)(1 + 4u) makes theta = alpha rho~ dual feasible on A
//   alpha = clip(Ry / (lambda R2), -1/M+, 1/M+)           (Sec. 2.3)
//   G     = 1/2 R2 + lambda l1 - lambda alpha Ry + 1/2 lambda^2 alpha^2 R2
//         = P(beta) - D(theta) with the 1/2||y||^2 terms cancelled analytically
//   errG  bounds the rounding in G plus the gap between rho~ and y - X beta
//   r+    = sqrt(2 (max(G,0) + errG)) / lambda (1 + 4u)   (Proposition 1)
// The sphere test then keeps j iff
//   |alpha c^_j| + |alpha| e_c ||x_j||+ + r+ ||x_j||+ >= 1 - 4u    (Sec. 2.1)
struct GapInfo {
  double alpha, gap, radius, e_c;
};

__device__ __forceinline__ GapInfo gap_safe(double R2, double Ry, double l1, double sbx,
                                            double xmax, double M, int nnz, int n,
                                            double lambda, double ynorm) {
  GapInfo g;
  const double up = 1.0 + gam(n + 2);
  const double rnorm = sqrt(R2) * up;
  g.e_c = gam(n + 1) * rnorm;
  const double Mp = (M + g.e_c * xmax * up) * (1.0 + 4.0 * kU);
  double a = (R2 > 0.0) ? Ry / (lambda * R2) : 0.0;  // no active column: unclipped
  if (Mp > 0.0) {
    a = fmax(a, -1.0 / Mp);
    a = fmin(a, 1.0 / Mp);
  }
  g.alpha = a;
  const double t1 = 0.5 * R2, t2 = lambda * l1, t3 = lambda * a * Ry,
               t4 = 0.5 * lambda * lambda * a * a * R2;
  g.gap = t1 + t2 - t3 + t4;
  const double drho = gam(nnz + 1) * (ynorm + sbx * up);
  const double errG = gam(n + 6) * (t1 + t2 + fabs(t3) + t4) + rnorm * drho + 0.5 * drho * drho;
  g.radius = sqrt(2.0 * (fmax(g.gap, 0.0) + errG)) / lambda * (1.0 + 4.0 * kU);
  return g;
}

__device__ __forceinline__ bool sphere_keep(const GapInfo& g, double c, double nrm2, int n) {
  if (!(nrm2 > 0.0)) return false;
  const double xn = sqrt(nrm2) * (1.0 + gam(n + 2));
  const double mu = fabs(g.alpha * c) + fabs(g.alpha) * g.e_c * xn + g.radius * xn;
  return mu >= 1.0 - 4.0 * kU;
}

}  // namespace gs
