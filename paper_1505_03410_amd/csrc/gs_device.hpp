// Device helpers for the gfx950 kernels: wavefront reductions, the
// soft-threshold, column loads and the GAP SAFE test with its rounding bound.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs_internal.hpp"

namespace gs {

constexpr double kU = 1.1102230246251565e-16;  // unit roundoff of FP64, 2^-53

// A pointer read out of device memory (a problem descriptor) is generic to
// the compiler, which then emits flat instructions; those count against the
// LDS wait counter as well, so an LDS wait would also drain every prefetched
// global load.  Pointers typed in the global address space (gbl<T>*) make
// the compiler emit global_load/global_store instead.
template <typename T>
using gbl = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gbl<T>* gptr(T* p) {
  return (gbl<T>*)p;
}

// Higham's gamma_m = m u / (1 - m u): relative error bound of an m-term sum
// or dot product in FP64.
__device__ __forceinline__ double gam(double m) { return m * kU / (1.0 - m * kU); }

// ST(u, x) = sign(x) (|x| - u)_+   (Algorithm 1).
__device__ __forceinline__ double soft_thr(double u, double x) {
  return x > u ? x - u : (x < -u ? x + u : 0.0);
}

// ---- cross-lane reductions (wave64).  Butterflies give every lane of the
// group the bitwise-same result (FP addition is commutative).  Lane exchange
// uses DPP inside a row of 16 (quad_perm xor 1 and xor 2, half-row mirror,
// row mirror: once a group of 2^k lanes holds one value, the mirror pairs it
// with the neighbouring group) and the gfx950 permlane swaps across rows.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  return __hiloint2double(dpp_i<CTRL>(__double2hiint(v)), dpp_i<CTRL>(__double2loint(v)));
}
// Cross-row exchange: permlane16_swap (rows 2i <-> 2i+1) and permlane32_swap
// (lower <-> upper half) applied to (v, v) return, in every lane, the pair
// (value of the lower partner, value of the upper partner); combining a[0]
// with a[1] therefore uses the same operand order in all lanes.
__device__ __forceinline__ void swap16_d(double v, double& a, double& b) {
  auto h = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
  auto l = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
  a = __hiloint2double((int)h[0], (int)l[0]);
  b = __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ void swap32_d(double v, double& a, double& b) {
  auto h = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
  auto l = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
  a = __hiloint2double((int)h[0], (int)l[0]);
  b = __hiloint2double((int)h[1], (int)l[1]);
}

template <int S>
__device__ __forceinline__ double seg_sum(double v) {
  if constexpr (S >= 2) v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  if constexpr (S >= 4) v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  if constexpr (S >= 8) v += dpp_d<0x141>(v);   // row_half_mirror
  if constexpr (S >= 16) v += dpp_d<0x140>(v);  // row_mirror
  if constexpr (S >= 32) {
    double a, b;
    swap16_d(v, a, b);
    v = a + b;
  }
  if constexpr (S >= 64) {
    double a, b;
    swap32_d(v, a, b);
    v = a + b;
  }
  return v;
}
__device__ __forceinline__ double wave_sum(double v) { return seg_sum<64>(v); }
__device__ __forceinline__ double wave_max(double v) {
  double a, b;
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  swap16_d(v, a, b);
  v = fmax(a, b);
  swap32_d(v, a, b);
  return fmax(a, b);
}
__device__ __forceinline__ double wave_min(double v) { return -wave_max(-v); }
__device__ __forceinline__ int wave_sum_i(int v) {
  v += dpp_i<0xB1>(v);
  v += dpp_i<0x4E>(v);
  v += dpp_i<0x141>(v);
  v += dpp_i<0x140>(v);
  auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = (int)r[0] + (int)r[1];
  auto q = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return (int)q[0] + (int)q[1];
}
// Orders LDS accesses of the lanes of one wavefront (LDS instructions of a
// wave execute in issue order) without waiting for outstanding global loads.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
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
// go_nt: the same load marked non-temporal (streamed data that is read once
// should not displace cached data).
template <>
struct VecLoad<float, 4> {
  __device__ static void go_nt(const float* p, float* o) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
  __device__ static void go(const float* p, float* o) {
    float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
  __device__ static void go(const gbl<float>* p, float* o) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 v = *reinterpret_cast<const gbl<v4>*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <>
struct VecLoad<double, 2> {
  __device__ static void go_nt(const double* p, double* o) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    o[0] = v.x; o[1] = v.y;
  }
  __device__ static void go(const double* p, double* o) {
    double2 v = *reinterpret_cast<const double2*>(p);
    o[0] = v.x; o[1] = v.y;
  }
  __device__ static void go(const gbl<double>* p, double* o) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 v = *reinterpret_cast<const gbl<v2>*>(p);
    o[0] = v.x; o[1] = v.y;
  }
};
template <typename XT>
struct VecLoad<XT, 1> {
  __device__ static void go_nt(const XT* p, XT* o) { o[0] = __builtin_nontemporal_load(p); }
  __device__ static void go(const XT* p, XT* o) { o[0] = p[0]; }
  __device__ static void go(const gbl<XT>* p, XT* o) { o[0] = p[0]; }
};

// Lane layout of one column: lane (slot, seg), seg in [0,S), owns the rows
// r = (seg + S*m)*VEC + e for m < NG, e < VEC.  With a row list (gather, VEC
// must be 1) the row index comes from ridx[m].  Vector loads are only used
// when n is a multiple of VEC, so a group is either wholly inside the column
// or wholly outside it.
template <typename XT, int VEC, int S, int NG, bool GATHER>
struct ColLayout {
  static constexpr int RPL = NG * VEC;  // rows per lane
  static constexpr int C = 64 / S;      // columns per wavefront step
  static constexpr int NMAX = S * NG * VEC;
  static_assert(RPL <= 64, "row mask holds 64 rows per lane");

  __device__ static __forceinline__ int row(int seg, int m, int e) {
    return (seg + S * m) * VEC + e;
  }

  // Bit (m*VEC + e) is set when that row of the lane is < n.  Constant per
  // lane: loads are issued unmasked and the mask is applied where the values
  // are used, so that a prefetched load is not waited for early.
  __device__ static __forceinline__ uint64_t rowmask(int seg, int n) {
    uint64_t mk = 0;
#pragma unroll
    for (int m = 0; m < NG; ++m)
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        if (row(seg, m, e) < n) mk |= 1ull << (m * VEC + e);
    return mk;
  }

  // Issues the loads of the lane's rows of column `col`; groups beyond row
  // n-1 read row 0 instead (their values are masked at use).  ridx holds the
  // clamped source rows of a gather.
  template <typename P>
  __device__ static __forceinline__ void load_raw(P col, int n, int seg, const int* ridx,
                                                  XT (&xv)[RPL]) {
#pragma unroll
    for (int m = 0; m < NG; ++m) {
      if constexpr (GATHER) {
        xv[m] = col[ridx[m]];
      } else {
        const int r0 = (seg + S * m) * VEC;
        VecLoad<XT, VEC>::go(col + (r0 < n ? r0 : 0), &xv[m * VEC]);
      }
    }
  }

  // load_raw for a column that is streamed once (non-temporal loads; no row
  // list).
  __device__ static __forceinline__ void load_raw_nt(const XT* col, int n, int seg,
                                                     XT (&xv)[RPL]) {
#pragma unroll
    for (int m = 0; m < NG; ++m) {
      const int r0 = (seg + S * m) * VEC;
      VecLoad<XT, VEC>::go_nt(col + (r0 < n ? r0 : 0), &xv[m * VEC]);
    }
  }

  __device__ static __forceinline__ double at(const XT (&xv)[RPL], uint64_t mk, int i) {
    return ((mk >> i) & 1ull) ? (double)xv[i] : 0.0;
  }

  // Masked load (values usable at once).
  template <typename P>
  __device__ static __forceinline__ void load(P col, int n, int seg, const int* ridx,
                                              uint64_t mk, XT (&xv)[RPL]) {
    load_raw(col, n, seg, ridx, xv);
#pragma unroll
    for (int i = 0; i < RPL; ++i) xv[i] = ((mk >> i) & 1ull) ? xv[i] : XT(0);
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
//   errG  bounds the rounding in G plus the gap between rho~ and y - X beta;
//         the computed Ry may be off by gamma_n ||y|| ||rho~|| whatever its
//         own size (its terms have both signs), which enters G through
//         lambda |alpha| Ry
//   r+    = sqrt(2 (max(G,0) + errG)) / lambda (1 + 4u)   (Proposition 1)
// The sphere test then keeps j iff
//   |alpha c^_j| + |alpha| e_c ||x_j||+ + r+ ||x_j||+ >= 1 - 4u    (Sec. 2.1)
//
// GAP SAFE dome (Sec. 3.2; dome support function of the appendix), the ball
// of diameter [theta, y/lambda] cut by the plane through its intersection
// with the sphere of radius r_check[beta] around y/lambda, normal
// w = (y/lambda - theta)/R_hat, R_hat = ||theta - y/lambda||.  Its safe
// parameters enlarge the dome by the rounding of the inputs: R_hat between
// Rlo and Rhi (R_hat^2 = alpha^2 R2 - 2 alpha Ry/lambda + ||y||^2/lambda^2),
// rc2lo a lower bound of r_check^2 = (||y||^2 - ||y - X beta||^2 -
// 2 lambda ||beta||_1)_+/lambda^2, e_y the error of x_j^T y/lambda per
// unit ||x_j||.
struct GapInfo {
  double alpha, gap, radius, e_c;
  double lambda, Rlo, Rhi, rc2lo, e_y;
  bool dome;
  // comparison rules (Table 1), rule 2-4: sphere test with center term
  // x_j^T y/lambda - shift x_j^T x_{j*} and radius rad_s (rounding-safe)
  int rule;
  double shift, rad_s, e_shift, nstar;
};

__device__ __forceinline__ GapInfo gap_safe(double R2, double Ry, double l1, double sbx,
                                            double xmax, double M, int nnz, int n,
                                            double lambda, double ynorm, int q = 0,
                                            bool dome = false, bool rule_ball = false) {
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
  const double errG = gam(n + 6) * (t1 + t2 + fabs(t3) + t4) +
                      lambda * fabs(a) * gam(n) * (ynorm * up) * rnorm + rnorm * drho +
                      0.5 * drho * drho;
  g.radius = sqrt(2.0 * (fmax(g.gap, 0.0) + errG)) / lambda * (1.0 + 4.0 * kU);
  g.lambda = lambda;
  g.dome = dome;
  g.rule = dome ? 1 : 0;
  g.shift = g.rad_s = g.e_shift = g.nstar = 0.0;
  g.Rlo = g.Rhi = g.rc2lo = g.e_y = 0.0;
  if (dome || rule_ball) {
    const double yy = ynorm * ynorm, il = 1.0 / lambda, il2 = il * il;
    const double yn = ynorm * up;
    const double Rs2 = a * a * R2 - 2.0 * a * Ry * il + yy * il2;
    const double eR2 = gam(n + 6) * (a * a * R2 + 2.0 * fabs(a * Ry) * il + yy * il2) +
                       2.0 * fabs(a) * il * gam(n) * yn * rnorm;
    g.Rhi = sqrt(fmax(Rs2 + eR2, 0.0)) * (1.0 + 4.0 * kU);
    g.Rlo = sqrt(fmax(Rs2 - eR2, 0.0)) * (1.0 - 4.0 * kU);
    const double rt = rnorm + drho;  // bounds ||y - X beta||
    g.rc2lo = fmax((yy * (1.0 - gam(n + 2)) - rt * rt * (1.0 + 4.0 * kU) -
                    2.0 * lambda * l1 * (1.0 + gam(q + 2))) * il2 * (1.0 - 4.0 * kU),
                   0.0);
    g.e_y = gam(n + 1) * yn * il;
  }
  return g;
}

// The comparison rules of Table 1 as sphere tests (rule 2 static SAFE:
// B(y/lambda, ||y|| |1/lambda - 1/lambda_max|); rule 3 Dynamic Safe:
// B(y/lambda, R_hat); rule 4 Dynamic ST3: B(y/lambda, R_hat) cut by the plane
// s* x*^T t = 1, held in the ball around the projection of y/lambda on it:
// center y/lambda - shift x*, shift = s* (lambda_max/lambda - 1)/||x*||^2,
// radius (R_hat^2 - d^2)^(1/2), d = (lambda_max/lambda - 1)/||x*||).  The
// radius is rounding-safe (R_hat by Rhi, lambda_max and d by lower bounds);
// e_shift bounds the error of the computed shift per unit ||x_j||.
__device__ __forceinline__ void rule_ball(GapInfo& g, int rule, double lmax, double sstar,
                                          double nstar, double ynorm, int n) {
  g.rule = rule;
  g.nstar = nstar;
  const double yn = ynorm * (1.0 + gam(n + 2));
  const double e_lm = gam(n + 1) * nstar * yn;
  const double lambda = g.lambda;
  if (rule == 2) {
    g.rad_s = yn *
              (fabs(1.0 / lambda - 1.0 / lmax) +
               (lmax > e_lm ? e_lm / (lmax * (lmax - e_lm)) : INFINITY)) *
              (1.0 + 4.0 * kU);
  } else if (rule == 3 || !(lambda < lmax)) {
    g.rad_s = g.Rhi;
  } else {
    const double ratio = lmax / lambda - 1.0;
    g.shift = sstar * ratio / (nstar * nstar);
    const double dlo = fmax(((lmax - e_lm) / lambda - 1.0) / (nstar * (1.0 + gam(n + 2))), 0.0);
    g.rad_s = sqrt(fmax(g.Rhi * g.Rhi * (1.0 + 4.0 * kU) - dlo * dlo * (1.0 - 4.0 * kU), 0.0)) *
              (1.0 + 4.0 * kU);
    g.e_shift = (e_lm / lambda / (nstar * nstar) + 8.0 * kU * fabs(g.shift)) * nstar;
  }
}

__device__ __forceinline__ bool rule_keep(const GapInfo& g, double xty, double gj, double nrm2,
                                          int n) {
  if (!(nrm2 > 0.0)) return false;
  const double xn = sqrt(nrm2) * (1.0 + gam(n + 2));
  const double yl = xty / g.lambda, sg = g.shift * gj;
  const double cx = yl - sg;
  const double e = g.e_y * xn + g.e_shift * xn + fabs(g.shift) * gam(n + 1) * xn * g.nstar +
                   4.0 * kU * (fabs(yl) + fabs(sg));
  return fabs(cx) + e + g.rad_s * xn >= 1.0 - 4.0 * kU;
}

// Support function of the dome at x given c^T x (cx), w^T x (wx) and ||x||:
// the ball's maximizer c + r x/||x|| when it lies on the kept side of the
// plane (w^T x <= -ra ||x||), else the best point of the circle where the
// plane cuts the sphere.  Non-increasing in wx.
__device__ __forceinline__ double dome_sigma(double cx, double wx, double xn, double r,
                                             double ra) {
  if (wx <= -ra * xn) return cx + r * xn;
  return cx - r * ra * wx + r * sqrt(fmax((xn * xn - wx * wx) * (1.0 - ra * ra), 0.0));
}

// The dome test for column j (keep iff max(sigma(x_j), sigma(-x_j)) >= 1),
// with every input replaced by the bound that enlarges the dome: Rhi for the
// ball, rc2lo for the plane, an upper bound of c^T x, a lower bound of w^T x
// and of ||x||'s upper bound, plus a margin for the evaluation.
__device__ __forceinline__ bool dome_keep(const GapInfo& g, double xty, double c, double nrm2,
                                          int n) {
  if (!g.dome) return true;
  if (!(nrm2 > 0.0)) return false;
  if (!(g.Rhi > 0.0)) return true;
  const double xn = sqrt(nrm2) * (1.0 + gam(n + 2));
  const double r = 0.5 * g.Rhi;
  const double ra = fmax(2.0 * g.rc2lo / (g.Rhi * g.Rhi) - 1.0, -1.0);
  const double yl = xty / g.lambda, ac = g.alpha * c;
  const double cx = 0.5 * (yl + ac), num = yl - ac;
  const double ey = g.e_y * xn, eac = fabs(g.alpha) * g.e_c * xn;
  const double ro = 4.0 * kU * (fabs(yl) + fabs(ac));
  const double ecx = 0.5 * (ey + eac) + ro, ewn = ey + eac + ro;
  double mu = -INFINITY;
#pragma unroll
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    const double cs = sgn * cx + ecx;
    const double ns = sgn * num - ewn;
    double m;
    if (ns >= 0.0)
      m = dome_sigma(cs, ns / g.Rhi, xn, r, ra);
    else if (g.Rlo > 0.0)
      m = dome_sigma(cs, ns / g.Rlo, xn, r, ra);
    else
      m = cs + r * xn;
    mu = fmax(mu, m);
  }
  return mu >= 1.0 - 16.0 * kU * (fabs(cx) + 3.0 * r * xn + 1.0);
}

__device__ __forceinline__ bool sphere_keep(const GapInfo& g, double c, double nrm2, int n) {
  if (!(nrm2 > 0.0)) return false;
  const double xn = sqrt(nrm2) * (1.0 + gam(n + 2));
  const double mu = fabs(g.alpha * c) + fabs(g.alpha) * g.e_c * xn + g.radius * xn;
  return mu >= 1.0 - 4.0 * kU;
}

}  // namespace gs
