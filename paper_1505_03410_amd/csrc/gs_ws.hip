// The restricted solve of the learned start.  On a working set W of columns
// with a sign pattern sigma, the Lasso's optimality conditions (Sec. 2: the
// subgradient of ||beta||_1 is sign(beta_j) on the support) reduce to the
// linear system
//     (X_W^T X_W) b = X_W^T y - lambda sigma,
// whose solution is the Lasso solution at lambda whenever W holds the
// support, sigma its signs, b has those signs and every other column's
// correlation stays within lambda.  The system is solved in FP64 by a blocked
// Cholesky factorization (64 x 64 tiles): the Gram matrix of W (products of
// the stored values, exact in FP64), then per tile column a factorization of
// the diagonal tile, a triangular solve of the tiles below it and an update of
// the trailing tiles, then the backward triangular solve.  The matrix is M x M
// with M = m rounded up to 64 and the identity on the padding, stored column
// major with M + 64 rows: the right-hand side b is row M (rows M + 1 .. M + 63
// are zero), an extra tile row that the factorization treats like the others,
// so that it leaves z = L^{-1} b in that row (the forward substitution comes
// with the panel and update steps).  The factor L lives in the lower triangle
// and its transpose is mirrored into the upper triangle so that the backward
// solve reads columns.
//
// Around it, the working-set kernels of the learned path driver: the initial
// set from the network's support logits, dropping coordinates whose sign
// disagrees with sigma, the largest violators of |x_j^T rho| <= lambda added,
// and the scatter of b into a p-vector.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "../../include/gapsafe.h"
#include "gs_device.hpp"
#include "gs_internal.hpp"

namespace gs {
namespace {

static_assert(kWsMaxSet == GS_WS_MAX, "working-set limit of the C ABI");
constexpr int TB = 64;  // tile size

__device__ __forceinline__ bool ws_failed(const int32_t* info) { return *info != 0; }

// ---- Gram tiles: block (I, J, s), I >= J, computes G[I-tile rows][J-tile
// cols] over the rows [s R, min(n, (s + 1) R)); rows pass through LDS 32 at a
// time, the next 32 loaded into registers while the current ones are used.
// With one split (gridDim.y = 1) the tile goes to G with the identity on the
// padding; otherwise the raw partial sum goes to the split's own M x M slice
// of out, and k_ws_gram_sum adds the slices.
template <typename XT>
__global__ __launch_bounds__(256) void k_ws_gram(const XT* __restrict__ X, int64_t ldx, int n,
                                                 int p, const int32_t* __restrict__ W, int m,
                                                 int M, int R, double* __restrict__ out) {
  constexpr int RC = 32;
  constexpr int NL = (RC * TB) / 256;  // loads per thread and operand per chunk
  __shared__ double A[RC][TB + 1], B[RC][TB + 1];
  __shared__ int64_t ca[TB], cb[TB];
  // tile (I, J) from the block index: lower tiles in column order
  int b = blockIdx.x, J = 0;
  const int NT = M / TB;
  while (b >= NT - J) {
    b -= NT - J;
    ++J;
  }
  const int I = J + b;
  const int t = threadIdx.x;
  if (t < TB) {
    const int a = I * TB + t;
    ca[t] = a < m ? (int64_t)min(max(W[a], 0), p - 1) * ldx : -1;
  } else if (t < 2 * TB) {
    const int a = J * TB + (t - TB);
    cb[t - TB] = a < m ? (int64_t)min(max(W[a], 0), p - 1) * ldx : -1;
  }
  __syncthreads();
  // this thread's (column, row) slots of a chunk: 64 columns x 32 rows,
  // consecutive threads on consecutive rows
  int64_t oa[NL], ob[NL];
  int rr[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int e = t + 256 * i;
    rr[i] = e % RC;
    oa[i] = ca[e / RC];
    ob[i] = cb[e / RC];
  }
  // loads with the address clamped into X (a padding column reads X[0]); the
  // value is masked when it reaches LDS
  XT va[NL], vb[NL];
  auto load = [&](int r0) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int r = min(r0 + rr[i], n - 1);
      va[i] = X[oa[i] >= 0 ? oa[i] + r : 0];
      vb[i] = X[ob[i] >= 0 ? ob[i] + r : 0];
    }
  };
  const int ta = t >> 4, tb = t & 15;  // this thread's 4 x 4 entries
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  const int rbeg = blockIdx.y * R, rend = min(n, rbeg + R);
  load(rbeg);
  for (int r0 = rbeg; r0 < rend; r0 += RC) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int e = t + 256 * i;
      const bool in = r0 + rr[i] < rend;
      A[rr[i]][e / RC] = (oa[i] >= 0 && in) ? (double)va[i] : 0.0;
      B[rr[i]][e / RC] = (ob[i] >= 0 && in) ? (double)vb[i] : 0.0;
    }
    __syncthreads();
    if (r0 + RC < rend) load(r0 + RC);
#pragma unroll 4
    for (int q = 0; q < RC; ++q) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = A[q][ta * 4 + u];
        bv[u] = B[q][tb * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
    }
    __syncthreads();
  }
  const bool split = gridDim.y > 1;
  double* G = out + (split ? (size_t)blockIdx.y * M * M : 0);
  const int64_t ldo = split ? M : M + TB;  // slices are M x M, G has M + 64 rows
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ga = I * TB + ta * 4 + u, gb = J * TB + tb * 4 + v;
      double val = acc[u][v];
      if (!split && (ga >= m || gb >= m)) val = ga == gb ? 1.0 : 0.0;
      G[gb * ldo + ga] = val;
    }
}

// G (M + 64 rows) = the sum of the S slices of P (M x M each) on the tiles
// I >= J, the identity on the padding.
__global__ void k_ws_gram_sum(const double* __restrict__ P, int S, int M, int m,
                              double* __restrict__ G) {
  const int64_t MM = (int64_t)M * M;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < MM;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % M), b = (int)(e / M);
    if (a / TB < b / TB) continue;
    double v;
    if (a >= m || b >= m) {
      v = a == b ? 1.0 : 0.0;
    } else {
      v = 0.0;
      for (int k = 0; k < S; ++k) v += P[k * MM + e];
    }
    G[(int64_t)b * (M + TB) + a] = v;
  }
}

// row splits of the Gram product: enough blocks for the chip's 256 compute
// units, at most 8, each split at least 64 rows
int gram_splits(int NT, int n) {
  const int ntile = NT * (NT + 1) / 2;
  int S = std::max(1, std::min(8, 256 / ntile));
  return std::max(1, std::min(S, n / 64));
}
// ---- right-hand side b_a = x_{W_a}^T y - lambda sigma_a (0 on the padding)
// into row M of G, with rows M + 1 .. M + 63 of column a set to zero; one
// wavefront per entry; an index outside [0, p) sets info = -1.
template <typename XT>
__global__ __launch_bounds__(256) void k_ws_rhs(const XT* __restrict__ X, int64_t ldx, int n, int p,
                                                const XT* __restrict__ y,
                                                const int32_t* __restrict__ W,
                                                const double* __restrict__ sigma, int m, int M,
                                                double lambda, double* __restrict__ G,
                                                int32_t* info) {
  const int lane = threadIdx.x & 63;
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a >= M) return;
  double* b = G + (int64_t)a * (M + TB) + M;  // rows M .. M + 63 of column a
  if (lane > 0) b[lane] = 0.0;
  if (a >= m) {
    if (lane == 0) b[0] = 0.0;
    return;
  }
  const int j0 = W[a];
  if (j0 < 0 || j0 >= p) {
    if (lane == 0) *info = -1;
    return;
  }
  const XT* col = X + (int64_t)j0 * ldx;
  double s = 0.0;
  for (int i = lane; i < n; i += 64) s = fma((double)col[i], (double)y[i], s);
  s = wave_sum(s);
  if (lane == 0) b[0] = s - lambda * sigma[a];
}

// ---- factorization of the diagonal tile K (unblocked, right-looking) by 256
// threads: four per row, thread (i, q) holding the entries T_ij, j = q mod 4,
// of row i in registers.  Column c stays unscaled (T_ic = L_ic L_cc, T_cc =
// L_cc^2) while the trailing entries take T_ij -= (T_ic / T_cc) T_jc, so a
// step needs only column c, which its owners (q = c mod 4) put in LDS before
// the step's single barrier (two buffers alternate, so the next step's writes
// cannot meet this step's reads); L is formed from the unscaled columns at
// the end.  Writes L_KK to the lower triangle and its transpose to the upper
// one.  A pivot that is not a positive normal number stops the factorization
// with info = its 1-based row.
__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ G, int M, int K,
                                                   int32_t* info) {
  __shared__ double col[2][TB];
  if (ws_failed(info)) return;
  const int t = threadIdx.x;
  const int i = t >> 2, qd = t & 3;
  const int64_t o = (int64_t)K * TB, ld = M + TB;
  double a[TB / 4];   // T_{i, 4u + qd}
  double pv[TB / 4];  // the unscaled pivot T_jj of each column j = 4u + qd
#pragma unroll
  for (int u = 0; u < TB / 4; ++u) {
    a[u] = G[(o + 4 * u + qd) * ld + o + i];
    pv[u] = 1.0;
  }
#pragma unroll
  for (int c = 0; c < TB; ++c) {
    const int uc = c >> 2, qc = c & 3;
    double* cb = col[c & 1];
    if (qd == qc) cb[i] = a[uc];
    __syncthreads();
    const double piv = cb[c];
    if (!(piv >= 2.2250738585072014e-308) || !isfinite(piv)) {  // uniform value
      if (t == 0) *info = (int32_t)(o + c + 1);
      return;
    }
    if (qd == qc) pv[uc] = piv;
    // 1 / piv by the hardware reciprocal and two Newton steps (error under
    // 2 ulp for a normal pivot)
    double r = __builtin_amdgcn_rcp(piv);
    r = fma(r, fma(-piv, r, 1.0), r);
    r = fma(r, fma(-piv, r, 1.0), r);
    const double f = cb[i] * r;
    // the entries j > c: all of u > uc, and j = 4 uc + q for q > qc
    {
      const double nv = fma(-f, cb[4 * uc + qd], a[uc]);
      a[uc] = qd > qc ? nv : a[uc];
    }
#pragma unroll
    for (int u = uc + 1; u < TB / 4; ++u) a[u] = fma(-f, cb[4 * u + qd], a[u]);
    // the updated entries are materialized here: left to itself the compiler
    // defers these products toward their next use and keeps every step's
    // factor live, which spills
#pragma unroll
    for (int u = uc; u < TB / 4; ++u) asm volatile("" : "+v"(a[u]));
  }
#pragma unroll
  for (int u = 0; u < TB / 4; ++u) {
    const int j = 4 * u + qd;
    if (i >= j) {
      const double d = sqrt(pv[u]);
      const double v = i == j ? d : a[u] / d;
      G[(o + j) * ld + o + i] = v;
      G[(o + i) * ld + o + j] = v;
    }
  }
}

// value of lane Q of each group of four lanes, by a DPP quad permutation
template <int Q>
__device__ __forceinline__ double quad_bcast(double v) {
  constexpr int ctrl = Q | (Q << 2) | (Q << 4) | (Q << 6);
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double quad_bcast(double v, int q) {
  switch (q) {
    case 0: return quad_bcast<0>(v);
    case 1: return quad_bcast<1>(v);
    case 2: return quad_bcast<2>(v);
    default: return quad_bcast<3>(v);
  }
}

// ---- tiles below the diagonal: L_IK = G_IK L_KK^{-T}, one block per tile
// row I > K up to the right-hand side's tile row I = M / 64 (which has no
// mirror in the upper triangle), four threads per row of the tile: thread (r, q) holds the
// entries x_c, c = q mod 4, of row r.  Right-looking: at step c the owner of
// x_c divides it by L_cc, its three neighbours get it by a quad broadcast, and
// every thread subtracts x_c L_jc from its entries j > c.  A row's four
// threads are neighbouring lanes of one wavefront, so the steps need no
// barrier.
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ G, int M, int K,
                                                   int32_t* info) {
  __shared__ double Lt[TB][TB + 1];  // Lt[c][j] = L_jc
  __shared__ double rd[TB];          // 1 / L_cc
  if (ws_failed(info)) return;
  const int t = threadIdx.x;
  const int r = t >> 2, qd = t & 3;
  const int I = K + 1 + blockIdx.x;
  const int64_t o = (int64_t)K * TB, oi = (int64_t)I * TB, ld = M + TB;
  const bool mirror = oi < M;
#pragma unroll
  for (int k = 0; k < TB * TB / 256; ++k) {
    const int e = t + 256 * k;
    const int j = e % TB, c = e / TB;
    Lt[c][j] = G[(o + c) * ld + o + j];
  }
  if (t < TB) rd[t] = 1.0 / G[(o + t) * ld + o + t];
  double x[TB / 4];  // G_IK[r][4u + qd], then L_IK[r][4u + qd]
#pragma unroll
  for (int u = 0; u < TB / 4; ++u) x[u] = G[(o + 4 * u + qd) * ld + oi + r];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < TB; ++c) {
    const int uc = c >> 2, qc = c & 3;
    const double own = x[uc] * rd[c];  // meaningful on the owner, q = qc
    if (qd == qc) x[uc] = own;
    const double xc = quad_bcast(own, qc);
    {
      const double nv = fma(-xc, Lt[c][4 * uc + qd], x[uc]);
      x[uc] = qd > qc ? nv : x[uc];
    }
#pragma unroll
    for (int u = uc + 1; u < TB / 4; ++u) x[u] = fma(-xc, Lt[c][4 * u + qd], x[u]);
    // materialized here, as in the diagonal kernel
#pragma unroll
    for (int u = uc; u < TB / 4; ++u) asm volatile("" : "+v"(x[u]));
  }
#pragma unroll
  for (int u = 0; u < TB / 4; ++u) {
    G[(o + 4 * u + qd) * ld + oi + r] = x[u];
    if (mirror) G[(oi + r) * ld + o + 4 * u + qd] = x[u];
  }
}

// ---- trailing update G_IJ -= L_IK L_JK^T for K < J <= I < M / 64, one block
// per tile, then the right-hand side's tiles I = M / 64, K < J < M / 64.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ G, int M, int K,
                                                     int32_t* info) {
  __shared__ double A[TB][TB + 1], B[TB][TB + 1];
  if (ws_failed(info)) return;
  const int NT = M / TB;
  const int T = NT - K - 1;
  int b = blockIdx.x, I, J;
  if (b >= T * (T + 1) / 2) {
    I = NT;
    J = K + 1 + (b - T * (T + 1) / 2);
  } else {
    int jj = 0;
    while (b >= T - jj) {
      b -= T - jj;
      ++jj;
    }
    J = K + 1 + jj;
    I = J + b;
  }
  const int t = threadIdx.x;
  const int64_t o = (int64_t)K * TB, oi = (int64_t)I * TB, oj = (int64_t)J * TB, ld = M + TB;
  const int ta = t >> 4, tb = t & 15;
  // this thread's 4 x 4 entries of G_IJ, read with the operands (a store
  // after each read would keep the reads from overlapping)
  double g[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) g[u][v] = G[(oj + tb * 4 + v) * ld + oi + ta * 4 + u];
#pragma unroll
  for (int h = 0; h < TB * TB / 256; ++h) {
    const int e = t + 256 * h;
    const int i = e % TB, k = e / TB;
    A[i][k] = G[(o + k) * ld + oi + i];
    B[i][k] = G[(o + k) * ld + oj + i];
  }
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll 8
  for (int k = 0; k < TB; ++k) {
    double av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = A[ta * 4 + u][k];
      bv[u] = B[tb * 4 + u][k];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      G[(oj + tb * 4 + v) * ld + oi + ta * 4 + u] = g[u][v] - acc[u][v];
    }
}

// ---- L^T x = z, one block, with z = L^{-1} b left in row M by the
// factorization; x_out gets the first m entries.  Blocked by tiles of 64,
// bottom to top: the diagonal tile's 64 steps run on wavefront 0 (lane i owns
// entry i of the tile, the tile of L in LDS), then every thread applies the
// tile's columns to the entries above it.  L_cj for j < c is column c of the
// mirrored upper triangle, so the sweep reads columns.
constexpr int kSolveThreads = 1024;
// acc - sum_c G[g + c ld] zt[c] over the 64 entries c of a tile, the loads of
// G issued 16 at a time ahead of their use (G holds at most 2048 x 2112
// entries, so 32-bit indices)
__device__ __forceinline__ double tile_dot(const double* __restrict__ G, int g, int ld,
                                           const double* zt, double acc) {
#pragma unroll
  for (int h = 0; h < TB; h += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = G[g + (h + u) * ld];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 16; ++u) acc = fma(-v[u], zt[h + u], acc);
  }
  return acc;
}
__global__ __launch_bounds__(kSolveThreads) void k_chol_solve(const double* __restrict__ G, int M,
                                                              int m, double* __restrict__ x_out,
                                                              int32_t* info) {
  __shared__ double z[2048];
  __shared__ double L[TB][TB + 1];
  if (ws_failed(info)) return;
  const int t = threadIdx.x;
  const int NT = M / TB;
  const int ld = M + TB;
  for (int i = t; i < M; i += kSolveThreads) z[i] = G[(int64_t)i * ld + M];
  for (int K = NT - 1; K >= 0; --K) {
    const int64_t o = (int64_t)K * TB;
    __syncthreads();  // z and the previous tile's use of L are complete
#pragma unroll
    for (int k = 0; k < TB * TB / kSolveThreads; ++k) {
      const int e = t + kSolveThreads * k;
      const int i = e % TB, j = e / TB;
      L[i][j] = G[(o + j) * ld + o + i];
    }
    __syncthreads();
    if (t < TB) {
      double zi = z[o + t];
      const double ri = 1.0 / L[t][t];
      for (int c0 = TB - 8; c0 >= 0; c0 -= 8) {
        double lv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) lv[u] = L[c0 + u][t];
#pragma unroll
        for (int u = 7; u >= 0; --u) {
          // lane c's entry is final at step c; the others read it by readlane
          const int c = c0 + u;
          const double xc = readlane_d(zi * ri, c);
          const double nz = fma(-lv[u], xc, zi);
          zi = t == c ? xc : (t < c ? nz : zi);
        }
      }
      z[o + t] = zi;
    }
    __syncthreads();
    // rows above the tile: z_j -= sum_c L_{o+c, j} x_{o+c} (upper triangle)
    for (int j = t; j < (int)o; j += kSolveThreads)
      z[j] = tile_dot(G, (int)o * ld + j, ld, z + o, z[j]);
  }
  __syncthreads();
  for (int i = t; i < m; i += kSolveThreads) x_out[i] = z[i];
}

// ---- working-set kernels of the learned driver (one block each unless
// stated).  cnt[0] = |W|; mark (p int32) flags the members of W.

// Counts over the positions of act (q of them): cnt[0] = members of the
// support of beta_prev, cnt[1 + i] = the others that violate the optimality
// conditions at beta_prev (|c_j| > lambda, c indexed by column) and whose
// support logit o1 > taus[i], i < kWsTaus.
constexpr int kWsTaus = 7;
// chunks of 1024 positions per step of the single-block scans below: their
// loads are issued together, so a step costs one or two memory latencies
constexpr int kWsScan = 8;
static_assert(kWsScan * 16 == 128, "two table entries per lane");
// inclusive prefix sum over the 64 lanes of a wavefront
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(v, d, 64);
    v += lane >= d ? o : 0;
  }
  return v;
}
// ordered compaction of those scans: with the kept count of every wave x and
// chunk u in wc[u][x] (after a barrier), off[u] = base plus everything kept
// before wave w's part of chunk u; returns base plus everything kept.  Each
// wavefront scans the 128 counts in (u, x) order itself, two per lane.
__device__ __forceinline__ int ws_chunk_offs(const int (*wc)[16], int w, int base,
                                             int (&off)[kWsScan]) {
  const int lane = threadIdx.x & 63;
  const int v0 = wc[lane >> 4][lane & 15], v1 = wc[4 + (lane >> 4)][lane & 15];
  const int s0 = wave_incl_scan(v0), s1 = wave_incl_scan(v1);
  const int t0 = __builtin_amdgcn_readlane(s0, 63), t1 = __builtin_amdgcn_readlane(s1, 63);
  const int e0 = s0 - v0, e1 = t0 + s1 - v1;  // exclusive prefixes
  const int wu = __builtin_amdgcn_readfirstlane(w);
#pragma unroll
  for (int u = 0; u < kWsScan; ++u) {
    const int e = u * 16 + wu;
    off[u] = base + (u < 4 ? __builtin_amdgcn_readlane(e0, e) : __builtin_amdgcn_readlane(e1, e - 64));
  }
  return base + t0 + t1;
}
// sum of the 128 entries of such a table, by every wavefront
__device__ __forceinline__ int ws_table_sum(const int (*tb)[16]) {
  const int lane = threadIdx.x & 63;
  return wave_sum_i(tb[lane >> 4][lane & 15] + tb[4 + (lane >> 4)][lane & 15]);
}
struct WsTaus {
  float v[kWsTaus];
};
__global__ __launch_bounds__(1024) void k_ws_count(const float* __restrict__ out,
                                                   const int32_t* __restrict__ act, int q,
                                                   const double* __restrict__ bprev,
                                                   const double* __restrict__ c, double lambda,
                                                   WsTaus taus, int32_t* __restrict__ cnt) {
  __shared__ int acc[1 + kWsTaus];
  const int t = threadIdx.x;
  if (t <= kWsTaus) acc[t] = 0;
  __syncthreads();
  int loc[1 + kWsTaus] = {};
  for (int base = 0; base < q; base += 1024 * kWsScan) {
    // every load of the step issued before the first is used (positions
    // past the end clamped to the last one and not counted)
    int jv[kWsScan];
    double bp[kWsScan], cj[kWsScan];
    float o1[kWsScan];
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) jv[u] = act[min(base + 1024 * u + t, q - 1)];
    // without a previous point the load reads c (a valid column-indexed
    // array) and the value is discarded: no branch between the loads
    const double* bsrc = bprev ? bprev : c;
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) {
      const double bl = bsrc[jv[u]];
      bp[u] = bprev ? bl : 0.0;
      cj[u] = c[jv[u]];
      o1[u] = out[2 * (int64_t)jv[u] + 1];
    }
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) {
      if (base + 1024 * u + t >= q) continue;
      if (bp[u] != 0.0) {
        ++loc[0];
      } else if (fabs(cj[u]) > lambda) {
#pragma unroll
        for (int i = 0; i < kWsTaus; ++i) loc[1 + i] += o1[u] > taus.v[i] ? 1 : 0;
      }
    }
  }
#pragma unroll
  for (int i = 0; i <= kWsTaus; ++i)
    if (loc[i]) atomicAdd(&acc[i], loc[i]);
  __syncthreads();
  if (t <= kWsTaus) cnt[t] = acc[t];
}

// W = positions of act (q of them) on the support of beta_prev, or violating
// the optimality conditions at beta_prev (|c_j| > lambda) with support logit
// o1 > tau, in order; sigma = sign(beta_prev) on its support, else sign(c)
// (c indexed by column).  cnt[0] = |W|, cnt[1] = the members off the
// previous support.
__global__ __launch_bounds__(1024) void k_ws_select(const float* __restrict__ out,
                                                    const int32_t* __restrict__ act, int q,
                                                    const double* __restrict__ bprev,
                                                    const double* __restrict__ c, double lambda,
                                                    float tau, int cap,
                                                    int32_t* __restrict__ W,
                                                    double* __restrict__ sigma,
                                                    int32_t* __restrict__ mark,
                                                    int32_t* __restrict__ cnt) {
  __shared__ int wc[kWsScan][16];
  __shared__ int nw[kWsScan][16];
  // the selection is staged here and written out after the scan: a global
  // store in the loop would have to complete before each barrier
  __shared__ int32_t sW[kWsMaxSet];
  __shared__ double sS[kWsMaxSet];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  cap = min(cap, kWsMaxSet);
  int base_off = 0, new_tot = 0;
  for (int base = 0; base < q; base += 1024 * kWsScan) {
    int jv[kWsScan];
    double bp[kWsScan], cj[kWsScan];
    float o1[kWsScan];
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) jv[u] = act[min(base + 1024 * u + t, q - 1)];
    // without a previous point the load reads c (a valid column-indexed
    // array) and the value is discarded: no branch between the loads
    const double* bsrc = bprev ? bprev : c;
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) {
      const double bl = bsrc[jv[u]];
      bp[u] = bprev ? bl : 0.0;
      cj[u] = c[jv[u]];
      o1[u] = out[2 * (int64_t)jv[u] + 1];
    }
    bool in[kWsScan];
    uint64_t m[kWsScan];
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) {
      const bool v = base + 1024 * u + t < q;
      const bool prev = v && bp[u] != 0.0;
      const bool fresh = v && !prev && fabs(cj[u]) > lambda && o1[u] > tau;
      in[u] = prev || fresh;
      const uint64_t fm = ballot(fresh);
      m[u] = ballot(in[u]);
      if (lane == 0) {
        nw[u][w] = __popcll(fm);
        wc[u][w] = __popcll(m[u]);
      }
    }
    __syncthreads();
    int off[kWsScan];
    const int next_off = ws_chunk_offs(wc, w, base_off, off);
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) {
      if (in[u]) {
        const int pos = off[u] + __popcll(m[u] & lt);
        if (pos < cap) {
          sW[pos] = jv[u];
          sS[pos] = bp[u] != 0.0 ? (bp[u] > 0.0 ? 1.0 : -1.0) : (cj[u] >= 0.0 ? 1.0 : -1.0);
        }
      }
    }
    base_off = next_off;
    new_tot += ws_table_sum(nw);
    __syncthreads();
  }
  const int ns = min(base_off, cap);
  for (int a = t; a < ns; a += 1024) {
    const int j = sW[a];
    W[a] = j;
    sigma[a] = sS[a];
    mark[j] = 1;
  }
  if (t == 0) {
    cnt[0] = base_off;  // may exceed cap: the caller checks
    cnt[1] = new_tot;
  }
}

// Drops the members whose coefficient disagrees with sigma (b_a sigma_a <=
// 0): those off the support of beta_prev when there are any such, else the
// others; compacts W, sigma and b in order and unmarks the dropped columns.
// cnt[1] = number dropped, cnt[0] = new |W|.  Does nothing (cnt[1] = 0) when
// the solve failed (cnt[3] != 0).
__global__ __launch_bounds__(1024) void k_ws_drop(int32_t* __restrict__ W,
                                                  double* __restrict__ sigma,
                                                  double* __restrict__ b, int32_t* __restrict__ mark,
                                                  const double* __restrict__ bprev,
                                                  int32_t* __restrict__ cnt) {
  __shared__ int wc[16];
  __shared__ int nbad;
  __shared__ int32_t sW[2048];
  __shared__ double sS[2048], sB[2048];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (cnt[3] != 0) {
    if (t == 0) cnt[1] = 0;
    return;
  }
  const int m = cnt[0];
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  if (t == 0) nbad = 0;
  __syncthreads();
  for (int a = t; a < m; a += 1024) {
    sW[a] = W[a];
    sS[a] = sigma[a];
    sB[a] = b[a];
    if (!(sB[a] * sS[a] > 0.0) && !(bprev && bprev[sW[a]] != 0.0)) atomicAdd(&nbad, 1);
  }
  __syncthreads();
  const bool only_new = nbad > 0;
  int base_off = 0;
  for (int base = 0; base < m; base += 1024) {
    const int a = base + t;
    const bool wrong = a < m && !(sB[a] * sS[a] > 0.0);
    const bool keep =
        a < m && !(wrong && (!only_new || !(bprev && bprev[sW[a]] != 0.0)));
    const uint64_t msk = ballot(keep);
    if (lane == 0) wc[w] = __popcll(msk);
    __syncthreads();
    int off = base_off, tot = 0;
    for (int v = 0; v < 16; ++v) {
      if (v < w) off += wc[v];
      tot += wc[v];
    }
    if (keep) {
      const int pos = off + __popcll(msk & lt);
      W[pos] = sW[a];
      sigma[pos] = sS[a];
      b[pos] = sB[a];
    } else if (a < m) {
      mark[sW[a]] = 0;
    }
    base_off += tot;
    __syncthreads();
  }
  if (t == 0) {
    cnt[1] = m - base_off;
    cnt[0] = base_off;
  }
}

// Adds to W the (at most kadd) largest violators |c_k| - lambda > 0 over the
// positions k < q of act that are not in W (c indexed by position), sigma =
// sign(c_k), while |W| < cap; cnt[2] = number added.  Candidates pass through
// LDS (the first kWsCand in order when there are more).
constexpr int kWsCand = 4096;
__global__ __launch_bounds__(1024) void k_ws_add(const int32_t* __restrict__ act, int q,
                                                 const double* __restrict__ c, double lambda,
                                                 int kadd, int cap, int32_t* __restrict__ W,
                                                 double* __restrict__ sigma,
                                                 int32_t* __restrict__ mark,
                                                 int32_t* __restrict__ cnt) {
  __shared__ int wc[kWsScan][16];
  __shared__ double sv[kWsCand];
  __shared__ int32_t sk[kWsCand];
  __shared__ double rv[16];
  __shared__ int ri[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int nc = 0;
  for (int base = 0; base < q && nc < kWsCand; base += 1024 * kWsScan) {
    int jv[kWsScan], mk[kWsScan];
    double cv[kWsScan];
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) {
      const int kk = min(base + 1024 * u + t, q - 1);
      jv[u] = act[kk];
      cv[u] = c[kk];
    }
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) mk[u] = mark[jv[u]];
    bool f[kWsScan];
    double v[kWsScan];
    uint64_t msk[kWsScan];
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) {
      v[u] = fabs(cv[u]) - lambda;
      f[u] = base + 1024 * u + t < q && v[u] > 0.0 && mk[u] == 0;
      msk[u] = ballot(f[u]);
      if (lane == 0) wc[u][w] = __popcll(msk[u]);
    }
    __syncthreads();
    int off[kWsScan];
    const int next_nc = ws_chunk_offs(wc, w, nc, off);
#pragma unroll
    for (int u = 0; u < kWsScan; ++u) {
      if (f[u]) {
        const int pos = off[u] + __popcll(msk[u] & lt);
        if (pos < kWsCand) {
          sv[pos] = v[u];
          sk[pos] = base + 1024 * u + t;
        }
      }
    }
    nc = min(kWsCand, next_nc);
    __syncthreads();
  }
  int m = cnt[0];
  const int take = min(min(kadd, nc), max(0, cap - m));
  for (int r = 0; r < take; ++r) {
    // block argmax over the candidates (ties: the smaller position)
    double bv = -1.0;
    int bi = -1;
    for (int e = t; e < nc; e += 1024)
      if (sv[e] > bv) {
        bv = sv[e];
        bi = e;
      }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > bv || (ov == bv && oi >= 0 && (bi < 0 || oi < bi))) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      rv[w] = bv;
      ri[w] = bi;
    }
    __syncthreads();
    if (t == 0) {
      double gv = -1.0;
      int gi = -1;
      for (int u = 0; u < 16; ++u)
        if (ri[u] >= 0 && (rv[u] > gv || (rv[u] == gv && ri[u] < gi))) {
          gv = rv[u];
          gi = ri[u];
        }
      if (gi >= 0) {
        const int k = sk[gi];
        const int j = act[k];
        W[m] = j;
        sigma[m] = c[k] >= 0.0 ? 1.0 : -1.0;
        mark[j] = 1;
        sv[gi] = -1.0;
      }
      ri[0] = gi;
    }
    __syncthreads();
    if (ri[0] < 0) break;
    ++m;
    __syncthreads();
  }
  if (t == 0) {
    cnt[2] = m - cnt[0];
    cnt[0] = m;
  }
}

// beta0 = 0 (grid-wide), then beta0[W_a] = b_a by a second launch.
__global__ void k_ws_zero(int p, double* __restrict__ beta0) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < p; j += gridDim.x * blockDim.x)
    beta0[j] = 0.0;
}
__global__ void k_ws_scatter(const int32_t* __restrict__ W, const double* __restrict__ b,
                             const int32_t* __restrict__ cnt, double* __restrict__ beta0) {
  const int m = cnt[0];
  for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < m; a += gridDim.x * blockDim.x)
    beta0[W[a]] = b[a];
}

__global__ void k_ws_info0(int32_t* info) {
  if (threadIdx.x == 0) *info = 0;
}

int ws_last(const char* where) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GS_OK : set_hip_error(e, where);
}

}  // namespace

// G with its right-hand-side tile row ((M + 64) x M), then the Gram slices
// (S x M x M when S > 1); the slices take the largest need of any set size up
// to m, so that a workspace sized for a limit serves every smaller set
size_t ws_solve_bytes(int m) {
  const int NT = (m + TB - 1) / TB;
  const size_t M = (size_t)NT * TB;
  size_t slices = 0;
  for (int nt = 1; nt <= NT; ++nt) {
    const int S = gram_splits(nt, 1 << 30);
    const size_t Mt = (size_t)nt * TB;
    if (S > 1) slices = std::max(slices, (size_t)S * Mt * Mt);
  }
  return ((M + TB) * M + slices) * sizeof(double) + 256;
}

int ws_solve(int n, int p, int64_t ldx, int dtype, const void* X, const void* y, const int32_t* W,
             const double* sigma, int m, double lambda, double* b_out, int32_t* info,
             void* workspace, hipStream_t s) {
  const int M = (m + TB - 1) / TB * TB;
  const int NT = M / TB;
  double* G = static_cast<double*>(workspace);
  double* gend = G + (size_t)(M + TB) * M;
  hipLaunchKernelGGL(k_ws_info0, dim3(1), dim3(64), 0, s, info);
  int rc = ws_last("k_ws_info0");
  if (rc) return rc;
  const int ntile = NT * (NT + 1) / 2;
  const int rgrid = (M + 3) / 4;
  const int S = gram_splits(NT, n);
  const int R = ((n + S - 1) / S + 31) / 32 * 32;  // rows per split, whole chunks of 32
  double* gout = S > 1 ? gend : G;
  if (dtype == GS_F32) {
    hipLaunchKernelGGL(k_ws_gram<float>, dim3(ntile, S), dim3(256), 0, s,
                       static_cast<const float*>(X), ldx, n, p, W, m, M, R, gout);
    rc = ws_last("k_ws_gram");
    if (rc) return rc;
    hipLaunchKernelGGL(k_ws_rhs<float>, dim3(rgrid), dim3(256), 0, s, static_cast<const float*>(X),
                       ldx, n, p, static_cast<const float*>(y), W, sigma, m, M, lambda, G, info);
  } else {
    hipLaunchKernelGGL(k_ws_gram<double>, dim3(ntile, S), dim3(256), 0, s,
                       static_cast<const double*>(X), ldx, n, p, W, m, M, R, gout);
    rc = ws_last("k_ws_gram");
    if (rc) return rc;
    hipLaunchKernelGGL(k_ws_rhs<double>, dim3(rgrid), dim3(256), 0, s,
                       static_cast<const double*>(X), ldx, n, p, static_cast<const double*>(y), W,
                       sigma, m, M, lambda, G, info);
  }
  rc = ws_last("k_ws_rhs");
  if (rc) return rc;
  if (S > 1) {
    const int64_t MM = (int64_t)M * M;
    const int sgrid = (int)std::min<int64_t>((MM + 255) / 256, 2048);
    hipLaunchKernelGGL(k_ws_gram_sum, dim3(sgrid), dim3(256), 0, s, gout, S, M, m, G);
    rc = ws_last("k_ws_gram_sum");
    if (rc) return rc;
  }
  for (int K = 0; K < NT; ++K) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, G, M, K, info);
    rc = ws_last("k_chol_diag");
    if (rc) return rc;
    // the tile rows below K, the right-hand side's included
    const int T = NT - K - 1;
    hipLaunchKernelGGL(k_chol_panel, dim3(T + 1), dim3(256), 0, s, G, M, K, info);
    rc = ws_last("k_chol_panel");
    if (rc) return rc;
    if (T == 0) break;
    hipLaunchKernelGGL(k_chol_update, dim3(T * (T + 1) / 2 + T), dim3(256), 0, s, G, M, K, info);
    rc = ws_last("k_chol_update");
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(kSolveThreads), 0, s, G, M, m, b_out, info);
  return ws_last("k_chol_solve");
}

int ws_count(const float* out, const int32_t* act, int q, const double* bprev, const double* c,
             double lambda, const float* taus, int32_t* cnt8, hipStream_t s) {
  WsTaus tv;
  for (int i = 0; i < kWsTaus; ++i) tv.v[i] = taus[i];
  hipLaunchKernelGGL(k_ws_count, dim3(1), dim3(1024), 0, s, out, act, q, bprev, c, lambda, tv,
                     cnt8);
  return ws_last("k_ws_count");
}

int ws_select(const float* out, const int32_t* act, int q, const double* bprev, const double* c,
              double lambda, float tau, int cap, int32_t* W, double* sigma, int32_t* mark,
              int32_t* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_select, dim3(1), dim3(1024), 0, s, out, act, q, bprev, c, lambda, tau,
                     cap, W, sigma, mark, cnt);
  return ws_last("k_ws_select");
}

int ws_drop(int32_t* W, double* sigma, double* b, int32_t* mark, const double* bprev,
            int32_t* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_drop, dim3(1), dim3(1024), 0, s, W, sigma, b, mark, bprev, cnt);
  return ws_last("k_ws_drop");
}

int ws_add(const int32_t* act, int q, const double* c, double lambda, int kadd, int cap,
           int32_t* W, double* sigma, int32_t* mark, int32_t* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_add, dim3(1), dim3(1024), 0, s, act, q, c, lambda, kadd, cap, W, sigma,
                     mark, cnt);
  return ws_last("k_ws_add");
}

int ws_scatter(const int32_t* W, const double* b, const int32_t* cnt, int p, double* beta0,
               hipStream_t s) {
  const int g = std::max(1, std::min(1024, (p + 255) / 256));
  hipLaunchKernelGGL(k_ws_zero, dim3(g), dim3(256), 0, s, p, beta0);
  int rc = ws_last("k_ws_zero");
  if (rc) return rc;
  hipLaunchKernelGGL(k_ws_scatter, dim3(8), dim3(256), 0, s, W, b, cnt, beta0);
  return ws_last("k_ws_scatter");
}

}  // namespace gs

using namespace gs;

extern "C" {

size_t gs_restricted_solve_workspace_size(int32_t m) {
  if (m < 1 || m > kWsMaxSet) return 0;
  return ws_solve_bytes(m);
}

int gs_restricted_solve(int32_t n, int32_t p, int64_t ldx, int32_t dtype, const void* X,
                        const void* y, const int32_t* W, const double* sigma, int32_t m,
                        double lambda, double* b_out, int32_t* info_out, void* workspace,
                        size_t ws_bytes, void* stream) {
  if (n < 1 || p < 1 || ldx < n || !X || !y || !W || !sigma || !b_out || !info_out)
    return GS_EINVAL;
  if (dtype != GS_F32 && dtype != GS_F64) return GS_EINVAL;
  if (m < 1 || m >= n || m > kWsMaxSet || m > p) return GS_EINVAL;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return GS_EINVAL;
  if (!workspace || ws_bytes < ws_solve_bytes(m)) return GS_EWORKSPACE;
  return ws_solve(n, p, ldx, dtype, X, y, W, sigma, m, lambda, b_out, info_out, workspace,
                  static_cast<hipStream_t>(stream));
}

}  // extern "C"
