// The learned warm start: block max correlation of the design, the
// per-feature inputs, the 4 -> 64 -> 64 -> 2 network (inference with a BF16
// matrix-core second layer; training forward/backward with per-block partial
// gradients, then a fixed-order reduction and an Adam step), the assembly of
// the candidate start, and the path driver that uses it.  The network only
// proposes a starting point: GAP SAFE rules are safe for any primal point
// (Theorem 2), so the path keeps the proposal only when its duality gap is
// smaller than the plain warm start's, and Algorithm 1 then runs unchanged
// from there.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/gapsafe.h"
#include "gs_device.hpp"

namespace gs {
namespace {

// ---- bfloat16, round to nearest with ties to even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float rbf(float x) { return bf2f(f2bf(x)); }

constexpr int kPartStride = kMlpParams + 1;  // partial gradient + partial loss
static_assert(GS_MLP_PARAMS == kMlpParams, "parameter count of the C ABI");

// ---------------------------------------------------------------------------
// Block max correlation: bmc_j = max over k != j in j's block of
// |x_j^T x_k| / (||x_j|| ||x_k||), 0 for a block of one column or a zero
// column.  One workgroup per block of at most 64 columns: rows stream through
// LDS in tiles of 64, each thread accumulates 16 Gram entries in FP32.
// ---------------------------------------------------------------------------
template <typename XT>
__global__ __launch_bounds__(256) void k_block_corr(const XT* __restrict__ X, int64_t ldx, int n,
                                                    int p, int block, float* __restrict__ bmc) {
  __shared__ float tile[64][65];
  __shared__ float G[64][65];
  const int b0 = blockIdx.x * block;
  const int nb = min(block, p - b0);
  const int t = threadIdx.x;
  float acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.f;
  for (int r0 = 0; r0 < n; r0 += 64) {
    const int nr = min(64, n - r0);
    for (int idx = t; idx < 64 * 64; idx += 256) {
      const int c = idx >> 6, r = idx & 63;  // consecutive threads read down a column
      tile[r][c] = (c < nb && r < nr) ? (float)X[(int64_t)(b0 + c) * ldx + r0 + r] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int idx = t + 256 * e;
      const int a = idx >> 6, c = idx & 63;
      float s = acc[e];
      for (int r = 0; r < nr; ++r) s = fmaf(tile[r][a], tile[r][c], s);
      acc[e] = s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int idx = t + 256 * e;
    G[idx >> 6][idx & 63] = acc[e];
  }
  __syncthreads();
  if (t < nb) {
    const float dj = sqrtf(G[t][t]);
    float best = 0.f;
    for (int k = 0; k < nb; ++k) {
      if (k == t) continue;
      const float dk = sqrtf(G[k][k]);
      if (dj > 0.f && dk > 0.f) best = fmaxf(best, fabsf(G[t][k]) / (dj * dk));
    }
    bmc[b0 + t] = best;
  }
}

// ---------------------------------------------------------------------------
// The network.  One wavefront handles 64 features (lane = feature).  The
// second layer, H2 = relu(H1 W2^T + b2) over 64 features x 64 units, is four
// 32x32 tiles of v_mfma_f32_32x32x8bf16_1k (BF16 operands, FP32
// accumulation); layers one and three run on the vector ALUs in FP32 with
// BF16-rounded weights.
// ---------------------------------------------------------------------------
struct MlpLds {
  float w1[256], b1[64], b2[64], w3[128], b3[2], pad_[2];
  uint16_t w2[64][72];  // BF16, row = output unit, column = input unit (padded)
  uint16_t h1[64][72];  // BF16 first hidden layer, row = feature
  float h2[64][65];     // second hidden layer after ReLU, row = feature
  float u[64][4];       // inputs, row = feature
};

__device__ __forceinline__ void mlp_load_weights(const float* __restrict__ P, MlpLds& L) {
  const int lane = threadIdx.x;
  for (int i = lane; i < 256; i += 64) L.w1[i] = rbf(P[kMlpW1 + i]);
  L.b1[lane] = P[kMlpB1 + lane];
  L.b2[lane] = P[kMlpB2 + lane];
  for (int i = lane; i < 128; i += 64) L.w3[i] = rbf(P[kMlpW3 + i]);
  if (lane < 2) L.b3[lane] = P[kMlpB3 + lane];
  for (int i = lane; i < 64 * 64; i += 64) L.w2[i >> 6][i & 63] = f2bf(P[kMlpW2 + i]);
  wave_lds_order();
}

// Forward pass of features f0 .. f0+63 (rows of U, m in total): returns the
// lane's two outputs and leaves u, h1 (BF16) and h2 in LDS.
__device__ __forceinline__ void mlp_forward64(const float* __restrict__ U, int f0, int m,
                                              MlpLds& L, float& o0, float& o1) {
  const int lane = threadIdx.x;
  const int f = f0 + lane;
  const bool v = f < m;
  float u[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    u[c] = v ? U[(int64_t)f * 4 + c] : 0.f;
    L.u[lane][c] = u[c];
  }
#pragma unroll 8
  for (int k = 0; k < 64; ++k) {
    float z = L.b1[k];
#pragma unroll
    for (int c = 0; c < 4; ++c) z = fmaf(L.w1[k * 4 + c], u[c], z);
    L.h1[lane][k] = f2bf(fmaxf(z, 0.f));
  }
  wave_lds_order();
  typedef short v4s __attribute__((ext_vector_type(4)));
  typedef float v16f __attribute__((ext_vector_type(16)));
  const int col = lane & 31, half = lane >> 5;
#pragma unroll
  for (int ft = 0; ft < 2; ++ft)
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      v16f acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        const int kk = ks * 8 + 4 * half;
        // A[i][k] = H1[feature 32 ft + i][k], B[k][j] = W2[unit 32 it + j][k]
        const v4s a = *reinterpret_cast<const v4s*>(&L.h1[ft * 32 + col][kk]);
        const v4s b = *reinterpret_cast<const v4s*>(&L.w2[it * 32 + col][kk]);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
      }
      // D[i][j] sits in lane j + 32 h, register r, with i = 8 (r / 4) + 4 h + r % 4
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int fi = ft * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        const int ui = it * 32 + col;
        L.h2[fi][ui] = fmaxf(acc[r] + L.b2[ui], 0.f);
      }
    }
  wave_lds_order();
  float a0 = L.b3[0], a1 = L.b3[1];
#pragma unroll 8
  for (int i = 0; i < 64; ++i) {
    const float h = L.h2[lane][i];
    a0 = fmaf(L.w3[i], h, a0);
    a1 = fmaf(L.w3[64 + i], h, a1);
  }
  o0 = a0;
  o1 = a1;
}

__global__ __launch_bounds__(64) void k_mlp_infer(const float* __restrict__ P,
                                                  const float* __restrict__ U, int m,
                                                  float* __restrict__ out) {
  __shared__ MlpLds L;
  mlp_load_weights(P, L);
  for (int f0 = blockIdx.x * 64; f0 < m; f0 += gridDim.x * 64) {
    float o0, o1;
    mlp_forward64(U, f0, m, L, o0, o1);
    const int f = f0 + threadIdx.x;
    if (f < m) {
      out[(int64_t)f * 2] = o0;
      out[(int64_t)f * 2 + 1] = o1;
    }
    wave_lds_order();
  }
}

// Training forward and backward of one 64-feature block.  Targets are rows
// (step, support, mask); the loss is the mean over all m features of
// BCE(logit o1, support) + mask (o0 - step)^2.  The block writes its partial
// gradient (kMlpParams floats, in the parameter layout) and partial loss to
// part[block * kPartStride].  The gradient passes through the BF16 roundings
// unchanged: the derivatives are those of the network the forward evaluated.
__global__ __launch_bounds__(64) void k_mlp_train_fb(const float* __restrict__ P,
                                                     const float* __restrict__ U,
                                                     const float* __restrict__ tgt, int m,
                                                     float* __restrict__ part) {
  __shared__ MlpLds L;
  __shared__ float g1[64][65];  // d loss / d first-layer pre-activation, row = feature
  __shared__ float go[64][2];   // d loss / d outputs
  mlp_load_weights(P, L);
  const int lane = threadIdx.x;
  const int f = blockIdx.x * 64 + lane;
  const bool v = f < m;
  float o0, o1;
  mlp_forward64(U, blockIdx.x * 64, m, L, o0, o1);
  const float ts = v ? tgt[(int64_t)f * 3] : 0.f;
  const float tp = v ? tgt[(int64_t)f * 3 + 1] : 0.f;
  const float mk = v ? tgt[(int64_t)f * 3 + 2] : 0.f;
  const float inv_m = 1.f / (float)m;
  const float d = o0 - ts;
  const float bce = fmaxf(o1, 0.f) - o1 * tp + log1pf(expf(-fabsf(o1)));
  const float loss = v ? bce + mk * d * d : 0.f;
  const float sg = 1.f / (1.f + expf(-o1));
  go[lane][0] = v ? 2.f * mk * d * inv_m : 0.f;
  go[lane][1] = v ? (sg - tp) * inv_m : 0.f;
  wave_lds_order();
  float* out = part + (int64_t)blockIdx.x * kPartStride;
  {  // W3, b3: lane = hidden unit i
    float a0 = 0.f, a1 = 0.f, s0 = 0.f, s1 = 0.f;
    for (int ff = 0; ff < 64; ++ff) {
      const float h = L.h2[ff][lane];
      a0 = fmaf(go[ff][0], h, a0);
      a1 = fmaf(go[ff][1], h, a1);
      s0 += go[ff][0];
      s1 += go[ff][1];
    }
    out[kMlpW3 + lane] = a0;
    out[kMlpW3 + 64 + lane] = a1;
    if (lane == 0) {
      out[kMlpB3] = s0;
      out[kMlpB3 + 1] = s1;
    }
  }
  wave_lds_order();
  {  // second-layer pre-activation gradient, in place of h2 (lane = feature)
    const float q0 = go[lane][0], q1 = go[lane][1];
    for (int i = 0; i < 64; ++i) {
      const float h = L.h2[lane][i];
      const float g = fmaf(q0, L.w3[i], q1 * L.w3[64 + i]);
      L.h2[lane][i] = h > 0.f ? g : 0.f;
    }
  }
  wave_lds_order();
  {  // W2, b2: lane = output unit i, the 64 inputs in registers
    float acc[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) acc[k] = 0.f;
    float sb = 0.f;
    for (int ff = 0; ff < 64; ++ff) {
      const float g = L.h2[ff][lane];
      sb += g;
#pragma unroll
      for (int k = 0; k < 64; ++k) acc[k] = fmaf(g, bf2f(L.h1[ff][k]), acc[k]);
    }
#pragma unroll
    for (int k = 0; k < 64; ++k) out[kMlpW2 + lane * 64 + k] = acc[k];
    out[kMlpB2 + lane] = sb;
  }
  {  // first-layer pre-activation gradient (lane = feature)
    float acc[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) acc[k] = 0.f;
    for (int i = 0; i < 64; ++i) {
      const float g = L.h2[lane][i];
#pragma unroll
      for (int k = 0; k < 64; ++k) acc[k] = fmaf(g, bf2f(L.w2[i][k]), acc[k]);
    }
#pragma unroll
    for (int k = 0; k < 64; ++k) g1[lane][k] = bf2f(L.h1[lane][k]) > 0.f ? acc[k] : 0.f;
  }
  wave_lds_order();
  {  // W1, b1: lane = hidden unit k
    float a[4] = {0.f, 0.f, 0.f, 0.f}, sb = 0.f;
    for (int ff = 0; ff < 64; ++ff) {
      const float g = g1[ff][lane];
      sb += g;
#pragma unroll
      for (int c = 0; c < 4; ++c) a[c] = fmaf(g, L.u[ff][c], a[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) out[kMlpW1 + lane * 4 + c] = a[c];
    out[kMlpB1 + lane] = sb;
  }
  float ls = loss;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) ls += __shfl_xor(ls, o);
  if (lane == 0) out[kMlpParams] = ls * inv_m;
}

// Sums the nblk partials (stride kPartStride) in block order into grad/loss
// (either may be null); with P non-null it then applies one Adam step
// (Kingma & Ba) to the FP32 master weights.  With nblk == 0 the gradient is
// read from `part` as a plain kMlpParams array (no loss slot).
__global__ __launch_bounds__(256) void k_mlp_reduce_adam(
    float* __restrict__ P, float* __restrict__ M, float* __restrict__ V,
    const float* __restrict__ part, int nblk, float lr, float bc1, float bc2,
    float* __restrict__ grad_out, float* __restrict__ loss_out) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int top = nblk > 0 ? kMlpParams + 1 : kMlpParams;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < top; i += gridDim.x * blockDim.x) {
    float g = 0.f;
    if (nblk > 0)
      for (int b = 0; b < nblk; ++b) g += part[(int64_t)b * kPartStride + i];
    else
      g = part[i];
    if (i == kMlpParams) {
      if (loss_out) *loss_out = g;
      continue;
    }
    if (grad_out) grad_out[i] = g;
    if (P) {
      const float mm = b1 * M[i] + (1.f - b1) * g;
      const float vv = b2 * V[i] + (1.f - b2) * g * g;
      M[i] = mm;
      V[i] = vv;
      P[i] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    }
  }
}

// ---------------------------------------------------------------------------
// Inputs of the network for every feature j, with c_j = x_j^T (y - X beta):
// (|c_j| / lambda, lambda / lambda_max, beta_j ||x_j|| / ||y||, bmc_j).
// ---------------------------------------------------------------------------
__global__ void k_warm_features(const double* __restrict__ c, const double* __restrict__ bprev,
                                const double* __restrict__ nrm2, const float* __restrict__ bmc,
                                int p, double lam, double lam_max, double ynorm,
                                float* __restrict__ U) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < p; j += gridDim.x * blockDim.x) {
    U[(int64_t)j * 4] = (float)(fabs(c[j]) / lam);
    U[(int64_t)j * 4 + 1] = (float)(lam / lam_max);
    U[(int64_t)j * 4 + 2] = (float)(bprev[j] * sqrt(nrm2[j]) / ynorm);
    U[(int64_t)j * 4 + 3] = bmc[j];
  }
}

// ||x_j||^2 and x_j^T y in FP64, one wavefront per column.
template <typename XT>
__global__ __launch_bounds__(256) void k_col_stats(const XT* __restrict__ X,
                                                   const XT* __restrict__ y, int64_t ldx, int n,
                                                   int p, double* __restrict__ nrm2,
                                                   double* __restrict__ xty) {
  const int lane = threadIdx.x & 63;
  const int waves = (gridDim.x * blockDim.x) >> 6;
  for (int j = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; j < p; j += waves) {
    double s = 0.0, sy = 0.0;
    for (int i = lane; i < n; i += 64) {
      const double v = (double)X[(int64_t)j * ldx + i];
      s = fma(v, v, s);
      sy = fma(v, (double)y[i], sy);
    }
    s = wave_sum(s);
    sy = wave_sum(sy);
    if (lane == 0) {
      nrm2[j] = s;
      xty[j] = sy;
    }
  }
}

// out2 = (max_j |v_j|, ||y||^2), one workgroup.
template <typename YT>
__global__ __launch_bounds__(256) void k_absmax_ynorm(const double* __restrict__ v, int p,
                                                      const YT* __restrict__ y, int n,
                                                      double* __restrict__ out2) {
  __shared__ double s1[256], s2[256];
  double m = 0.0, yy = 0.0;
  for (int j = threadIdx.x; j < p; j += 256) m = fmax(m, fabs(v[j]));
  for (int i = threadIdx.x; i < n; i += 256) yy = fma((double)y[i], (double)y[i], yy);
  s1[threadIdx.x] = m;
  s2[threadIdx.x] = yy;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + w]);
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = s1[0];
    out2[1] = s2[0];
  }
}

// start = the network's candidate when its gap is strictly smaller, else the
// plain one; flag = 1 when the network's was taken.
__global__ void k_warm_choose(const double* __restrict__ gap_plain,
                              const double* __restrict__ gap_net,
                              const double* __restrict__ beta_net,
                              const double* __restrict__ beta_plain, int p,
                              double* __restrict__ start, int32_t* __restrict__ flag,
                              int32_t* __restrict__ taken) {
  const bool net = *gap_net < *gap_plain;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < p; j += gridDim.x * blockDim.x)
    start[j] = net ? beta_net[j] : beta_plain[j];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (flag) *flag = net ? 1 : 0;
    *taken = net ? 1 : 0;
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int cnt, int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
    a[i] = v;
}
__global__ void k_fill_f64(double* __restrict__ a, int cnt, double v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
    a[i] = v;
}

// ------------------------------------------------------------------ host
int grid_for(int64_t count, int threads, int cap = 4096) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (count + threads - 1) / threads));
}

int last_launch(const char* where) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GS_OK : set_hip_error(e, where);
}

size_t al256(size_t v) { return (v + 255) / 256 * 256; }

int launch_block_corr(int n, int p, int64_t ldx, int dtype, const void* X, int block, float* bmc,
                      hipStream_t s) {
  const int nblk = (p + block - 1) / block;
  if (dtype == GS_F32)
    hipLaunchKernelGGL(k_block_corr<float>, dim3(nblk), dim3(256), 0, s,
                       static_cast<const float*>(X), ldx, n, p, block, bmc);
  else
    hipLaunchKernelGGL(k_block_corr<double>, dim3(nblk), dim3(256), 0, s,
                       static_cast<const double*>(X), ldx, n, p, block, bmc);
  return last_launch("k_block_corr");
}

int launch_mlp_forward(const float* P, const float* U, int m, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_infer, dim3(grid_for(m, 64, 2048)), dim3(64), 0, s, P, U, m, out);
  return last_launch("k_mlp_infer");
}

int launch_features(int p, const double* c, const double* bprev, const double* nrm2,
                    const float* bmc, double lam, double lam_max, double ynorm, float* U,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_warm_features, dim3(grid_for(p, 256)), dim3(256), 0, s, c, bprev, nrm2,
                     bmc, p, lam, lam_max, ynorm, U);
  return last_launch("k_warm_features");
}

int fill_i32(int32_t* a, int cnt, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(cnt, 256)), dim3(256), 0, s, a, cnt, v);
  return last_launch("k_fill_i32");
}

struct LearnedWs {
  void* inner;  // shared by screen() and the per-lambda lasso_path
  size_t inner_bytes;
  float *bmc, *U, *out;
  double *nrm2, *c, *beta0, *start, *scal;  // scal: lmax, ||y||^2, gap_plain, gap_net, alpha, radius
  int32_t *act, *act2, *q;
  // working set: W, sigma, b (cap entries each), membership marks (p), c at
  // beta0 by position (p), counters (|W|, dropped, added, info), solve space
  int32_t *W, *mark, *cnt;
  double *sig, *bw, *c2;
  void* wsolve;
  int cap;
  size_t total;
};

LearnedWs carve_learned(const gs_problem* pr, char* base) {
  const size_t path_b = lasso_workspace_size(pr, 1, nullptr);
  const size_t scr_b = screen_workspace_size(pr->n, pr->p);
  LearnedWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = base ? base + off : nullptr;
    off += al256(std::max<size_t>(bytes, 1));
    return q;
  };
  const size_t P = (size_t)pr->p;
  w.inner_bytes = al256(std::max(path_b, scr_b));
  w.inner = take(w.inner_bytes);
  w.bmc = reinterpret_cast<float*>(take(sizeof(float) * P));
  w.U = reinterpret_cast<float*>(take(sizeof(float) * 4 * P));
  w.out = reinterpret_cast<float*>(take(sizeof(float) * 2 * P));
  w.nrm2 = reinterpret_cast<double*>(take(sizeof(double) * P));
  w.c = reinterpret_cast<double*>(take(sizeof(double) * P));
  w.beta0 = reinterpret_cast<double*>(take(sizeof(double) * P));
  w.start = reinterpret_cast<double*>(take(sizeof(double) * P));
  w.scal = reinterpret_cast<double*>(take(sizeof(double) * 8));
  w.act = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * P));
  w.act2 = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * P));
  w.q = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 4));
  w.cap = std::max(0, std::min(pr->n - 1, std::min(pr->p, kWsMaxSet)));
  const size_t C = (size_t)std::max(w.cap, 1);
  w.W = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * C));
  w.sig = reinterpret_cast<double*>(take(sizeof(double) * C));
  w.bw = reinterpret_cast<double*>(take(sizeof(double) * C));
  w.mark = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * P));
  w.c2 = reinterpret_cast<double*>(take(sizeof(double) * P));
  w.cnt = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 16));
  w.wsolve = take(ws_solve_bytes((int)C));
  w.total = off;
  return w;
}

// lambda_t output from the working-set start certified on the safe set: beta0,
// that pass's gap and kept count, 0 epochs, status 0.
__global__ void k_ws_emit(const double* __restrict__ beta0, int p, double* __restrict__ beta_out,
                          const double* __restrict__ gap, const int32_t* __restrict__ kept,
                          double* __restrict__ gap_out, int32_t* __restrict__ epochs_out,
                          int32_t* __restrict__ nactive_out, int32_t* __restrict__ status_out,
                          double* __restrict__ lambda_out, double lam,
                          int32_t* __restrict__ flag) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < p; j += gridDim.x * blockDim.x)
    beta_out[j] = beta0[j];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *gap_out = *gap;
    *epochs_out = 0;
    *nactive_out = *kept;
    *status_out = GS_STATUS_CONVERGED;
    if (lambda_out) *lambda_out = lam;
    if (flag) *flag = 1;
  }
}

// Reads the four working-set counters (|W|, dropped, added, info).
int read_cnt(const LearnedWs& w, int32_t (&h)[4], hipStream_t s) {
  hipError_t e = hipMemcpyAsync(h, w.cnt, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? GS_OK : set_hip_error(e, "lasso_path_learned: working set");
}

// The working-set start (steps 2-4 of lasso_path_learned) into w.beta0; m
// receives |W| (0: no start, the plain one is used).  Needs the network's
// outputs in w.out, A_plain in w.act (q positions) and c at beta_prev in w.c.
int ws_start(const gs_problem* pr, const LearnedWs& w, int q, const double* bprev, double lam,
             int rule, int& m, bool& gap_known, hipStream_t s) {
  const int n = pr->n, p = pr->p, dt = pr->dtype;
  m = 0;
  gap_known = false;
  // the previous support and the network's predicted entrants, the logit
  // threshold raised until at most min(GS_WS_ADD, (cap - |previous support|)
  // / 2) enter (none when even the last threshold admits more); the counts
  // for every threshold come from one pass
  static const float taus[7] = {0.f, 1.f, 2.f, 3.f, 4.f, 6.f, 8.f};
  int rc = ws_count(w.out, w.act, q, bprev, w.c, lam, taus, w.cnt + 4, s);
  if (rc) return rc;
  int32_t c8[8];
  {
    hipError_t e = hipMemcpyAsync(c8, w.cnt + 4, sizeof(c8), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_hip_error(e, "lasso_path_learned: working set");
  }
  const int kin = std::min((int)GS_WS_ADD, std::max(0, (w.cap - c8[0]) / 2));
  float tau = INFINITY;
  int fresh = 0;
  for (int i = 0; i < 7; ++i)
    if (c8[1 + i] <= kin) {
      tau = taus[i];
      fresh = c8[1 + i];
      break;
    }
  int mm = c8[0] + fresh;
  if (mm < 1 || mm > w.cap) return GS_OK;
  rc = fill_i32(w.mark, p, 0, s);
  if (rc) return rc;
  rc = fill_i32(w.cnt, 4, 0, s);
  if (rc) return rc;
  rc = ws_select(w.out, w.act, q, bprev, w.c, lam, tau, w.cap, w.W, w.sig, w.mark, w.cnt, s);
  if (rc) return rc;
  int32_t h[4];
  for (int r = 0;; ++r) {
    for (int dd = 0;; ++dd) {
      rc = ws_solve(n, p, pr->ldx, dt, pr->X, pr->y, w.W, w.sig, mm, lam, w.bw, w.cnt + 3,
                    w.wsolve, s);
      if (rc) return rc;
      rc = ws_drop(w.W, w.sig, w.bw, w.mark, bprev, w.cnt, s);
      if (rc) return rc;
      rc = read_cnt(w, h, s);
      if (rc) return rc;
      if (h[3] != 0) return GS_OK;  // factorization failed: plain start
      mm = h[0];
      if (mm < 1) return GS_OK;
      if (h[1] == 0 || dd >= GS_WS_DROPS) break;
    }
    rc = ws_scatter(w.W, w.bw, w.cnt, p, w.beta0, s);
    if (rc) return rc;
    if (r >= GS_WS_ROUNDS) break;
    // violators of the optimality conditions at beta0 over A_plain
    rc = screen(n, p, pr->ldx, dt, pr->X, pr->y, w.beta0, lam, rule, w.act, q, w.act2, w.q + 1,
                w.scal + 3, w.scal + 4, w.scal + 5, w.c2, w.inner, w.inner_bytes, s);
    if (rc) return rc;
    rc = ws_add(w.act, q, w.c2, lam, GS_WS_ADD, w.cap, w.W, w.sig, w.mark, w.cnt, s);
    if (rc) return rc;
    rc = read_cnt(w, h, s);
    if (rc) return rc;
    if (h[2] == 0) {  // no violator: the pass just made was at this beta0
      gap_known = true;
      break;
    }
    mm = h[0];
  }
  m = mm;
  return GS_OK;
}

bool learned_problem_ok(const gs_problem* pr) {
  return pr && pr->n >= 1 && pr->p >= 1 && pr->T >= 1 && pr->X && pr->y && !pr->rows &&
         pr->ldx >= pr->n && (pr->dtype == GS_F32 || pr->dtype == GS_F64) && pr->beta_out &&
         pr->gap_out && pr->epochs_out && pr->nactive_out && pr->status_out;
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

int gs_block_corr(int32_t n, int32_t p, int64_t ldx, int32_t dtype, const void* X, int32_t block,
                  float* bmc, void* stream) {
  if (n < 1 || p < 1 || ldx < n || !X || !bmc) return GS_EINVAL;
  if (dtype != GS_F32 && dtype != GS_F64) return GS_EINVAL;
  if (block < 1 || block > 64) return GS_EINVAL;
  return launch_block_corr(n, p, ldx, dtype, X, block, bmc, static_cast<hipStream_t>(stream));
}

int gs_mlp_forward(const float* params, const float* U, int32_t m, float* out, void* stream) {
  if (m < 0 || (m > 0 && (!params || !U || !out))) return GS_EINVAL;
  if (m == 0) return GS_OK;
  return launch_mlp_forward(params, U, m, out, static_cast<hipStream_t>(stream));
}

size_t gs_mlp_train_workspace_size(int32_t m) {
  if (m < 1) return 0;
  return al256(sizeof(float) * (size_t)kPartStride * (size_t)((m + 63) / 64));
}

int gs_mlp_grad(const float* params, const float* U, const float* targets, int32_t m, float* grad,
                float* loss, void* workspace, size_t ws_bytes, void* stream) {
  if (m < 1 || !params || !U || !targets) return GS_EINVAL;
  if (!workspace || ws_bytes < gs_mlp_train_workspace_size(m)) return GS_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* part = static_cast<float*>(workspace);
  const int nblk = (m + 63) / 64;
  hipLaunchKernelGGL(k_mlp_train_fb, dim3(nblk), dim3(64), 0, s, params, U, targets, m, part);
  int rc = last_launch("k_mlp_train_fb");
  if (rc) return rc;
  float* none = nullptr;
  hipLaunchKernelGGL(k_mlp_reduce_adam, dim3(grid_for(kMlpParams + 1, 256)), dim3(256), 0, s,
                     none, none, none, part, nblk, 0.f, 1.f, 1.f, grad, loss);
  return last_launch("k_mlp_reduce_adam");
}

int gs_mlp_adam(float* params, float* adam_m, float* adam_v, const float* grad, int32_t t,
                float lr, void* stream) {
  if (!params || !adam_m || !adam_v || !grad || t < 1 || !std::isfinite(lr)) return GS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float bc1 = (float)(1.0 - std::pow(0.9, (double)t));
  const float bc2 = (float)(1.0 - std::pow(0.999, (double)t));
  float* none = nullptr;
  hipLaunchKernelGGL(k_mlp_reduce_adam, dim3(grid_for(kMlpParams, 256)), dim3(256), 0, s, params,
                     adam_m, adam_v, grad, 0, lr, bc1, bc2, none, none);
  return last_launch("k_mlp_reduce_adam");
}

int gs_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t t, float lr,
                      const float* U, const float* targets, int32_t m, float* loss,
                      void* workspace, size_t ws_bytes, void* stream) {
  if (m < 1 || !params || !adam_m || !adam_v || !U || !targets || t < 1 || !std::isfinite(lr))
    return GS_EINVAL;
  if (!workspace || ws_bytes < gs_mlp_train_workspace_size(m)) return GS_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* part = static_cast<float*>(workspace);
  const int nblk = (m + 63) / 64;
  hipLaunchKernelGGL(k_mlp_train_fb, dim3(nblk), dim3(64), 0, s, params, U, targets, m, part);
  int rc = last_launch("k_mlp_train_fb");
  if (rc) return rc;
  const float bc1 = (float)(1.0 - std::pow(0.9, (double)t));
  const float bc2 = (float)(1.0 - std::pow(0.999, (double)t));
  float* none = nullptr;
  hipLaunchKernelGGL(k_mlp_reduce_adam, dim3(grid_for(kMlpParams + 1, 256)), dim3(256), 0, s,
                     params, adam_m, adam_v, part, nblk, lr, bc1, bc2, none, loss);
  return last_launch("k_mlp_reduce_adam");
}

int gs_warm_features(int32_t p, const double* c, const double* beta_prev, const double* nrm2,
                     const float* bmc, double lambda, double lambda_max, double ynorm, float* U,
                     void* stream) {
  if (p < 1 || !c || !beta_prev || !nrm2 || !bmc || !U) return GS_EINVAL;
  if (!(lambda > 0.0) || !(lambda_max > 0.0) || !(ynorm > 0.0) || !std::isfinite(lambda) ||
      !std::isfinite(lambda_max) || !std::isfinite(ynorm))
    return GS_EINVAL;
  return launch_features(p, c, beta_prev, nrm2, bmc, lambda, lambda_max, ynorm, U,
                         static_cast<hipStream_t>(stream));
}

size_t lasso_path_learned_workspace_size(const gs_problem* prob) {
  if (!learned_problem_ok(prob)) return 0;
  if (lasso_workspace_size(prob, 1, nullptr) == 0) return 0;
  return carve_learned(prob, nullptr).total;
}

int lasso_path_learned(const gs_problem* prob, const gs_opts* opts, const float* params,
                       int32_t block, int32_t* learned_out, void* workspace, size_t ws_bytes,
                       void* stream) {
  if (!learned_problem_ok(prob)) return GS_EINVAL;
  if (opts && ((opts->enet_alpha != 0.0 && opts->enet_alpha != 1.0) ||
               opts->rule >= GS_RULE_STATIC))
    return GS_EUNSUPPORTED;  // the learned start is built for the Lasso with GAP SAFE tests
  if (params && (block < 1 || block > 64)) return GS_EINVAL;
  if (prob->lambdas) {
    for (int t = 0; t < prob->T; ++t)
      if (!(prob->lambdas[t] > 0.0) || !std::isfinite(prob->lambdas[t])) return GS_EINVAL;
  } else if (!(prob->lambda_min_ratio > 0.0 && prob->lambda_min_ratio <= 1.0)) {
    return GS_EINVAL;
  }
  if (prob->n > 2048) return GS_EUNSUPPORTED;
  if (!workspace) return GS_EWORKSPACE;
  if (lasso_workspace_size(prob, 1, opts) == 0) return GS_EINVAL;
  const LearnedWs w = carve_learned(prob, static_cast<char*>(workspace));
  if (ws_bytes < w.total) return GS_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = prob->n, p = prob->p, T = prob->T;
  const int dt = prob->dtype;
  const int rule = opts ? opts->rule : GS_RULE_SPHERE;
  int rc;

  // once per problem: ||x_j||^2, x_j^T y, lambda_max, ||y||, bmc
  const int cgrid = grid_for((int64_t)p * 64, 256, 8192);
  if (dt == GS_F32) {
    hipLaunchKernelGGL(k_col_stats<float>, dim3(cgrid), dim3(256), 0, s,
                       static_cast<const float*>(prob->X), static_cast<const float*>(prob->y),
                       prob->ldx, n, p, w.nrm2, w.c);
    rc = last_launch("k_col_stats");
    if (rc) return rc;
    hipLaunchKernelGGL(k_absmax_ynorm<float>, dim3(1), dim3(256), 0, s, w.c, p,
                       static_cast<const float*>(prob->y), n, w.scal);
  } else {
    hipLaunchKernelGGL(k_col_stats<double>, dim3(cgrid), dim3(256), 0, s,
                       static_cast<const double*>(prob->X), static_cast<const double*>(prob->y),
                       prob->ldx, n, p, w.nrm2, w.c);
    rc = last_launch("k_col_stats");
    if (rc) return rc;
    hipLaunchKernelGGL(k_absmax_ynorm<double>, dim3(1), dim3(256), 0, s, w.c, p,
                       static_cast<const double*>(prob->y), n, w.scal);
  }
  rc = last_launch("k_absmax_ynorm");
  if (rc) return rc;
  if (params) {
    rc = launch_block_corr(n, p, prob->ldx, dt, prob->X, block, w.bmc, s);
    if (rc) return rc;
  }
  double host2[2];
  {
    hipError_t e = hipMemcpyAsync(host2, w.scal, sizeof(host2), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_hip_error(e, "lasso_path_learned: lambda_max");
  }
  const double lam_max = host2[0], ynorm = std::sqrt(host2[1]);
  if (learned_out) {
    rc = fill_i32(learned_out, T, 0, s);
    if (rc) return rc;
  }
  if (!(lam_max > 0.0) || !std::isfinite(lam_max) || !std::isfinite(ynorm)) {
    // degenerate or non-finite data: the plain path reports it
    rc = lasso_path(prob, opts, w.inner, w.inner_bytes, s);
    if (rc < 0) return rc;
    hipError_t e = hipStreamSynchronize(s);
    return e == hipSuccess ? rc : set_hip_error(e, "lasso_path_learned");
  }
  std::vector<double> lam(T);
  for (int t = 0; t < T; ++t) {
    if (prob->lambdas)
      lam[t] = prob->lambdas[t] * (prob->lambda_relative ? lam_max : 1.0);
    else
      lam[t] = T == 1 ? lam_max
                      : lam_max * std::pow(prob->lambda_min_ratio, (double)t / (double)(T - 1));
  }
  const int64_t P = p;
  int agg = GS_OK;
  gs_opts od;
  gs_opts_default(&od);
  const double eps_abs = (opts ? opts->eps_rel : od.eps_rel) * ynorm * ynorm;
  for (int t = 0; t < T; ++t) {
    const double* bprev = t == 0 ? prob->beta_init : prob->beta_out + (t - 1) * P;
    const double* startp = bprev;
    bool net_start = false;
    if (params && bprev) {
      // plain screening pass at the previous solution: A_plain and c
      rc = screen(n, p, prob->ldx, dt, prob->X, prob->y, bprev, lam[t], rule, nullptr, 0, w.act, w.q,
                  w.scal + 2, w.scal + 4, w.scal + 5, w.c, w.inner, w.inner_bytes, s);
      if (rc) return rc;
      rc = launch_features(p, w.c, bprev, w.nrm2, w.bmc, lam[t], lam_max, ynorm, w.U, s);
      if (rc) return rc;
      rc = launch_mlp_forward(params, w.U, p, w.out, s);
      if (rc) return rc;
      int32_t q = 0;
      hipError_t e = hipMemcpyAsync(&q, w.q, sizeof(q), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return set_hip_error(e, "lasso_path_learned: active size");
      bool emitted = false;
      if (q > 0 && q <= p && w.cap >= 1) {
        int m = 0;
        bool gap_known = false;
        rc = ws_start(prob, w, q, bprev, lam[t], rule, m, gap_known, s);
        if (rc) return rc;
        if (m >= 1 && gap_known) {
          // already certified on the safe set: Algorithm 1 would stop at its
          // first pass from this start, so lambda_t is output from it
          double g = INFINITY;
          hipError_t e3 = hipMemcpyAsync(&g, w.scal + 3, sizeof(g), hipMemcpyDeviceToHost, s);
          if (e3 == hipSuccess) e3 = hipStreamSynchronize(s);
          if (e3 != hipSuccess) return set_hip_error(e3, "lasso_path_learned: gap");
          if (g <= eps_abs) {
            hipLaunchKernelGGL(k_ws_emit, dim3(grid_for(p, 256)), dim3(256), 0, s, w.beta0, p,
                               prob->beta_out + t * P, w.scal + 3, w.q + 1, prob->gap_out + t,
                               prob->epochs_out + t, prob->nactive_out + t,
                               prob->status_out + t,
                               prob->lambda_out ? prob->lambda_out + t : nullptr, lam[t],
                               learned_out ? learned_out + t : nullptr);
            rc = last_launch("k_ws_emit");
            if (rc) return rc;
            emitted = true;
          }
        }
        if (m >= 1 && !emitted) {
          // both candidates' gaps on the reduced problem over A_plain
          rc = screen(n, p, prob->ldx, dt, prob->X, prob->y, bprev, lam[t], rule, w.act, q,
                      w.act2, w.q + 1, w.scal + 2, w.scal + 4, w.scal + 5, nullptr, w.inner,
                      w.inner_bytes, s);
          if (rc) return rc;
          rc = screen(n, p, prob->ldx, dt, prob->X, prob->y, w.beta0, lam[t], rule, w.act, q,
                      w.act2, w.q + 1, w.scal + 3, w.scal + 4, w.scal + 5, nullptr, w.inner,
                      w.inner_bytes, s);
          if (rc) return rc;
          hipLaunchKernelGGL(k_warm_choose, dim3(grid_for(p, 256)), dim3(256), 0, s, w.scal + 2,
                             w.scal + 3, w.beta0, bprev, p, w.start,
                             learned_out ? learned_out + t : nullptr, w.cnt + 12);
          rc = last_launch("k_warm_choose");
          if (rc) return rc;
          startp = w.start;
          int32_t taken = 0;
          hipError_t e2 = hipMemcpyAsync(&taken, w.cnt + 12, sizeof(taken), hipMemcpyDeviceToHost, s);
          if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
          if (e2 != hipSuccess) return set_hip_error(e2, "lasso_path_learned: choice");
          net_start = taken != 0;
        }
      }
      if (emitted) continue;
    }
    gs_problem sub = *prob;
    sub.T = 1;
    sub.lambdas = &lam[t];
    sub.lambda_relative = 0;
    sub.beta_init = startp;
    sub.beta_out = prob->beta_out + t * P;
    sub.gap_out = prob->gap_out + t;
    sub.epochs_out = prob->epochs_out + t;
    sub.nactive_out = prob->nactive_out + t;
    sub.status_out = prob->status_out + t;
    sub.lambda_out = prob->lambda_out ? prob->lambda_out + t : nullptr;
    // From the network's start the run is usually its first screening pass
    // alone: the wide schedule does that pass over the whole GPU, where the
    // narrow one spends a wavefront's prologue over all p columns.
    gs_opts so = opts ? *opts : gs_opts{};
    if (!opts) gs_opts_default(&so);
    if (net_start && so.schedule == GS_SCHED_AUTO) so.schedule = GS_SCHED_WIDE;
    rc = lasso_path(&sub, &so, w.inner, w.inner_bytes, s);
    if (rc < 0) return rc;
    if (rc == GS_NOT_CONVERGED) agg = GS_NOT_CONVERGED;
  }
  hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? agg : set_hip_error(e, "lasso_path_learned");
}

}  // extern "C"
