// Internal structures shared by the host dispatch code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

// Device-side descriptor of one Lasso path.  Built on the host, copied into
// the workspace, read by the kernels.  Pointers are device pointers.
struct ProbDesc {
  const void* X;           // dense: the design; CSC: the nonzero values
  const void* y;
  const int32_t* rows;
  const int64_t* col_ptr;  // CSC: p+1 offsets into row_idx and X
  const int32_t* row_idx;  // CSC: row of every nonzero
  int32_t format;          // 0 dense column-major, 1 CSC
  int64_t ldx;
  int32_t n, p, T, dtype;
  int32_t lambda_relative;
  int32_t has_lambdas;     // lam holds caller values (absolute or relative)
  double lambda_min_ratio;
  const double* beta_init;
  double* beta_out;
  double* gap_out;
  int32_t* epochs_out;
  int32_t* nactive_out;
  int32_t* status_out;
  double* lambda_out;
  // workspace arrays of this problem
  double* nrm2;   // p: ||x_j||^2
  double* inv;    // p: 1/||x_j||^2 (0 for a zero column)
  double* beta;   // p: working coefficients (FP64)
  double* c;      // p: x_j^T rho of the last sweep, indexed by position in A
  int32_t* act;   // 2p: active set (two buffers for the wide schedule)
  double* lam;    // T: the absolute lambdas of the path (set by the kernels)
  double* lam_in; // T: caller lambdas (absolute or relative), read only
  double* rho;    // n: residual (wide schedule)
  double* xty;    // p: x_j^T y (the dome test, the comparison rules)
  double* gst;    // p: x_j^T x_{j*} (the Dynamic ST3 rule)
  // pattern mode of the narrow schedule; the arrays hold ldg entries, so
  // that 256-position tiles never leave them
  float* gc;        // ns x ldg: Gram columns by slot, row j = feature j
  float* ng;        // ldg: ||G_{k,S}||_2 of the zero coordinates of A
  int32_t* pslot;   // ldg: slot holding the Gram column of feature j, or -1
  int32_t* pmem;    // ldg: 1 when position k is in the support list, else 0
  double* c2;       // ldg: second buffer of the correlations c
  int32_t* lst;     // 2p: positions of A the wide CD visits exactly, then their
                    // features (wide schedule)
  double* lval;     // 4p: per listed entry c_k, beta_j, 1/||x_j||^2, ||x_j||^2
  int64_t ldg;      // p rounded up to a multiple of 256
  int32_t ns;       // Gram slots of this problem (<= kSlotsMax)
  int32_t orig;     // index of the problem in the caller's array
};

// Largest number of Gram slots of one problem (and so the largest support
// handled by the pattern mode).
constexpr int kSlotsMax = 128;
// Counters of gs_opts.stats.
enum {
  kStatPatternEpochs = 0,  // epochs committed by the pattern mode
  kStatResidualEpochs,     // epochs run by the residual mode
  kStatRejected,           // pattern epochs rejected (re-run in residual mode)
  kStatBuilds,             // Gram columns computed
  kStatSetups,             // pattern set-ups
  kStatSupportChanges,     // set-ups whose support features changed
  kStatPasses,             // screening passes
  kStatSkipped,            // epochs skipped at an exact fixed point
  kStatExact,              // pattern epochs that needed the exact zero-coordinate check
  kStatNear,               // pattern epochs that checked at most 64 coordinates exactly
  kStatWideVisits,         // wide schedule: coordinates visited exactly by the CD rounds
  kStatWideRounds,         // wide schedule: CD rounds (an epoch or the part of one after
                           // a re-anchor)
  kStatWideStops,          // wide schedule: rounds that stopped to re-anchor
  kNumStats
};

struct PathOpts {
  double eps_rel;
  int32_t f, K;
  int32_t lds_cap;         // floats of LDS for staging the active coefficients
  int32_t pattern;         // 1: pattern mode allowed, 0: residual mode only
  int32_t gs_cap;          // floats of LDS for the support's Gram block
  int32_t rule;            // 0: GAP SAFE sphere, 1: sphere and GAP SAFE dome,
                           // 2-4: static SAFE, Dynamic Safe, Dynamic ST3
  int32_t* select_counts;  // T x p or null
  long long* timestamps;   // 2B or null
  long long* stats;        // kNumStats or null
  double enet;             // elastic net mixing alpha in (0, 1]; 1 = the Lasso
};

// Parameters of the warm-start network (4 -> 64 -> 64 -> 2), one FP32 array:
// W1 (64x4, row = hidden unit), b1, W2 (64x64, row = output unit), b2,
// W3 (2x64), b3.
constexpr int kMlpW1 = 0, kMlpB1 = 256, kMlpW2 = 320, kMlpB2 = 4416, kMlpW3 = 4480,
              kMlpB3 = 4608, kMlpParams = 4610;

// Records the text of a HIP failure for lasso_strerror and returns GS_EHIP.
int set_hip_error(hipError_t e, const char* where);

// ---- restricted solve and working sets of the learned start (gs_ws.hip).
constexpr int kWsMaxSet = 2047;  // largest working set (a system of at most 2048 unknowns)
size_t ws_solve_bytes(int m);
// (X_W^T X_W) b = X_W^T y - lambda sigma for the m columns W; info (device) = 0 on
// success, the 1-based row of a non-positive pivot, or -1 for an index outside [0, p).
int ws_solve(int n, int p, int64_t ldx, int dtype, const void* X, const void* y, const int32_t* W,
             const double* sigma, int m, double lambda, double* b_out, int32_t* info,
             void* workspace, hipStream_t s);
// cnt8[0] = |supp beta_prev within act|, cnt8[1 + i] = entrants (violators at beta_prev,
// |c_j| > lambda) with logit > taus[i] (7 taus)
int ws_count(const float* out, const int32_t* act, int q, const double* bprev, const double* c,
             double lambda, const float* taus, int32_t* cnt8, hipStream_t s);
int ws_select(const float* out, const int32_t* act, int q, const double* bprev, const double* c,
              double lambda, float tau, int cap, int32_t* W, double* sigma, int32_t* mark,
              int32_t* cnt, hipStream_t s);
int ws_drop(int32_t* W, double* sigma, double* b, int32_t* mark, const double* bprev,
            int32_t* cnt, hipStream_t s);
int ws_add(const int32_t* act, int q, const double* c, double lambda, int kadd, int cap,
           int32_t* W, double* sigma, int32_t* mark, int32_t* cnt, hipStream_t s);
int ws_scatter(const int32_t* W, const double* b, const int32_t* cnt, int p, double* beta0,
               hipStream_t s);

// Scalars of the wide schedule's state machine (one problem).
struct WideState {
  // set by init
  double lambda_max, ynorm2, eps;
  // current lambda
  int32_t t, k, q, full, cur;  // cur: which act buffer holds A
  int32_t done, phase;         // phase: 1 = a test is pending after the gap
  int32_t need_refresh, passes, status_acc, nonfinite;
  // last pass
  double gap, alpha_s, radius_s, e_c, M;
  double R2, Ry, l1, sbx, xmax;
  int32_t nnz, nblk_sweep, q_new, pad_;
  // CD rounds of the wide schedule: an epoch is walked from position
  // `resume`; zero coordinates whose anchored correlation keeps them at zero
  // while the residual moves by at most tau are skipped
  int32_t resume, first_epoch;
  double tau, tau_first, dmax2;
  double pb2;  // 2 P(beta) at the last pass: bounds ||rho||^2 of the CD iterates
  // dome parameters of the last pass (rule 1)
  double Rlo, Rhi, rc2lo, e_y;
  int32_t rule, jstar;
  // comparison rules (rules 2-4): x_{j*} and the sphere of the last pass
  double sstar, nstar, shift, rad_s, e_shift;
  double enet;  // elastic net alpha (1: the Lasso)
  long long n_visits, n_rounds, n_stops, n_epochs;
};

// Kernel configuration: rows per lane layout.  S lanes share one column
// (a "segment" of the column each), C = 64/S columns are processed at once.
struct Cfg {
  int id;
  int dtype;   // 0 f32, 1 f64
  int vec;     // elements per 16-byte load (4 f32, 2 f64) or 1 (scalar)
  int S, NG;   // lanes per column, row groups per lane
  int gather;  // 1: rows come from an index list
  int nmax() const { return S * NG * vec; }
};

}  // namespace gs
