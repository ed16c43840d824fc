// The per-problem ("narrow") schedule: one wavefront runs Algorithm 1 for one
// Lasso path, with the residual in LDS (canonical copy) and in registers
// (working copy in the column layout), and X streamed from L2/HBM.
//
// Column layout: lane = slot * S + seg.  Each of the C = 64/S slots works on
// its own column; the S lanes of a slot split that column's rows.  A column
// dot product is a per-lane FMA chain followed by a butterfly over S lanes.
//
// The epochs between two screening passes run in one of two modes; both are
// cyclic CD over the active set A in ascending order (Algorithm 1) and make
// the same updates up to the order of rounding:
//
//  * pattern mode.  Let S be the positions of A whose coefficient is nonzero
//    (s of them, ascending), sigma their signs and g = X_A^T rho the
//    correlations at the start of an epoch.  As long as no coordinate of S
//    changes sign or reaches zero and no other coordinate leaves zero, the
//    epoch is a linear map: its steps delta solve
//        (D + L) delta = g_S - lambda sigma,
//    with D + L the diagonal and lower part of the Gram matrix G_SS in the
//    cyclic order, and a zero coordinate k is visited with the correlation
//    g_k - sum_{m in S before k} G_km delta_m.  The mode solves the system by
//    forward substitution, then checks the premise exactly: the signs of
//    beta_S + delta, and |g_k| + sum_m |G_km delta_m| <= lambda for every zero
//    coordinate (a bound on its correlation at its visit, so that it stays
//    at zero).  If both hold, the result is the cyclic epoch's and it is
//    committed (beta_S += delta, g -= G_{A,S} delta); otherwise nothing is
//    written and the residual mode runs that epoch.  The Gram columns of S
//    over A sit in a global (L2-resident) cache indexed by position; they
//    follow the compactions of A and are computed again for a new lambda.
//    The columns and the substitution are FP32, the coefficients and g FP64;
//    the FP32 error on g is proportional to the steps, and every screening
//    pass recomputes g from a fresh residual.
//
//  * residual mode.  A chunk of C consecutive active coordinates: the C dot
//    products x_j^T rho are formed at once against the current residual; the
//    chunk is then resolved in order: the first coordinate whose
//    soft-threshold update changes beta is applied (rho -= delta x_j), the
//    later dot products of the chunk are recomputed against the new residual,
//    and the scan continues after it.  Column loads are software-pipelined
//    two chunks ahead; beta and 1/||x_j||^2 of the active positions sit in
//    LDS, so the loop's only global traffic is X.
//
// Lanes of one wavefront order their LDS accesses without block barriers, so
// pending global loads are never drained inside the loops.
#pragma once

#include <type_traits>

#include "gs_device.hpp"

namespace gs {

// The constant address space: a wave-uniform load through such a pointer is
// a scalar load, whose completion is counted apart from the vector loads.
// Only for data that no wave writes while the kernel runs.
template <typename T>
using cst = __attribute__((address_space(4))) T;

__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
// v with lane LANE replaced by the uniform value w (one v_writelane_b32).
template <int LANE>
__device__ __forceinline__ float writelane_f(float v, float w) {
  int r = __float_as_int(v);
  asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(r) : "s"(__float_as_int(w)), "i"(LANE));
  return __int_as_float(r);
}

template <typename XT, int VEC, int S, int NG, bool GATHER>
struct Narrow {
  using L = ColLayout<XT, VEC, S, NG, GATHER>;
  static constexpr int RPL = L::RPL;
  static constexpr int C = L::C;
  static constexpr int NMAX = L::NMAX;
  static constexpr int NT = (NMAX + 63) / 64;        // rows per lane, row-major layout
  static constexpr int NB = NT <= 2 ? 8 : (NT <= 4 ? 4 : (NT <= 8 ? 2 : 1));  // refresh batch
  static constexpr int U = RPL <= 8 ? 4 : (RPL <= 24 ? 3 : (RPL <= 32 ? 2 : 1));  // sweep batch
  static constexpr int NSC = kSlotsMax;          // Gram slots (largest support in pattern mode)
  static constexpr int NBLD = RPL <= 20 ? 4 : 2;  // Gram columns computed per sweep of A

  // Per-wave context.
  struct Ctx {
    const gbl<XT>* X;
    int64_t ldx;
    int n, p;
    int lane, slot, seg;
    int ridx[GATHER ? NG : 1];  // gather: clamped source row of (seg, m)
    uint64_t mk;                // bit i set when the lane's row i is < n
    double* y_l;                // LDS, n
    double* rho_l;              // LDS, n
    XT* tile;                   // LDS, 64 * RPL
    int* rows_l;                // LDS, n (gather)
    float* stg;                 // LDS staging region of the residual mode
    int stg_cap;                // its size in floats
    gbl<double>* nrm2;
    gbl<double>* xty;           // x_j^T y (the dome test)
    gbl<double>* inv;           // 1/||x_j||^2 (0 for a zero column)
    gbl<double>* beta;
    gbl<double>* c;             // correlations by position (one of two buffers)
    gbl<int32_t>* act;
    const cst<int32_t>* act_c;  // act, read-only view (kernels that never write A)
  };

  // Pattern-mode state.  Scalars are wavefront-uniform; sp..u hold the
  // support members m = lane (index 0) and m = lane + 64 (index 1).
  struct Pat {
    gbl<float>* gc;       // slot v: x_j^T x_{owner[v]} at gc[v*ldg + j] for features j of A
    gbl<float>* ng;       // position -> ||G_{k,S}||_2 (zero coordinates of A)
    gbl<int32_t>* pslot;  // feature -> slot, or -1
    gbl<int32_t>* pmem;   // position -> 1 when in S, else 0 (set up with S)
    gbl<double>* c2;      // the other correlation buffer
    int64_t ldg;
    int ns;               // slots of this problem
    int gs_cap;           // LDS floats of the block
    int* owner;           // LDS ns: feature whose column a slot holds, or -1
    int* spos;            // LDS NSC: positions of S
    int* sfeat;           // LDS NSC: features of S when the block was built
    int* cand;            // LDS 64: zero coordinates whose bound failed
    int* bslot;           // LDS NBLD: slots of the columns being computed
    int* bfeat;           // LDS NBLD: their features
    float* stage;         // LDS NBLD x NMAX: those columns
    float* gs;            // LDS: column l of G_SS / ||x_m||^2 at gs[l*gsp + m], 1 on the diagonal
    int s;                // |S|
    int gsp;              // column stride of gs (64 or 128)
    int s_t;              // |S| when the block was built (-1: never)
    int victim;           // round-robin cursor of the slot search
    bool valid;           // registers and block describe the current S and c
    bool ng_ok;           // ng holds the row norms for S over the current A
    double tau;           // min over zero coordinates of (lambda - |c0_k|) / ng_k
    int sp[2], sl[2], sj[2];
    double sb[2], b0[2], sg[2];
    float id[2], u[2];
  };

  struct Stage {
    XT x[RPL];
    double b, inv;
    int j, k;
    bool v;
  };

  static __device__ __forceinline__ const gbl<XT>* col(const Ctx& x, int j) {
    return x.X + (int64_t)j * x.ldx;
  }
  static __device__ __forceinline__ int src_row(const Ctx& x, int i) {
    if constexpr (GATHER) return x.rows_l[i];
    return i;
  }

  static __device__ __forceinline__ void setup(Ctx& x, const gbl<int32_t>* rows) {
    x.mk = L::rowmask(x.seg, x.n);
    if constexpr (GATHER) {
      for (int i = x.lane; i < x.n; i += 64) x.rows_l[i] = rows[i];
      wave_lds_order();
#pragma unroll
      for (int m = 0; m < NG; ++m) {
        int r = x.seg + S * m;
        x.ridx[m] = x.rows_l[r < x.n ? r : 0];
      }
    }
  }

  static __device__ __forceinline__ int act_at(const Ctx& x, int k, int q, bool full) {
    const int kk = k < q ? k : q - 1;
    return full ? kk : x.act[kk];
  }

  // Issues the loads of the column, coefficient and 1/||x||^2 of position k
  // of A (clamped to the last position; s.v says whether k is in A).  With
  // POSL the coefficient and the inverse norm come from the LDS position
  // arrays.  Nothing here consumes the loaded values.
  template <bool POSL>
  static __device__ __forceinline__ void fetch_j(const Ctx& x, int k, int j, int q,
                                                 const double* pb, const double* pinv,
                                                 Stage& s) {
    s.v = k < q;
    s.j = j;
    s.k = k < q ? k : q - 1;
    L::load_raw(col(x, j), x.n, x.seg, x.ridx, s.x);
    if constexpr (POSL) {
      s.b = pb[s.k];
      s.inv = pinv[s.k];
    } else {
      s.b = x.beta[j];
      s.inv = x.inv[j];
    }
  }

  static __device__ __forceinline__ double dotd(const double (&xd)[RPL], const double (&r)[RPL]) {
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; i += 2) {
      a0 = fma(xd[i], r[i], a0);
      if (i + 1 < RPL) a1 = fma(xd[i + 1], r[i + 1], a1);
    }
    return seg_sum<S>(a0 + a1);
  }
  // dot of a raw column with a vector whose rows >= n are zero (the raw rows
  // >= n are finite copies of row 0, so they contribute nothing)
  static __device__ __forceinline__ double dotx(const XT (&xv)[RPL], const double (&r)[RPL]) {
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; i += 2) {
      a0 = fma((double)xv[i], r[i], a0);
      if (i + 1 < RPL) a1 = fma((double)xv[i + 1], r[i + 1], a1);
    }
    return seg_sum<S>(a0 + a1);
  }

  // A vector indexed by problem row, in the column layout (zero padded).
  static __device__ __forceinline__ void load_rows(const Ctx& x, const double* v_l, double (&r)[RPL]) {
#pragma unroll
    for (int m = 0; m < NG; ++m)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        int i = L::row(x.seg, m, e);
        r[m * VEC + e] = (i < x.n) ? v_l[i] : 0.0;
      }
  }

  // rho = y - sum_{j in A, beta_j != 0} beta_j x_j (ascending j), written to
  // LDS.  Returns nnz; R2 = ||rho||^2 and Ry = y^T rho.  (Sec. 2.3.)
  static __device__ __forceinline__ int refresh(const Ctx& x, int q, bool full, double& R2, double& Ry) {
    double rr[NT];
    int rw[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      int i = x.lane + 64 * t;
      rr[t] = (i < x.n) ? x.y_l[i] : 0.0;
      rw[t] = src_row(x, (i < x.n) ? i : 0);
    }
    int nnz = 0;
    for (int base = 0; base < q; base += 256) {
      int jv[4];
      double bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) jv[u] = act_at(x, base + 64 * u + x.lane, q, full);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double b = x.beta[jv[u]];
        bv[u] = (base + 64 * u + x.lane < q) ? b : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        uint64_t m = ballot(bv[u] != 0.0);
        nnz += __popcll(m);
        const int jpad = __builtin_amdgcn_readfirstlane(jv[u]);
        while (m) {
          int jj[NB];
          double bb[NB];
#pragma unroll
          for (int e = 0; e < NB; ++e) {
            if (m) {
              int l = __builtin_ctzll(m);
              m &= m - 1;
              jj[e] = __builtin_amdgcn_readlane(jv[u], l);
              bb[e] = readlane_d(bv[u], l);
            } else {
              jj[e] = jpad;  // a valid column with a zero weight
              bb[e] = 0.0;
            }
          }
          XT xs[NB][NT];
#pragma unroll
          for (int e = 0; e < NB; ++e)
#pragma unroll
            for (int t = 0; t < NT; ++t) xs[e][t] = col(x, jj[e])[rw[t]];
#pragma unroll
          for (int e = 0; e < NB; ++e)
#pragma unroll
            for (int t = 0; t < NT; ++t) rr[t] = fma(-bb[e], (double)xs[e][t], rr[t]);
        }
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
    wave_lds_order();
    return nnz;
  }

  // c_k = x_{A[k]}^T rho for every position k of A; M = max |c_k|,
  // l1 = ||beta||_1, sbx = sum |beta_j| ||x_j||, xmax = max ||x_j|| over A.
  static __device__ __forceinline__ void sweep(const Ctx& x, int q, bool full, double& M, double& l1,
                               double& sbx, double& xmax) {
    double r[RPL];
    load_rows(x, x.rho_l, r);
    double Ml = 0.0, l1l = 0.0, sbl = 0.0, xml = 0.0;
    // The column indices of the next step are loaded a step ahead; every
    // lane of a slot stores the slot's value, positions past the end
    // clamped to the last one (whose value is stored again, the same), so
    // that the step has no data-dependent branch and its memory waits stay
    // exact.
    int jn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) jn[u] = q > 0 ? act_at(x, u * C + x.slot, q, full) : 0;
    for (int base = 0; base < q; base += U * C) {
      Stage st[U];
      double nr[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = base + u * C + x.slot;
        fetch_j<false>(x, k, jn[u], q, nullptr, nullptr, st[u]);
        nr[u] = x.nrm2[st[u].j];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) jn[u] = act_at(x, base + (U + u) * C + x.slot, q, full);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double d = dotx(st[u].x, r);
        x.c[st[u].k] = d;
        const bool own = st[u].v && x.seg == 0;  // one contribution per position
        const double xn = sqrt(nr[u]);
        const double ab = own ? fabs(st[u].b) : 0.0;
        Ml = fmax(Ml, own ? fabs(d) : 0.0);
        l1l += ab;
        sbl += ab * xn;
        xml = fmax(xml, own ? xn : 0.0);
      }
    }
    M = wave_max(Ml);
    l1 = wave_sum(l1l);
    sbx = wave_sum(sbl);
    xmax = wave_max(xml);
    __threadfence_block();
  }

  // Sphere test over A with ordered in-place compaction of A and c; screened
  // nonzero coefficients are set to zero (dropped_nz is then set).  With np,
  // the new position of every old one (-1 when dropped) is recorded; fv, a
  // per-position array, moves with c.
  static __device__ __forceinline__ int test_compact(const Ctx& x, const GapInfo& g, int q, bool full,
                                     bool& dropped_nz, gbl<int32_t>* np = nullptr,
                                     gbl<float>* fv = nullptr) {
    int q2 = 0;
    bool dn = false;
    const uint64_t lt = (x.lane == 0) ? 0ull : (~0ull >> (64 - x.lane));
    for (int base = 0; base < q; base += 256) {
      int jv[4];
      double cv[4], nv[4], bv[4];
      float fw[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = base + 64 * u + x.lane;
        jv[u] = act_at(x, k, q, full);
        cv[u] = x.c[k < q ? k : q - 1];
        fw[u] = fv ? fv[k < q ? k : q - 1] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        nv[u] = x.nrm2[jv[u]];
        bv[u] = x.beta[jv[u]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = base + 64 * u + x.lane;
        const bool v = k < q;
        bool keep = v && sphere_keep(g, cv[u], nv[u], x.n);
        if (g.dome && keep) keep = dome_keep(g, x.xty[jv[u]], cv[u], nv[u], x.n);
        if (v && !keep && bv[u] != 0.0) {
          x.beta[jv[u]] = 0.0;
          dn = true;
        }
        const uint64_t m = ballot(keep);
        const int pos = q2 + __popcll(m & lt);
        if (keep) {
          x.act[pos] = jv[u];
          x.c[pos] = cv[u];  // c of kept coordinates moves with them
          if (fv) fv[pos] = fw[u];
        }
        if (np && v) np[k] = keep ? pos : -1;
        q2 += __popcll(m);
      }
    }
    dropped_nz = ballot(dn) != 0;
    __threadfence_block();
    return q2;
  }

  // ---- residual mode -------------------------------------------------------

  // Resolves one chunk whose loads (stage s) have landed: the C dot products
  // against the current residual, then the in-order soft-threshold scan.
  template <bool POSL>
  static __device__ __forceinline__ void resolve(const Ctx& x, const Stage& s, double lambda,
                                                 double* pb, double (&r)[RPL]) {
    // Rows >= n hold copies of row 0: they meet zeros of the residual in the
    // dot products, and are zeroed in the tile that updates the residual.
    // With one column per chunk the lane's own registers are that tile.
    XT* mytile = x.tile + x.lane * RPL;
    double xd[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      xd[i] = (double)s.x[i];
      if constexpr (C > 1) mytile[i] = ((x.mk >> i) & 1ull) ? s.x[i] : XT(0);
    }
    double b = s.b;
    const double inv = s.inv;
    const bool live = s.v && inv > 0.0;
    const double thr = lambda * inv;
    double d = dotd(xd, r);
    wave_lds_order();
    int start = 0;
    bool changed = false;
    for (;;) {
      bool chg = false;
      double bn = b;
      if (live && x.slot >= start) {
        bn = soft_thr(thr, b + d * inv);
        chg = (bn != b);
      }
      const uint64_t mk = ballot(chg);
      if (!mk) break;
      const int l0 = __builtin_ctzll(mk);
      const int cs = l0 / S;
      const double delta = readlane_d(bn - b, l0);
      if (x.slot == cs) {
        b = bn;
        changed = true;
      }
      if constexpr (C == 1) {
#pragma unroll
        for (int i = 0; i < RPL; ++i)
          r[i] = fma(-delta, ((x.mk >> i) & 1ull) ? xd[i] : 0.0, r[i]);
        break;
      } else {
        const XT* tx = x.tile + (cs * S + x.seg) * RPL;
#pragma unroll
        for (int i = 0; i < RPL; ++i) r[i] = fma(-delta, (double)tx[i], r[i]);
      }
      if (cs + 1 >= C) break;
      d = dotd(xd, r);
      start = cs + 1;
    }
    if (changed && x.seg == 0) {
      if constexpr (POSL)
        pb[s.k] = b;
      else
        x.beta[s.j] = b;
    }
    wave_lds_order();
  }

  // Depth of the load ring: with one column per chunk (S = 64) a chunk's
  // work is short against the latency of its column, so more columns are in
  // flight where a stage is small enough (up to 64 bytes per lane) to stay
  // in registers.
  static constexpr int RING = (C == 1 && RPL * sizeof(XT) <= 64) ? 6 : 3;

  // The column index at position k of A for the load ring.  With CA (A is
  // not written while the kernel runs) and one column per chunk the
  // position is wave-uniform and the index comes by a scalar load: a vector
  // load of it would be counted in order with the column loads in flight,
  // and waiting for it would wait for all of them.
  // With POSL the indices were staged in LDS (pa) with the coefficients.
  template <bool POSL, bool CA>
  static __device__ __forceinline__ int ring_ix(const Ctx& x, int k, int q, bool full,
                                                const int* pa) {
    if constexpr (POSL) {
      return pa[k < q ? k : q - 1];
    } else if constexpr (CA && C == 1) {
      const int kk = __builtin_amdgcn_readfirstlane(k < q ? k : q - 1);
      return full ? kk : x.act_c[kk];
    } else {
      return act_at(x, k, q, full);
    }
  }

  // Steps CUR.. of one round of the RING-deep load ring.  The chunk at
  // P = base + CUR C sits in st[CUR]; the loads of chunk P + (RING-1) C go
  // into the stage freed last round, with the index fetched one step
  // earlier, and the index of chunk P + RING C is requested.
  template <int CUR, bool POSL, bool CA>
  static __device__ __forceinline__ bool ring_steps(const Ctx& x, int base, int q, bool full,
                                                    double lambda, double* pb,
                                                    const double* pinv, const int* pa,
                                                    Stage (&st)[RING], int (&ix)[RING],
                                                    double (&r)[RPL]) {
    if constexpr (CUR < RING) {
      constexpr int NXT = (CUR + RING - 1) % RING;
      const int P = base + CUR * C;
      fetch_j<POSL>(x, P + (RING - 1) * C + x.slot, ix[NXT], q, pb, pinv, st[NXT]);
      ix[CUR] = ring_ix<POSL, CA>(x, P + RING * C + x.slot, q, full, pa);
      resolve<POSL>(x, st[CUR], lambda, pb, r);
      if (P + C >= q) return true;
      return ring_steps<CUR + 1, POSL, CA>(x, base, q, full, lambda, pb, pinv, pa, st, ix, r);
    } else {
      return false;
    }
  }

  // One cyclic CD epoch over A (Algorithm 1):
  //   beta_j <- ST(lambda/||x_j||^2, beta_j + x_j^T rho / ||x_j||^2),
  //   rho    <- rho - (beta_j' - beta_j) x_j.
  // The epoch may start at position k0 > 0: positions before k0 are left
  // alone.  Positions past the end are clamped to the last one (q >= 1).
  template <bool POSL, bool CA>
  static __device__ __forceinline__ void cd_epoch(const Ctx& x, int q, bool full, double lambda, double* pb,
                                  const double* pinv, const int* pa, double (&r)[RPL], int k0) {
    if (q <= k0) return;
    const int b0 = k0 - k0 % C;
    Stage st[RING];
    int ix[RING];
#pragma unroll
    for (int i = 0; i < RING; ++i) ix[i] = ring_ix<POSL, CA>(x, b0 + i * C + x.slot, q, full, pa);
#pragma unroll
    for (int i = 0; i + 1 < RING; ++i) fetch_j<POSL>(x, b0 + i * C + x.slot, ix[i], q, pb, pinv, st[i]);
    st[0].v = st[0].v && b0 + x.slot >= k0;
    for (int base = b0;; base += RING * C)
      if (ring_steps<0, POSL, CA>(x, base, q, full, lambda, pb, pinv, pa, st, ix, r)) break;
  }

  // ne residual-mode epochs (the first one from position k0), the residual
  // taken from and returned to LDS.  With room for 20 q bytes in the staging
  // region, the column index, beta and 1/||x||^2 of the active positions are
  // staged in LDS for the interval.
  template <bool CA = false>
  static __device__ __forceinline__ void cd_epochs(const Ctx& x, int q, bool full, double lambda,
                                   int ne, int k0) {
    double r[RPL];
    load_rows(x, x.rho_l, r);
    const bool posl = q > 0 && (size_t)q * (2 * sizeof(double) + sizeof(int)) <=
                                   (size_t)x.stg_cap * sizeof(float);
    if (posl) {
      double* pb = reinterpret_cast<double*>(x.stg);
      double* pinv = pb + q;
      int* pa = reinterpret_cast<int*>(pinv + q);
      for (int k = x.lane; k < q; k += 64) {
        const int j = full ? k : x.act[k];
        pa[k] = j;
        pb[k] = x.beta[j];
        pinv[k] = x.inv[j];
      }
      wave_lds_order();
      for (int e = 0; e < ne; ++e)
        cd_epoch<true, CA>(x, q, full, lambda, pb, pinv, pa, r, e == 0 ? k0 : 0);
      for (int k = x.lane; k < q; k += 64) x.beta[pa[k]] = pb[k];
    } else {
      for (int e = 0; e < ne; ++e)
        cd_epoch<false, CA>(x, q, full, lambda, nullptr, nullptr, nullptr, r, e == 0 ? k0 : 0);
    }
    __threadfence_block();
#pragma unroll
    for (int m = 0; m < NG; ++m)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int i = L::row(x.seg, m, e);
        // every slot holds the same copy; slot 0 writes it back
        if (x.slot == 0 && i < x.n) x.rho_l[i] = r[m * VEC + e];
      }
    wave_lds_order();
  }

  // ---- pattern mode ----------------------------------------------------------
  //
  // State of a pattern (set up after a screening pass or a residual-mode
  // epoch, when c = X_A^T rho is exact):
  //   * the support list S (positions ascending), with per member m: the
  //     coefficient b_m, its sign sigma_m, 1/||x_m||^2 and
  //     u_m = (g_m - lambda sigma_m) / ||x_m||^2, the scaled gradient gap;
  //   * the Gram block of S, G_SS / ||x_m||^2 column by column in LDS;
  //   * an anchor: beta0 = beta_S and c0 = c at the last exact point, and for
  //     every zero coordinate k of A the row norm ng_k = ||G_{k,S}||_2, with
  //     tau = min_k (lambda - |c0_k|) / ng_k.
  // An epoch is the forward substitution on the block (its running vector is
  // u itself: step l takes delta_l = u_l and subtracts delta_l times column l
  // from u; the diagonal entry is 1, so u_l becomes 0 as in the coordinate
  // update, and u ends as the next epoch's gradient gap).  A zero coordinate
  // k is then visited with the correlation c0_k - G_{k,S} (Delta + delta
  // restricted to members before k), Delta = beta_S - beta0; its size is at
  // most |c0_k| + ng_k (||Delta||_2 + ||delta||_2) by Cauchy-Schwarz, so
  // ||Delta||_2 + ||delta||_2 < tau proves that every zero coordinate stays
  // at zero.  Otherwise the bound is applied coordinate by coordinate, and
  // the few coordinates it leaves open (at most 64) get the exact value at
  // their visit from the Gram columns of S in the global cache; with more,
  // the exact check covers all of A and moves the anchor to the new point.
  // The global cache is indexed by feature and only holds the rows of the
  // current lambda's active set, so a new lambda starts it afresh.

  // A new lambda: the active set restarts from all of {0..p-1}.
  static __device__ __forceinline__ void pattern_new_lambda(const Ctx& x, Pat& pt) {
    for (int v = x.lane; v < pt.ns; v += 64) pt.owner[v] = -1;
    for (int j = x.lane; j < x.p; j += 64) pt.pslot[j] = -1;
    pt.victim = 0;
    pt.valid = false;
    pt.ng_ok = false;
    wave_lds_order();
    __threadfence_block();
  }

  // Gram columns of the nb features in bfeat into the slots bslot:
  // gc[v*ldg + A[k]] = x_{A[k]}^T x_j for every position k < q, in one sweep.
  static __device__ __forceinline__ void build_cols(const Ctx& x, const Pat& pt, int q, bool full,
                                                    int nb) {
#pragma unroll
    for (int b = 0; b < NBLD; ++b) {
      if (b < nb) {
        const int j = __builtin_amdgcn_readfirstlane(pt.bfeat[b]);
        const gbl<XT>* cj = col(x, j);
        for (int i = x.lane; i < NMAX; i += 64)
          pt.stage[b * NMAX + i] = i < x.n ? (float)cj[src_row(x, i)] : 0.f;
      }
    }
    wave_lds_order();
    float v[NBLD][RPL];
    gbl<float>* dst[NBLD];
#pragma unroll
    for (int b = 0; b < NBLD; ++b) {
#pragma unroll
      for (int m = 0; m < NG; ++m)
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[b][m * VEC + e] = pt.stage[b * NMAX + L::row(x.seg, m, e)];
      const int sl = __builtin_amdgcn_readfirstlane(pt.bslot[b]);
      dst[b] = pt.gc + (int64_t)(b < nb ? sl : 0) * pt.ldg;
    }
    constexpr int UB = 2;
    for (int base = 0; base < q; base += UB * C) {
      XT xr[UB][RPL];
      int jr[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        jr[u] = act_at(x, base + u * C + x.slot, q, full);
        L::load_raw(col(x, jr[u]), x.n, x.seg, x.ridx, xr[u]);
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int k = base + u * C + x.slot;
#pragma unroll
        for (int b = 0; b < NBLD; ++b) {
          if (b < nb) {
            // rows >= n: raw copies of row 0 meet zeros of the staged column
            float a0 = 0.f, a1 = 0.f;
#pragma unroll
            for (int i = 0; i < RPL; i += 2) {
              a0 = fmaf((float)xr[u][i], v[b][i], a0);
              if (i + 1 < RPL) a1 = fmaf((float)xr[u][i + 1], v[b][i + 1], a1);
            }
            const double dsum = seg_sum<S>((double)a0 + (double)a1);
            if (x.seg == 0 && k < q) dst[b][jr[u]] = (float)dsum;
          }
        }
      }
    }
    __threadfence_block();
    wave_lds_order();
  }

  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
  typedef int i4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ void ld4(const gbl<float>* p, float (&o)[4]) {
    const f4 v = *reinterpret_cast<const gbl<f4>*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
  static __device__ __forceinline__ void ld4(const gbl<double>* p, double (&o)[4]) {
    const d2 a = *reinterpret_cast<const gbl<d2>*>(p);
    const d2 b = *reinterpret_cast<const gbl<d2>*>(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  }
  static __device__ __forceinline__ void ld4(const gbl<int32_t>* p, int (&o)[4]) {
    const i4 v = *reinterpret_cast<const gbl<i4>*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }

  // (lambda - |c|) / ng, with the FP32 row norm rounded up; a coordinate that
  // no support column touches stays at zero iff |c| <= lambda.
  static __device__ __forceinline__ double slack_ratio(double c, float ng, double lambda) {
    const double sl = lambda - fabs(c);
    if (ng > 0.f) return sl / ((double)ng * (1.0 + 1e-5));
    return sl >= 0.0 ? INFINITY : -1.0;
  }

  // Row norms ng_k = ||G_{k,S}||_2 of the zero coordinates of A (when
  // recompute) and tau = min (lambda - |c_k|) / ng_k over them.  Lane
  // positions base + 4 lane + e.
  static __device__ __forceinline__ double row_norms_tau(const Ctx& x, const Pat& pt, int q,
                                                         double lambda, bool recompute) {
    const int s = __builtin_amdgcn_readfirstlane(pt.s);
    double tau = INFINITY;
    for (int base = 0; base < q; base += 256) {
      const int k0 = base + 4 * x.lane;
      double cv[4];
      int mb[4];
      float nv[4];
      ld4(x.c + k0, cv);
      ld4(pt.pmem + k0, mb);
      if (recompute) {
        int jv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) jv[e] = act_at(x, k0 + e, q, false);
        float a[4] = {0.f, 0.f, 0.f, 0.f};
        for (int m0 = 0; m0 < s; m0 += 8) {
          float g[8][4];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int m = m0 + u;
            const int sl = m < s ? (m < 64 ? __builtin_amdgcn_readlane(pt.sl[0], m)
                                           : __builtin_amdgcn_readlane(pt.sl[1], m - 64))
                                 : 0;
            const gbl<float>* gcol = pt.gc + (int64_t)sl * pt.ldg;
#pragma unroll
            for (int e = 0; e < 4; ++e) g[u][e] = m < s ? gcol[jv[e]] : 0.f;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) a[e] = fmaf(g[u][e], g[u][e], a[e]);
        }
        typedef float f4v __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int e = 0; e < 4; ++e) nv[e] = sqrtf(a[e]);
        *reinterpret_cast<gbl<f4v>*>(pt.ng + k0) = f4v{nv[0], nv[1], nv[2], nv[3]};
      } else {
        ld4(pt.ng + k0, nv);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (k0 + e < q && !mb[e]) tau = fmin(tau, slack_ratio(cv[e], nv[e], lambda));
    }
    __threadfence_block();
    return wave_min(tau);
  }

  // Sets up the pattern of the current coefficients over A (requires c =
  // X_A^T rho for the current beta).  Returns false when the support exceeds
  // the slots or the LDS block.
  static __device__ __forceinline__ bool pattern_setup(const Ctx& x, Pat& pt, int q, bool full,
                                                       double lambda, int (&stc)[kNumStats]) {
    const uint64_t lt = (x.lane == 0) ? 0ull : (~0ull >> (64 - x.lane));
    int s = 0;
    for (int base = 0; base < q; base += 256) {
      int jv[4];
      double bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) jv[t] = act_at(x, base + 64 * t + x.lane, q, full);
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[t] = x.beta[jv[t]];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = base + 64 * t + x.lane;
        const bool nz = k < q && bv[t] != 0.0;
        const uint64_t m = ballot(nz);
        const int idx = s + __popcll(m & lt);
        if (nz && idx < NSC) pt.spos[idx] = k;
        if (k < q) pt.pmem[k] = nz ? 1 : 0;
        s += __popcll(m);
      }
    }
    s = __builtin_amdgcn_readfirstlane(s);
    __threadfence_block();
    wave_lds_order();
    const int sps = s > 64 ? 128 : 64;
    const int s8 = (s + 7) & ~7;
    if (s > pt.ns || s8 * sps > pt.gs_cap) return false;
    ++stc[kStatSetups];
    pt.s = s;
    pt.gsp = sps;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int m = x.lane + 64 * h;
      const bool v = m < s;
      const int k = v ? pt.spos[m] : 0;
      const int j = act_at(x, k, q, full);
      pt.sp[h] = v ? k : 0x3fffffff;
      pt.sj[h] = j;
      pt.sb[h] = v ? x.beta[j] : 0.0;
      pt.sg[h] = pt.sb[h] > 0.0 ? 1.0 : -1.0;
      pt.id[h] = v ? (float)x.inv[j] : 0.f;
      pt.sl[h] = v ? pt.pslot[j] : 0;
      pt.b0[h] = pt.sb[h];
      pt.u[h] = v ? (float)(x.c[k] - lambda * pt.sg[h]) * pt.id[h] : 0.f;
    }
    // a slot for every member, the missing columns computed NBLD at a time
    bool failed = false;
    while (!failed) {
      uint64_t need0 = ballot(x.lane < s && pt.sl[0] < 0);
      uint64_t need1 = ballot(x.lane + 64 < s && pt.sl[1] < 0);
      if (!need0 && !need1) break;
      int nb = 0;
      while (nb < NBLD && (need0 || need1)) {
        int m;
        if (need0) {
          m = __builtin_ctzll(need0);
          need0 &= need0 - 1;
        } else {
          m = 64 + __builtin_ctzll(need1);
          need1 &= need1 - 1;
        }
        // a slot whose owner is not in S (there is one: s <= ns and m has
        // none); the scan is bounded all the same
        int v = 0, o = 0;
        bool found = false;
        for (int tries = 0; tries < pt.ns && !found; ++tries) {
          v = pt.victim;
          pt.victim = v + 1 < pt.ns ? v + 1 : 0;
          o = __builtin_amdgcn_readfirstlane(pt.owner[v]);
          found = o < 0 || x.beta[o] == 0.0;
        }
        if (!found) {
          failed = true;
          break;
        }
        const int jm = m < 64 ? __builtin_amdgcn_readlane(pt.sj[0], m)
                              : __builtin_amdgcn_readlane(pt.sj[1], m - 64);
        wave_lds_order();
        if (x.lane == 0) {
          if (o >= 0) pt.pslot[o] = -1;
          pt.pslot[jm] = v;
          pt.owner[v] = jm;
          pt.bslot[nb] = v;
          pt.bfeat[nb] = jm;
        }
        if (m < 64) {
          if (x.lane == m) pt.sl[0] = v;
        } else {
          if (x.lane == m - 64) pt.sl[1] = v;
        }
        ++nb;
      }
      wave_lds_order();
      if (nb) build_cols(x, pt, q, full, nb);  // every assigned slot gets its column
      stc[kStatBuilds] += nb;
    }
    if (failed) return false;
    // the block depends on the features of S only
    bool same = (s == pt.s_t);
    if (same) {
      bool diff = false;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = x.lane + 64 * h;
        if (m < s && pt.sfeat[m] != pt.sj[h]) diff = true;
      }
      same = ballot(diff) == 0;
    }
    if (!same) {
      ++stc[kStatSupportChanges];
      // columns s..s8-1 are zero: the substitution runs whole groups of 8
      for (int l = 0; l < s8; ++l) {
        const int vl = l < s ? (l < 64 ? __builtin_amdgcn_readlane(pt.sl[0], l)
                                       : __builtin_amdgcn_readlane(pt.sl[1], l - 64))
                             : 0;
        const gbl<float>* gcol = pt.gc + (int64_t)vl * pt.ldg;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int m = x.lane + 64 * h;
          if (m < sps) {
            float val = (l < s && m < s) ? gcol[pt.sj[h]] * pt.id[h] : 0.f;
            if (m == l) val = 1.f;
            pt.gs[l * sps + m] = val;
          }
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = x.lane + 64 * h;
        if (m < s) pt.sfeat[m] = pt.sj[h];
      }
      pt.s_t = s;
      pt.ng_ok = false;
      wave_lds_order();
    }
    pt.tau = row_norms_tau(x, pt, q, lambda, !pt.ng_ok);
    pt.ng_ok = true;
    pt.valid = true;
    return true;
  }

  // Loads the Gram entries of members m0..m0+7 (< hi) at the lane's four
  // features jv, with their steps d and offsets dp.
  static __device__ __forceinline__ void member_group(const Pat& pt, int m0, int hi,
                                                      const int (&jv)[4],
                                                      const float (&d)[2], const float (&dp)[2],
                                                      float (&g)[8][4], float (&dm)[8],
                                                      float (&pm)[8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int m = m0 + u;
      const int ml = m & 63;
      int sl;
      if (m < 64) {
        sl = __builtin_amdgcn_readlane(pt.sl[0], ml);
        dm[u] = readlane_f(d[0], ml);
        pm[u] = readlane_f(dp[0], ml);
      } else {
        sl = __builtin_amdgcn_readlane(pt.sl[1], ml);
        dm[u] = readlane_f(d[1], ml);
        pm[u] = readlane_f(dp[1], ml);
      }
      if (m >= hi) {
        sl = 0;
        dm[u] = pm[u] = 0.f;
      }
      const gbl<float>* gcol = pt.gc + (int64_t)sl * pt.ldg;
#pragma unroll
      for (int e = 0; e < 4; ++e) g[u][e] = m < hi ? gcol[jv[e]] : 0.f;
    }
  }

  // The exact zero-coordinate check of an epoch (steps d, previous offset dp
  // = beta_S - beta0, both FP32): for every position k, with accP = G_{k,S} dp
  // and accD = G_{k,S} d, the coordinate's correlation at its visit is
  // c_k - accP - (accD over members before k); the new anchor value is
  // c_k - accP - accD (written to c2).  Returns true when every zero
  // coordinate stays at zero; tau_new is the slack ratio at the new anchor.
  // Lane positions base + 4 lane + e; the members split into those before
  // the 256-position block, inside it and after it.
  static __device__ __forceinline__ bool pattern_exact(const Ctx& x, const Pat& pt, int q,
                                                       double lambda, const float (&d)[2],
                                                       const float (&dp)[2], double& tau_new) {
    const int s = __builtin_amdgcn_readfirstlane(pt.s);
    bool bad = false;
    double tau = INFINITY;
    for (int base = 0; base < q; base += 256) {
      const int k0 = base + 4 * x.lane;
      const int lo = __popcll(ballot(x.lane < s && pt.sp[0] < base)) +
                     __popcll(ballot(x.lane + 64 < s && pt.sp[1] < base));
      const int hi = __popcll(ballot(x.lane < s && pt.sp[0] < base + 256)) +
                     __popcll(ballot(x.lane + 64 < s && pt.sp[1] < base + 256));
      double cv[4];
      int mb[4], jv[4];
      ld4(x.c + k0, cv);
      ld4(pt.pmem + k0, mb);
#pragma unroll
      for (int e = 0; e < 4; ++e) jv[e] = act_at(x, k0 + e, q, false);
      float accP[4] = {0.f, 0.f, 0.f, 0.f}, accD[4] = {0.f, 0.f, 0.f, 0.f}, part[4];
      float g[8][4], dm[8], pm[8];
      // members before the block: every position sees their steps
      for (int m0 = 0; m0 < lo; m0 += 8) {
        member_group(pt, m0, lo, jv, d, dp, g, dm, pm);
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            accP[e] = fmaf(g[u][e], pm[u], accP[e]);
            accD[e] = fmaf(g[u][e], dm[u], accD[e]);
          }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) part[e] = accD[e];
      // members inside: position k sees the steps of those before it
      for (int m0 = lo; m0 < hi; m0 += 8) {
        member_group(pt, m0, hi, jv, d, dp, g, dm, pm);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int m = m0 + u;
          const int pos = m < 64 ? __builtin_amdgcn_readlane(pt.sp[0], m & 63)
                                 : __builtin_amdgcn_readlane(pt.sp[1], m & 63);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            accP[e] = fmaf(g[u][e], pm[u], accP[e]);
            accD[e] = fmaf(g[u][e], dm[u], accD[e]);
            const float w = (m < hi && pos < k0 + e) ? dm[u] : 0.f;
            part[e] = fmaf(g[u][e], w, part[e]);
          }
        }
      }
      // members after the block
      for (int m0 = hi; m0 < s; m0 += 8) {
        member_group(pt, m0, s, jv, d, dp, g, dm, pm);
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            accP[e] = fmaf(g[u][e], pm[u], accP[e]);
            accD[e] = fmaf(g[u][e], dm[u], accD[e]);
          }
      }
      typedef double d2v __attribute__((ext_vector_type(2)));
      double cn[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        cn[e] = cv[e] - ((double)accP[e] + (double)accD[e]);
        if (k0 + e < q && !mb[e]) {
          const double vis = cv[e] - (double)accP[e] - (double)part[e];
          if (fabs(vis) > lambda) bad = true;
        }
      }
      // positions >= q of the block hold values nobody reads
      *reinterpret_cast<gbl<d2v>*>(pt.c2 + k0) = d2v{cn[0], cn[1]};
      *reinterpret_cast<gbl<d2v>*>(pt.c2 + k0 + 2) = d2v{cn[2], cn[3]};
      float nv[4];
      ld4(pt.ng + k0, nv);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (k0 + e < q && !mb[e]) tau = fmin(tau, slack_ratio(cn[e], nv[e], lambda));
    }
    __threadfence_block();
    tau_new = wave_min(tau);
    return ballot(bad) == 0;
  }

  // Zero coordinates of A for which |c0_k| + ng_k R <= lambda fails (R the
  // reach of the steps since the anchor); the first 64 positions go to cand.
  // Returns their number.
  static __device__ __forceinline__ int bound_filter(const Ctx& x, const Pat& pt, int q,
                                                     double lambda, double R) {
    const uint64_t lt = (x.lane == 0) ? 0ull : (~0ull >> (64 - x.lane));
    int n = 0;
    for (int base = 0; base < q; base += 256) {
      const int k0 = base + 4 * x.lane;
      double cv[4];
      int mb[4];
      float nv[4];
      ld4(x.c + k0, cv);
      ld4(pt.pmem + k0, mb);
      ld4(pt.ng + k0, nv);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool f = k0 + e < q && !mb[e] && !(slack_ratio(cv[e], nv[e], lambda) > R);
        const uint64_t m = ballot(f);
        const int idx = n + __popcll(m & lt);
        if (f && idx < 64) pt.cand[idx] = k0 + e;
        n += __popcll(m);
      }
    }
    wave_lds_order();
    return __builtin_amdgcn_readfirstlane(n);
  }

  // The exact correlation at its visit of each of the n (<= 64) coordinates
  // in cand, one per lane: c0_k - sum_m G_km (dp_m + [member m before k] d_m).
  // Returns true when all of them stay at zero.
  static __device__ __forceinline__ bool cand_check(const Ctx& x, const Pat& pt, int q, int n,
                                                   double lambda, const float (&d)[2],
                                                   const float (&dp)[2]) {
    const int s = __builtin_amdgcn_readfirstlane(pt.s);
    const bool mine = x.lane < n;
    const int k = mine ? pt.cand[x.lane] : 0;
    const int j = act_at(x, k, q, false);
    const double c0 = x.c[k];
    float acc = 0.f;
    for (int m0 = 0; m0 < s; m0 += 8) {
      float g[8], w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int m = m0 + u;
        const int ml = m & 63;
        int sl, pos;
        float dm, pm;
        if (m < 64) {
          sl = __builtin_amdgcn_readlane(pt.sl[0], ml);
          pos = __builtin_amdgcn_readlane(pt.sp[0], ml);
          dm = readlane_f(d[0], ml);
          pm = readlane_f(dp[0], ml);
        } else {
          sl = __builtin_amdgcn_readlane(pt.sl[1], ml);
          pos = __builtin_amdgcn_readlane(pt.sp[1], ml);
          dm = readlane_f(d[1], ml);
          pm = readlane_f(dp[1], ml);
        }
        const bool mv = m < s;
        const gbl<float>* gcol = pt.gc + (int64_t)(mv ? sl : 0) * pt.ldg;
        g[u] = mv ? gcol[j] : 0.f;
        w[u] = mv ? pm + (pos < k ? dm : 0.f) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = fmaf(g[u], w[u], acc);
    }
    const bool bad = mine && fabs(c0 - (double)acc) > lambda;
    return ballot(bad) == 0;
  }

  // Forward substitution on the scaled block: delta_l = u_l, u -= delta_l
  // col_l, for l < s8 (a multiple of 8; the columns beyond s are zero).
  // Group G holds the steps 8G..8G+7 with compile-time lanes; its columns
  // were loaded by the previous group, which also loads the next ones.
  template <int SPS, int G>
  static __device__ __forceinline__ void subst_group(const Ctx& x, const Pat& pt, int s8,
                                                     float (&u)[2], float (&d)[2],
                                                     const float (&t0)[8], const float (&t1)[8]) {
    if constexpr (G * 8 < (SPS == 64 ? 64 : 128)) {
      if (G * 8 < s8) {
        float n0[8], n1[8];
        const float* nb = pt.gs + x.lane + ((G + 1) * 8 < s8 ? (G + 1) * 8 : G * 8) * SPS;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          n0[v] = nb[v * SPS];
          n1[v] = SPS == 128 ? nb[v * SPS + 64] : 0.f;
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          constexpr int H = G * 8 >= 64 ? 1 : 0;
          const float dl = readlane_f(u[H], (G * 8 + v) & 63);
          switch (v) {  // compile-time lane of the step
            case 0: d[H] = writelane_f<(G * 8 + 0) & 63>(d[H], dl); break;
            case 1: d[H] = writelane_f<(G * 8 + 1) & 63>(d[H], dl); break;
            case 2: d[H] = writelane_f<(G * 8 + 2) & 63>(d[H], dl); break;
            case 3: d[H] = writelane_f<(G * 8 + 3) & 63>(d[H], dl); break;
            case 4: d[H] = writelane_f<(G * 8 + 4) & 63>(d[H], dl); break;
            case 5: d[H] = writelane_f<(G * 8 + 5) & 63>(d[H], dl); break;
            case 6: d[H] = writelane_f<(G * 8 + 6) & 63>(d[H], dl); break;
            default: d[H] = writelane_f<(G * 8 + 7) & 63>(d[H], dl); break;
          }
          u[0] = fmaf(-t0[v], dl, u[0]);
          if (SPS == 128) u[1] = fmaf(-t1[v], dl, u[1]);
        }
        subst_group<SPS, G + 1>(x, pt, s8, u, d, n0, n1);
      }
    }
  }

  template <int SPS>
  static __device__ __forceinline__ void substitute(const Ctx& x, const Pat& pt, int s8,
                                                    float (&u)[2], float (&d)[2]) {
    float t0[8], t1[8];
    const float* b0 = pt.gs + x.lane;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      t0[v] = b0[v * SPS];
      t1[v] = SPS == 128 ? b0[v * SPS + 64] : 0.f;
    }
    subst_group<SPS, 0>(x, pt, s8, u, d, t0, t1);
  }

  // One cyclic CD epoch over A by the pattern mode.  Returns 0 when the
  // premise fails (nothing written), 1 when committed, 2 when committed and
  // no coefficient moved (the state is a fixed point of the epoch).
  static __device__ __forceinline__ int pattern_epoch(Ctx& x, Pat& pt, int q, double lambda,
                                                      int (&stc)[kNumStats]) {
    const int s = __builtin_amdgcn_readfirstlane(pt.s);
    const int s8 = (s + 7) & ~7;
    float u[2] = {pt.u[0], pt.u[1]};
    float d[2] = {0.f, 0.f};
    if (s8 > 0) {
      if (pt.gsp == 64)
        substitute<64>(x, pt, s8, u, d);
      else
        substitute<128>(x, pt, s8, u, d);
    }
    double bn[2];
    float dp[2];
    bool bad = false, moved = false;
    double sD = 0.0, sd = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int m = x.lane + 64 * h;
      const bool v = m < s;
      if (!v) d[h] = 0.f;
      bn[h] = pt.sb[h] + (double)d[h];
      const double dprev = pt.sb[h] - pt.b0[h];
      dp[h] = (float)dprev;
      if (v) {
        if (!(pt.sg[h] > 0.0 ? bn[h] > 0.0 : bn[h] < 0.0)) bad = true;
        if (d[h] != 0.f) moved = true;
        sD = fma(dprev, dprev, sD);
        sd = fma((double)d[h], (double)d[h], sd);
      }
    }
    if (ballot(bad)) return 0;
    const double reach = (sqrt(wave_sum(sD)) + sqrt(wave_sum(sd))) * (1.0 + 1e-6);
    bool reanchor = false;
    double tau_new = 0.0;
    if (!(reach < pt.tau)) {
      const int nc = bound_filter(x, pt, q, lambda, reach);
      if (nc <= 64) {
        ++stc[kStatNear];
        if (nc > 0 && !cand_check(x, pt, q, nc, lambda, d, dp)) return 0;
      } else {
        ++stc[kStatExact];
        if (!pattern_exact(x, pt, q, lambda, d, dp, tau_new)) return 0;
        reanchor = true;
      }
    }
    // commit
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int m = x.lane + 64 * h;
      if (m < s && d[h] != 0.f) {
        pt.sb[h] = bn[h];
        x.beta[pt.sj[h]] = bn[h];
      }
      pt.u[h] = u[h];
    }
    if (reanchor) {
      gbl<double>* t = x.c;
      x.c = pt.c2;
      pt.c2 = t;
      pt.b0[0] = pt.sb[0];
      pt.b0[1] = pt.sb[1];
      pt.tau = tau_new;
    }
    __threadfence_block();
    return ballot(moved) ? 1 : 2;
  }
};

// LDS bytes the narrow kernel needs before its two dynamic regions (the
// support's Gram block, PathOpts::gs_cap floats, then the residual mode's
// staging region, PathOpts::lds_cap floats); they start 16-byte aligned at
// this offset.
template <typename XT, int VEC, int S, int NG, bool GATHER>
constexpr size_t narrow_lds_bytes() {
  using N = Narrow<XT, VEC, S, NG, GATHER>;
  return (2 * sizeof(double) * N::NMAX + sizeof(XT) * 64 * N::RPL + sizeof(int) * N::NMAX +
          4 * sizeof(int) * N::NSC + 2 * sizeof(int) * N::NBLD +
          sizeof(float) * N::NBLD * N::NMAX + 15) &
         ~(size_t)15;
}

template <typename N, typename XT, size_t GOFF>
__device__ __forceinline__ void bind_lds(typename N::Ctx& x, typename N::Pat& pt,
                                         unsigned char* smem, const PathOpts& opts) {
  x.y_l = reinterpret_cast<double*>(smem);
  x.rho_l = x.y_l + N::NMAX;
  x.tile = reinterpret_cast<XT*>(x.rho_l + N::NMAX);
  x.rows_l = reinterpret_cast<int*>(x.tile + 64 * N::RPL);
  pt.owner = x.rows_l + N::NMAX;
  pt.spos = pt.owner + N::NSC;
  pt.sfeat = pt.spos + N::NSC;
  pt.cand = pt.sfeat + N::NSC;
  pt.bslot = pt.cand + N::NSC;
  pt.bfeat = pt.bslot + N::NBLD;
  pt.stage = reinterpret_cast<float*>(pt.bfeat + N::NBLD);
  pt.gs = reinterpret_cast<float*>(smem + GOFF);
  pt.gs_cap = opts.gs_cap;
  // 16-byte aligned (gs_cap is a multiple of 64): the region holds doubles
  x.stg = pt.gs + opts.gs_cap;
  x.stg_cap = opts.lds_cap;
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
    gbl<double>* lam_g = gptr(d.lam);
    gbl<double>* bout_g = gptr(d.beta_out);

    typename N::Ctx x;
    typename N::Pat pt;
    x.X = gptr((const XT*)d.X);
    x.ldx = d.ldx;
    x.n = d.n;
    x.p = d.p;
    x.lane = lane;
    x.slot = lane / S;
    x.seg = lane % S;
    bind_lds<N, XT, narrow_lds_bytes<XT, VEC, S, NG, GATHER>()>(x, pt, smem, opts);
    x.nrm2 = gptr(d.nrm2);
    x.xty = gptr(d.xty);
    x.inv = gptr(d.inv);
    x.beta = gptr(d.beta);
    x.c = gptr(d.c);
    x.act = gptr(d.act);
    pt.gc = gptr(d.gc);
    pt.ng = gptr(d.ng);
    pt.pslot = gptr(d.pslot);
    pt.pmem = gptr(d.pmem);
    pt.c2 = gptr(d.c2);
    pt.ldg = d.ldg;
    pt.ns = d.ns;
    pt.s = 0;
    pt.gsp = 64;
    pt.s_t = -1;
    pt.victim = 0;
    pt.valid = false;
    pt.ng_ok = false;
    pt.tau = 0.0;
    int stc[kNumStats];
#pragma unroll
    for (int i = 0; i < kNumStats; ++i) stc[i] = 0;
    N::setup(x, gptr(d.rows));
    const int n = d.n, p = d.p, T = d.T;
    const gbl<XT>* Y = gptr((const XT*)d.y);
    // ---- y into LDS; precompute ||x_j||^2 and lambda_max = ||X^T y||_inf
    double yy = 0.0;
    for (int i = lane; i < n; i += 64) {
      double v = (double)Y[N::src_row(x, i)];
      x.y_l[i] = v;
      yy = fma(v, v, yy);
    }
    wave_lds_order();
    const double ynorm2 = wave_sum(yy);
    bool bad = !isfinite(ynorm2);
    double lmax_l = 0.0;
    {
      double yr[N::RPL];
      N::load_rows(x, x.y_l, yr);
      for (int base = 0; base < p; base += N::U * N::C) {
        typename N::Stage st[N::U];
#pragma unroll
        for (int u = 0; u < N::U; ++u) {
          const int j = base + u * N::C + x.slot;
          st[u].v = j < p;
          st[u].j = j < p ? j : p - 1;
          N::L::load_raw(N::col(x, st[u].j), n, x.seg, x.ridx, st[u].x);
        }
#pragma unroll
        for (int u = 0; u < N::U; ++u) {
          double s2 = 0.0, sy = 0.0;
#pragma unroll
          for (int i = 0; i < N::RPL; ++i) {
            const double xi = N::L::at(st[u].x, x.mk, i);
            s2 = fma(xi, xi, s2);
            sy = fma(xi, yr[i], sy);
          }
          s2 = seg_sum<S>(s2);
          sy = seg_sum<S>(sy);
          if (st[u].v && x.seg == 0) {
            x.nrm2[st[u].j] = s2;
            x.xty[st[u].j] = sy;
            x.inv[st[u].j] = s2 > 0.0 ? 1.0 / s2 : 0.0;
            lmax_l = fmax(lmax_l, fabs(sy));
            if (!isfinite(s2) || !isfinite(sy)) bad = true;
          }
        }
      }
    }
    const double lmax = wave_max(lmax_l);
    bad = ballot(bad) != 0;

    // ---- the lambda grid (Sec. 3.3) and the warm start beta^{lambda_0}
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
      for (int j = lane; j < p; j += 64) x.beta[j] = (bi && !bad) ? bi[j] : 0.0;
    }
    __threadfence_block();

    if (bad) {
      for (int t = 0; t < T; ++t) {
        for (int j = lane; j < p; j += 64) bout_g[(int64_t)t * p + j] = 0.0;
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
      const bool pat_on = opts.pattern != 0;
      for (int t = 0; t < T; ++t) {
        const double lambda = lam_g[t];
        int q = p;
        bool full = true;
        int k = 0, status = 1;
        double G = 0.0;
        if (pat_on) N::pattern_new_lambda(x, pt);
        bool c_ok = false, rho_ok = false;
        int rejects = 0;
        for (;;) {
          if (k % f == 0 || k == K) {
            double R2, Ry, M, l1, sbx, xmax;
            int nnz = N::refresh(x, q, full, R2, Ry);
            N::sweep(x, q, full, M, l1, sbx, xmax);
            ++stc[kStatPasses];
            GapInfo g = gap_safe(R2, Ry, l1, sbx, xmax, M, nnz, n, lambda, ynorm, q,
                                 opts.rule == 1);
            G = g.gap;
            if (G <= eps) {
              status = 0;
              break;
            }
            if (k == K) break;
            bool dropped;
            q = N::test_compact(x, g, q, full, dropped, nullptr, pat_on ? pt.ng : nullptr);
            full = false;
            rho_ok = true;
            c_ok = true;
            if (dropped) {
              N::refresh(x, q, full, R2, Ry);
              c_ok = false;
            }
            pt.valid = false;
            rejects = 0;
          }
          // epochs up to the next screening pass (or the budget): the pattern
          // mode while it holds; a rejected epoch runs in residual mode, and
          // after two rejections the interval stays there
          int ne = min(f - k % f, K - k);
          while (ne > 0) {
            if (pat_on && rejects < 2 && q > 0) {
              if (!pt.valid) {
                if (!c_ok) {
                  double M, l1, sbx, xmax;
                  N::sweep(x, q, full, M, l1, sbx, xmax);
                  c_ok = true;
                }
                if (!N::pattern_setup(x, pt, q, full, lambda, stc)) {
                  rejects = 2;
                  continue;
                }
              }
              const int r = N::pattern_epoch(x, pt, q, lambda, stc);
              if (r) {
                ++stc[kStatPatternEpochs];
                ++k;
                --ne;
                rho_ok = false;
                if (r == 2) {
                  stc[kStatSkipped] += ne;
                  k += ne;
                  ne = 0;
                }
                continue;
              }
              ++stc[kStatRejected];
              ++rejects;
              pt.valid = false;
            }
            if (!rho_ok) {
              double R2, Ry;
              N::refresh(x, q, full, R2, Ry);
              rho_ok = true;
            }
            const int nr = (pat_on && rejects < 2) ? 1 : ne;
            N::cd_epochs(x, q, full, lambda, nr, 0);
            stc[kStatResidualEpochs] += nr;
            k += nr;
            ne -= nr;
            c_ok = false;
            pt.valid = false;
          }
        }
        // beta^{lambda_t} and its certificate
        gbl<double>* bo = bout_g + (int64_t)t * p;
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
    if (opts.stats && lane == 0) {
#pragma unroll
      for (int i = 0; i < kNumStats; ++i)
        if (stc[i])
          atomicAdd(reinterpret_cast<unsigned long long*>(&opts.stats[i]), (unsigned long long)stc[i]);
    }
    if (opts.timestamps && lane == 0) {
      opts.timestamps[2 * d.orig] = t_start;
      opts.timestamps[2 * d.orig + 1] = wall_clock64();
    }
    __syncthreads();
  }
}

}  // namespace gs
