// The per-problem ("narrow") schedule: one wavefront runs Algorithm 1 for one
// Lasso path, with the residual in LDS (canonical copy) and in registers
// (working copy in the column layout), and X streamed from L2/HBM.
//
// Column layout: lane = slot * S + seg.  Each of the C = 64/S slots works on
// its own column; the S lanes of a slot split that column's rows.  A column
// dot product is a per-lane FMA chain followed by a butterfly over S lanes.
//
// The epochs between two screening passes run in one of two modes; both are
// cyclic CD over the active set A in ascending order and make the same
// updates in exact arithmetic:
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
//  * Gram mode, for active sets of at most QG coordinates whose nonzeros fit
//    the LDS column cache: the correlations g = X_A^T rho (exact at the start
//    of the interval, from the sweep) are held in registers, 8 positions per
//    lane, and a change delta at coordinate j becomes g -= delta X_A^T x_j: a
//    q/64-wide update with a cached Gram column from LDS instead of a
//    dependent n-long reduction.  A column is computed the first time its
//    coordinate changes at the current lambda and follows the compactions of
//    A.  The cached columns are FP32; their error on g is proportional to the
//    steps and vanishes at the fixed point, and every screening pass
//    recomputes g from a fresh residual.
//
// Lanes of one wavefront order their LDS accesses without block barriers, so
// pending global loads are never drained inside the loops.
#pragma once

#include <type_traits>

#include "gs_device.hpp"

namespace gs {

template <typename XT, int VEC, int S, int NG, bool GATHER>
struct Narrow {
  using L = ColLayout<XT, VEC, S, NG, GATHER>;
  static constexpr int RPL = L::RPL;
  static constexpr int C = L::C;
  static constexpr int NMAX = L::NMAX;
  static constexpr int NT = (NMAX + 63) / 64;        // rows per lane, row-major layout
  static constexpr int NB = NT <= 2 ? 8 : (NT <= 4 ? 4 : (NT <= 8 ? 2 : 1));  // refresh batch
  static constexpr int U = RPL <= 8 ? 4 : (RPL <= 24 ? 3 : (RPL <= 32 ? 2 : 1));  // sweep batch
  static constexpr int TQ = 8;        // active positions per lane in Gram mode
  static constexpr int QG = 64 * TQ;  // largest active set run in Gram mode
  static constexpr int NSMAX = 256;   // Gram cache slots

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
    gbl<double>* nrm2;
    gbl<double>* inv;           // 1/||x_j||^2 (0 for a zero column)
    gbl<double>* beta;
    gbl<double>* c;
    gbl<int32_t>* act;
  };

  // LDS state shared by the two modes.  The region `G` holds either the Gram
  // cache (Gram mode) or the active positions' beta and 1/||x||^2 (residual
  // mode, when 16 q bytes fit).  Scalars are wavefront-uniform.
  struct Gram {
    int* slot;    // QG: cache slot of position k, or -1 (between intervals)
    int* np;      // QG: position of k after the last compaction, or -1
    int* owner;   // NSMAX: position whose column a slot holds, or -1
    XT* xj;       // NMAX: staging of the column being correlated
    float* G;     // cap floats: slot s holds x_{A[k]}^T x_{A[owner[s]]} at G[s*q + k]
    int cap;      // floats available in G
    int ns;       // slots in use for the current q
    int victim;   // round-robin eviction cursor
    bool on;      // the cache describes the current active set
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
    for (int base = 0; base < q; base += U * C) {
      Stage st[U];
      double nr[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = base + u * C + x.slot;
        fetch_j<false>(x, k, act_at(x, k, q, full), q, nullptr, nullptr, st[u]);
        nr[u] = x.nrm2[st[u].j];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double d = dotx(st[u].x, r);
        if (st[u].v && x.seg == 0) {
          x.c[base + u * C + x.slot] = d;
          Ml = fmax(Ml, fabs(d));
          const double xn = sqrt(nr[u]);
          l1l += fabs(st[u].b);
          sbl += fabs(st[u].b) * xn;
          xml = fmax(xml, xn);
        }
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
  // the new position of every old one (-1 when dropped) is recorded.
  static __device__ __forceinline__ int test_compact(const Ctx& x, const GapInfo& g, int q, bool full,
                                     bool& dropped_nz, int* np = nullptr) {
    int q2 = 0;
    bool dn = false;
    const uint64_t lt = (x.lane == 0) ? 0ull : (~0ull >> (64 - x.lane));
    for (int base = 0; base < q; base += 256) {
      int jv[4];
      double cv[4], nv[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = base + 64 * u + x.lane;
        jv[u] = act_at(x, k, q, full);
        cv[u] = x.c[k < q ? k : q - 1];
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
        const bool keep = v && sphere_keep(g, cv[u], nv[u], x.n);
        if (v && !keep && bv[u] != 0.0) {
          x.beta[jv[u]] = 0.0;
          dn = true;
        }
        const uint64_t m = ballot(keep);
        const int pos = q2 + __popcll(m & lt);
        if (keep) {
          x.act[pos] = jv[u];
          x.c[pos] = cv[u];  // c of kept coordinates moves with them
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
    XT* mytile = x.tile + x.lane * RPL;
    double xd[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      xd[i] = (double)s.x[i];
      mytile[i] = ((x.mk >> i) & 1ull) ? s.x[i] : XT(0);
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
      const XT* tx = x.tile + (cs * S + x.seg) * RPL;
#pragma unroll
      for (int i = 0; i < RPL; ++i) r[i] = fma(-delta, (double)tx[i], r[i]);
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

  // One step of the 3-deep load ring: chunk at `base` sits in st[CUR]; the
  // loads of chunk base+2C go into st[(CUR+2)%3] with the index fetched one
  // step earlier, and the index of chunk base+3C is requested.
  template <int CUR, bool POSL>
  static __device__ __forceinline__ void ring_step(const Ctx& x, int base, int q, bool full,
                                                   double lambda, double* pb,
                                                   const double* pinv, Stage (&st)[3],
                                                   int (&ix)[3], double (&r)[RPL]) {
    constexpr int NXT = (CUR + 2) % 3;
    fetch_j<POSL>(x, base + 2 * C + x.slot, ix[NXT], q, pb, pinv, st[NXT]);
    ix[CUR] = act_at(x, base + 3 * C + x.slot, q, full);
    resolve<POSL>(x, st[CUR], lambda, pb, r);
  }

  // One cyclic CD epoch over A (Algorithm 1):
  //   beta_j <- ST(lambda/||x_j||^2, beta_j + x_j^T rho / ||x_j||^2),
  //   rho    <- rho - (beta_j' - beta_j) x_j.
  // The epoch may start at position k0 > 0 (the rest of an epoch begun in
  // Gram mode): positions before k0 are left alone.
  template <bool POSL>
  static __device__ __forceinline__ void cd_epoch(const Ctx& x, int q, bool full, double lambda, double* pb,
                                  const double* pinv, double (&r)[RPL], int k0) {
    if (q <= k0) return;
    const int b0 = k0 - k0 % C;
    Stage st[3];
    int ix[3];
    ix[0] = act_at(x, b0 + x.slot, q, full);
    ix[1] = act_at(x, b0 + C + x.slot, q, full);
    ix[2] = act_at(x, b0 + 2 * C + x.slot, q, full);
    fetch_j<POSL>(x, b0 + x.slot, ix[0], q, pb, pinv, st[0]);
    st[0].v = st[0].v && b0 + x.slot >= k0;
    fetch_j<POSL>(x, b0 + C + x.slot, ix[1], q, pb, pinv, st[1]);
    for (int base = b0;; base += 3 * C) {
      ring_step<0, POSL>(x, base, q, full, lambda, pb, pinv, st, ix, r);
      if (base + C >= q) break;
      ring_step<1, POSL>(x, base + C, q, full, lambda, pb, pinv, st, ix, r);
      if (base + 2 * C >= q) break;
      ring_step<2, POSL>(x, base + 2 * C, q, full, lambda, pb, pinv, st, ix, r);
      if (base + 3 * C >= q) break;
    }
  }

  // ne residual-mode epochs (the first one from position k0), the residual
  // taken from and returned to LDS.  With room for 16 q bytes in the cache
  // region, beta and 1/||x||^2 of the active positions are staged in LDS
  // for the interval (the region's Gram cache is then given up).
  static __device__ __forceinline__ void cd_epochs(const Ctx& x, Gram& gm, int q, bool full, double lambda,
                                   int ne, int k0) {
    double r[RPL];
    load_rows(x, x.rho_l, r);
    const bool posl = q > 0 && (size_t)q * 2 * sizeof(double) <= (size_t)gm.cap * sizeof(float);
    if (posl) {
      gm.on = false;
      double* pb = reinterpret_cast<double*>(gm.G);
      double* pinv = pb + q;
      for (int k = x.lane; k < q; k += 64) {
        const int j = full ? k : x.act[k];
        pb[k] = x.beta[j];
        pinv[k] = x.inv[j];
      }
      wave_lds_order();
      for (int e = 0; e < ne; ++e) cd_epoch<true>(x, q, full, lambda, pb, pinv, r, e == 0 ? k0 : 0);
      for (int k = x.lane; k < q; k += 64) x.beta[full ? k : x.act[k]] = pb[k];
    } else {
      for (int e = 0; e < ne; ++e)
        cd_epoch<false>(x, q, full, lambda, nullptr, nullptr, r, e == 0 ? k0 : 0);
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

  // ---- Gram mode -------------------------------------------------------------

  // Starts the cache for the active set of size q (when it is off).
  static __device__ __forceinline__ void gram_begin(const Ctx& x, Gram& gm, int q) {
    if (!gm.on) {
      for (int k = x.lane; k < q; k += 64) gm.slot[k] = -1;
      for (int s = x.lane; s < NSMAX; s += 64) gm.owner[s] = -1;
      gm.victim = 0;
      gm.on = true;
    }
    gm.ns = min(NSMAX, gm.cap / max(q, 1));
    wave_lds_order();
  }

  // After the active set shrank from q_old to q_new (new positions in gm.np):
  // move every cached column to stride q_new and drop the slots whose
  // coordinate left.  In place: in ascending order every destination address
  // is at most its source address, so no source is overwritten before read.
  static __device__ __forceinline__ void gram_compact(const Ctx& x, Gram& gm, int q_old, int q_new) {
    if (q_new == q_old) return;  // nothing dropped: positions unchanged
    for (int s = 0; s < gm.ns; ++s) {
      const int own = gm.owner[s];
      if (own < 0) continue;
      const int nown = gm.np[own];
      wave_lds_order();
      if (x.lane == 0) gm.owner[s] = nown;
      if (nown < 0) continue;
      for (int k0 = 0; k0 < q_old; k0 += 256) {
        float v[4];
        int dd[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + 64 * u + x.lane;
          v[u] = k < q_old ? gm.G[s * q_old + k] : 0.f;
          dd[u] = k < q_old ? gm.np[k] : -1;
        }
        wave_lds_order();
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (dd[u] >= 0) gm.G[s * q_new + dd[u]] = v[u];
        wave_lds_order();
      }
    }
    for (int k0 = 0; k0 < q_old; k0 += 64) {
      const int k = k0 + x.lane;
      const int sl = k < q_old ? gm.slot[k] : -1;
      const int d = k < q_old ? gm.np[k] : -1;
      wave_lds_order();
      if (d >= 0) gm.slot[d] = sl;
      wave_lds_order();
    }
  }

  // Computes the Gram column of position pos (x_{A[k]}^T x_{A[pos]} for all
  // k < q) into a slot; returns the slot and, in `evicted`, the position
  // whose column the slot held before (-1 if none).
  static __device__ __forceinline__ int gram_build(const Ctx& x, Gram& gm, int pos, int q,
                                                  bool full,
                                   int& evicted) {
    const int j = __builtin_amdgcn_readfirstlane(full ? pos : x.act[pos]);
    const gbl<XT>* cj = col(x, j);
    for (int i = x.lane; i < x.n; i += 64) gm.xj[i] = cj[src_row(x, i)];
    const int s = gm.victim;
    gm.victim = (gm.victim + 1 < gm.ns) ? gm.victim + 1 : 0;
    evicted = __builtin_amdgcn_readfirstlane(gm.owner[s]);
    wave_lds_order();
    if (x.lane == 0) gm.owner[s] = pos;
    float* Gc = gm.G + s * q;
    for (int k = x.lane; k < q; k += 64) {
      const gbl<XT>* ck = col(x, full ? k : x.act[k]);
      double a0 = 0.0, a1 = 0.0;
      if constexpr (GATHER || VEC == 1) {
        for (int i = 0; i < x.n; ++i) a0 = fma((double)ck[src_row(x, i)], (double)gm.xj[i], a0);
      } else {
        for (int i = 0; i < x.n; i += VEC) {
          XT t[VEC];
          VecLoad<XT, VEC>::go(ck + i, t);
#pragma unroll
          for (int e = 0; e < VEC; e += 2) {
            a0 = fma((double)t[e], (double)gm.xj[i + e], a0);
            if (e + 1 < VEC) a1 = fma((double)t[e + 1], (double)gm.xj[i + e + 1], a1);
          }
        }
      }
      Gc[k] = (float)(a0 + a1);
    }
    wave_lds_order();
    return s;
  }

  // Register state of the Gram mode: positions (t << 6) + lane, t < TQ.
  struct GramRegs {
    double gr[TQ], br[TQ], ir[TQ];
    int sr[TQ];
  };

  // The in-order scan of row T (positions 64T .. 64T+63); compile-time T keeps
  // every register array statically indexed.
  template <int T>
  static __device__ __forceinline__ void gram_row(const Ctx& x, Gram& gm, GramRegs& R, int q,
                                                  int nt, bool full, double lambda, int budget,
                                                  int& builds, int& kstart) {
    const double thr = lambda * R.ir[T];
    int start = 0;
    for (;;) {
      bool chg = false;
      double bn = R.br[T];
      if (R.ir[T] > 0.0 && x.lane >= start) {
        bn = soft_thr(thr, R.br[T] + R.gr[T] * R.ir[T]);
        chg = (bn != R.br[T]);
      }
      const uint64_t mk = ballot(chg);
      if (!mk) break;
      const int l0 = __builtin_ctzll(mk);
      const double delta = readlane_d(bn - R.br[T], l0);
      if (x.lane == l0) R.br[T] = bn;
      const int pos = (T << 6) + l0;
      int s = __builtin_amdgcn_readlane(R.sr[T], l0);
      if (s < 0) {
        int ev;
        s = gram_build(x, gm, pos, q, full, ev);
        ++builds;
        if (ev >= 0) {
#pragma unroll
          for (int t3 = 0; t3 < TQ; ++t3)
            if (t3 == (ev >> 6) && x.lane == (ev & 63)) R.sr[t3] = -1;
        }
        if (x.lane == l0) R.sr[T] = s;
      }
      const float* Gc = gm.G + s * q;
      float gv[TQ];
#pragma unroll
      for (int t2 = 0; t2 < TQ; ++t2) {
        const int kk = (t2 << 6) + x.lane;
        gv[t2] = (t2 < nt) ? Gc[kk < q ? kk : q - 1] : 0.f;
      }
#pragma unroll
      for (int t2 = 0; t2 < TQ; ++t2) R.gr[t2] = fma(-delta, (double)gv[t2], R.gr[t2]);
      if (builds > budget) kstart = pos + 1;
      start = l0 + 1;
      if (start >= 64 || kstart >= 0) break;
    }
  }

  template <int T>
  static __device__ __forceinline__ void gram_rows(const Ctx& x, Gram& gm, GramRegs& R, int q,
                                                   int nt, bool full, double lambda, int budget,
                                                   int& builds, int& kstart) {
    if constexpr (T < TQ) {
      if (T < nt && kstart < 0) {
        gram_row<T>(x, gm, R, q, nt, full, lambda, budget, builds, kstart);
        gram_rows<T + 1>(x, gm, R, q, nt, full, lambda, budget, builds, kstart);
      }
    }
  }

  // Up to ne cyclic CD epochs over A in Gram mode (g at entry in c); beta is
  // written back at the end.  Returns the number of complete epochs.  Once
  // more than `budget` columns were built in this call (the cache thrashes)
  // it stops right after the coordinate being updated and sets kstart to the
  // next position of the unfinished epoch (kstart = -1 otherwise); the caller
  // finishes the interval in residual mode from there, so the cyclic order is
  // unchanged.
  static __device__ __forceinline__ int gram_epochs(const Ctx& x, Gram& gm, int q, bool full, double lambda,
                                    int ne, int budget, int& kstart) {
    const int nt = (q + 63) >> 6;
    GramRegs R;
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
      const int k = (t << 6) + x.lane;
      const bool v = k < q;
      const int kk = v ? k : q - 1;
      const int j = full ? kk : x.act[kk];
      R.gr[t] = v ? x.c[kk] : 0.0;
      R.br[t] = v ? x.beta[j] : 0.0;
      R.ir[t] = v ? x.inv[j] : 0.0;
      R.sr[t] = v ? gm.slot[kk] : -1;
    }
    int builds = 0, e = 0;
    kstart = -1;
    for (; e < ne && kstart < 0; ++e)
      gram_rows<0>(x, gm, R, q, nt, full, lambda, budget, builds, kstart);
    if (kstart >= 0) --e;  // the last epoch is unfinished
#pragma unroll
    for (int t = 0; t < TQ; ++t) {
      const int k = (t << 6) + x.lane;
      if (k < q) {
        x.beta[full ? k : x.act[k]] = R.br[t];
        gm.slot[k] = R.sr[t];
      }
    }
    __threadfence_block();
    wave_lds_order();
    return e;
  }
};

// LDS bytes the narrow kernel needs before the Gram cache region (whose
// size in floats is a launch argument, PathOpts::gram_cap); the region
// starts 16-byte aligned at this offset.
template <typename XT, int VEC, int S, int NG, bool GATHER>
constexpr size_t narrow_lds_bytes() {
  using N = Narrow<XT, VEC, S, NG, GATHER>;
  return (2 * sizeof(double) * N::NMAX + sizeof(XT) * 64 * N::RPL + sizeof(int) * N::NMAX +
          sizeof(XT) * N::NMAX + 2 * sizeof(int) * N::QG + sizeof(int) * N::NSMAX + 15) &
         ~(size_t)15;
}

template <typename N, typename XT, size_t GOFF>
__device__ __forceinline__ void bind_lds(typename N::Ctx& x, typename N::Gram& gm,
                                         unsigned char* smem, int gram_cap) {
  x.y_l = reinterpret_cast<double*>(smem);
  x.rho_l = x.y_l + N::NMAX;
  x.tile = reinterpret_cast<XT*>(x.rho_l + N::NMAX);
  gm.xj = x.tile + 64 * N::RPL;
  x.rows_l = reinterpret_cast<int*>(gm.xj + N::NMAX);
  gm.slot = x.rows_l + N::NMAX;
  gm.np = gm.slot + N::QG;
  gm.owner = gm.np + N::QG;
  // 16-byte aligned: the region also holds doubles in residual mode
  gm.G = reinterpret_cast<float*>(smem + GOFF);
  gm.cap = gram_cap;
  gm.ns = 0;
  gm.victim = 0;
  gm.on = false;
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
    typename N::Gram gm;
    x.X = gptr((const XT*)d.X);
    x.ldx = d.ldx;
    x.n = d.n;
    x.p = d.p;
    x.lane = lane;
    x.slot = lane / S;
    x.seg = lane % S;
    bind_lds<N, XT, narrow_lds_bytes<XT, VEC, S, NG, GATHER>()>(x, gm, smem, opts.gram_cap);
    x.nrm2 = gptr(d.nrm2);
    x.inv = gptr(d.inv);
    x.beta = gptr(d.beta);
    x.c = gptr(d.c);
    x.act = gptr(d.act);
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
        lam = lam_g[t] * (d.lambda_relative ? lmax : 1.0);
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
      for (int t = 0; t < T; ++t) {
        const double lambda = lam_g[t];
        int q = p;
        bool full = true;
        int k = 0, status = 1;
        double G = 0.0;
        bool use_gram = false;
        gm.on = false;  // a new lambda resets the active set and the cache
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
            const int q_old = q;
            q = N::test_compact(x, g, q, full, dropped, gm.on ? gm.np : nullptr);
            full = false;
            if (gm.on) N::gram_compact(x, gm, q_old, q);
            // Gram mode when the cache holds the current nonzeros with room for
            // newcomers (nnz of this pass bounds the coordinates that keep moving)
            const int slots = q > 0 ? min(N::NSMAX, opts.gram_cap / q) : 0;
            use_gram = q > 0 && q <= N::QG && slots >= 8 && slots >= nnz + max(8, nnz / 4);
            if (dropped) {
              N::refresh(x, q, full, R2, Ry);
              if (use_gram) N::sweep(x, q, full, M, l1, sbx, xmax);  // g at the new rho
            }
            if (use_gram) N::gram_begin(x, gm, q);
          }
          // epochs up to the next screening pass (or the budget)
          int ne = min(f - k % f, K - k);
          int k0 = 0;
          if (use_gram) {
            int kstart;
            const int done = N::gram_epochs(x, gm, q, full, lambda, ne, gm.ns, kstart);
            k += done;
            ne -= done;
            if (kstart >= 0) {  // the cache thrashed: residual mode until the next pass
              double R2, Ry;
              N::refresh(x, q, full, R2, Ry);
              use_gram = false;
              gm.on = false;
              k0 = kstart;
            }
          }
          if (ne > 0) N::cd_epochs(x, gm, q, full, lambda, ne, k0);
          k += ne;
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
    if (opts.timestamps && lane == 0) {
      opts.timestamps[2 * d.orig] = t_start;
      opts.timestamps[2 * d.orig + 1] = wall_clock64();
    }
    __syncthreads();
  }
}

// The CD part of the wide schedule: one wavefront runs min(f, K - k) epochs
// over the active set the wide kernels left in the workspace (residual mode).
template <typename XT, int VEC, int S, int NG, bool GATHER>
__global__ __launch_bounds__(64) void k_wide_cd(ProbDesc d, WideState* st, PathOpts opts) {
  using N = Narrow<XT, VEC, S, NG, GATHER>;
  extern __shared__ __align__(16) unsigned char smem[];
  if (st->done || st->phase != 2) return;
  const int lane = threadIdx.x;
  typename N::Ctx x;
  typename N::Gram gm;
  x.X = gptr((const XT*)d.X);
  x.ldx = d.ldx;
  x.n = d.n;
  x.p = d.p;
  x.lane = lane;
  x.slot = lane / S;
  x.seg = lane % S;
  bind_lds<N, XT, narrow_lds_bytes<XT, VEC, S, NG, GATHER>()>(x, gm, smem, opts.gram_cap);
  x.nrm2 = gptr(d.nrm2);
  x.inv = gptr(d.inv);
  x.beta = gptr(d.beta);
  x.c = gptr(d.c);
  x.act = gptr(d.act) + (int64_t)st->cur * d.p;
  N::setup(x, gptr(d.rows));
  for (int i = lane; i < d.n; i += 64) x.rho_l[i] = gptr(d.rho)[i];
  wave_lds_order();
  const int q = st->q;
  const bool full = st->full != 0;
  const int k0 = st->k;
  const int ne = min(opts.f, opts.K - k0);
  const double lambda = gptr(d.lam)[st->t];
  N::cd_epochs(x, gm, q, full, lambda, ne, 0);
  if (lane == 0) {
    st->k = k0 + ne;
    st->phase = 0;
  }
}

}  // namespace gs
