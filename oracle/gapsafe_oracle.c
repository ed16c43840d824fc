/*
 * gapsafe_oracle.c -- plain, slow CPU FP64 reference for cyclic coordinate
 * descent on the Lasso with dynamic GAP SAFE sphere screening
 * (Fercoq, Gramfort, Salmon, "Mind the duality gap: safer rules for the
 * Lasso", ICML 2015).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness oracle for the HIP
 * library.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header or constant with the
 * GPU path and never calls it.
 *
 * Everything is FP64, single-threaded, written as the paper states it:
 * no blocking, no fusion, no reordering beyond what the formulas say.
 * X is dense, column-major, n x p with leading dimension ldx >= n.
 *
 * Readings of points the paper leaves open (each is also listed in the
 * design notes of the repository):
 *   R1  stop threshold eps = eps_rel * ||y||^2 (the paper's eps is absolute).
 *   R2  a screening pass runs before CD epoch k whenever k mod f == 0
 *       (0-based k); Algorithm 1 writes this as "k mod f = 1" for 1-based k.
 *   R3  the gap is tested on the (beta, theta) of the pass, before any
 *       screened coefficient is zeroed; a certified beta is output unchanged.
 *   R4  epochs = number of CD passes completed before the stop.
 *   R5  a coordinate that is screened out while nonzero is set to zero and the
 *       residual is updated (Sec. 2.3, Remark on convergence: zeroing screened
 *       coefficients can only bring beta closer to the solution).
 *   R6  ||X^T rho||_inf is taken over the current active set only (Sec. 4.1);
 *       the gap is then the gap of the Lasso restricted to A, whose dual
 *       optimum equals the full one.
 *   R7  the active set only shrinks inside one lambda and is reset to [p] when
 *       lambda changes; only beta is carried over (Algorithm 1 warm start).
 *   R8  rho = 0 gives alpha = 0; max|c| = 0 with rho != 0 gives the unclipped
 *       alpha; a zero column is skipped by CD and always screened.
 *   R9  ties: keep j when mu >= 1 (eq. of the safe active set); ST(u,x) = 0
 *       when |x| == u.
 *   R10 radius r = sqrt(2 max(G,0)) / lambda (Proposition 1, GAP SAFE sphere).
 *   R11 the kept set used by the oracle's own path is inflated by a stated
 *       rounding bound (unit roundoff u = 2^-53); the exact-formula kept set is
 *       also reported for set comparisons.
 *   R12 a grid of T values includes lambda_max as lambda_0 (Sec. 3.3).
 *   R13 after K epochs without certification one last gap is evaluated for the
 *       returned beta and status is set to "not converged".
 *   R14 coordinates are visited in ascending index order (cyclic CD).
 *   R15 GAP SAFE dome (Sec. 3.2, appendix "Dome test"): the normal is
 *       w = (y/lambda - theta) / R_hat and the ratio alpha_d =
 *       2 (r_check[beta] / R_hat)^2 - 1 with r_check taken at the primal
 *       point beta (the main text's normal has the opposite sign and the
 *       appendix writes r_check[theta]; with those the dome would not contain
 *       the dual optimum).  A coordinate is kept when either test keeps it
 *       (the dome lies inside the sphere, so with exact arithmetic the dome
 *       alone decides).
 *   R16 the comparison rules of Table 1 are sphere tests (Sec. 2.1) with:
 *       static SAFE: center y/lambda, radius ||y|| |1/lambda - 1/lambda_max|
 *       (Sec. 2.1 first example); Dynamic Safe: center y/lambda, radius
 *       R_hat[theta_k] = ||theta_k - y/lambda|| (Sec. 2.3 example); Dynamic
 *       ST3: the ball B(y/lambda, R_hat) cut by the half-space
 *       s* x*^T theta <= 1 (x* = x_{j*}, j* the first index of the largest
 *       |x_j^T y|, s* the sign of x*^T y), held in the ball around the
 *       projection of y/lambda on that plane: center y/lambda - delta s* x*
 *       with delta = (lambda_max/lambda - 1)/||x*||^2 (Table 1) and radius
 *       (R_hat^2 - d^2)^(1/2) with d = (lambda_max/lambda - 1)/||x*||, the
 *       distance to the plane (the remark after Proposition 1 writes this
 *       d as delta; the two coincide for unit-norm columns).  For lambda >=
 *       lambda_max ST3 falls back to the Dynamic Safe ball.  These rules
 *       replace the GAP SAFE test; the gap still decides the stop.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-4)

/* ---------------------------------------------------------------- helpers */

static const double ORC_U = 1.1102230246251565e-16; /* 2^-53 */

/* Higham's gamma_m = m u / (1 - m u): bound on the relative error of a
 * length-m dot product or sum evaluated in floating point. */
static double gamma_m(double m) { return m * ORC_U / (1.0 - m * ORC_U); }

static double col_dot(int n, const double* xj, const double* v) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += xj[i] * v[i];
  return s;
}

/* ST(u, x) = sign(x) (|x| - u)_+  (Algorithm 1, soft-threshold). */
static double soft_threshold(double u, double x) {
  if (x > u) return x - u;
  if (x < -u) return x + u;
  return 0.0;
}

/* ------------------------------------------------------------- precompute */

/* lambda_max = ||X^T y||_inf (Sec. 1.2: for lambda >= lambda_max, 0 is a
 * solution), plus the column squared norms ||x_j||^2 used by CD. */
int orc_precompute(int n, int p, int64_t ldx, const double* X, const double* y,
                   double* nrm2, double* xty, double* lambda_max,
                   double* ynorm2) {
  if (n <= 0 || p <= 0 || ldx < n) return ORC_EINVAL;
  double lmax = 0.0;
  for (int j = 0; j < p; ++j) {
    const double* xj = X + (int64_t)j * ldx;
    nrm2[j] = col_dot(n, xj, xj);
    xty[j] = col_dot(n, xj, y);
    if (fabs(xty[j]) > lmax) lmax = fabs(xty[j]);
  }
  *lambda_max = lmax;
  *ynorm2 = col_dot(n, y, y);
  return ORC_OK;
}

/* The usual grid lambda_t = lambda_0 10^(-delta t / (T-1)), t = 0..T-1,
 * lambda_0 = lambda_max (Sec. 3.3). */
void orc_grid(double lambda_max, int T, double delta, double* out) {
  for (int t = 0; t < T; ++t)
    out[t] = (T == 1) ? lambda_max
                      : lambda_max * pow(10.0, -delta * (double)t / (double)(T - 1));
}

/* ------------------------------------------------------- objective / gap */

/* Plain definitions: P(beta) = 1/2 ||X beta - y||^2 + lambda ||beta||_1
 * (Sec. 1.1, the Lasso) and D(theta) = 1/2 ||y||^2 - lambda^2/2
 * ||theta - y/lambda||^2 (Sec. 1.1, the dual).  Returns P - D; writes P, D. */
double orc_gap(int n, int p, int64_t ldx, const double* X, const double* y,
               const double* beta, const double* theta, double lambda,
               double* P_out, double* D_out) {
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  if (!r) return NAN;
  for (int i = 0; i < n; ++i) r[i] = -y[i];
  for (int j = 0; j < p; ++j)
    if (beta[j] != 0.0) {
      const double* xj = X + (int64_t)j * ldx;
      for (int i = 0; i < n; ++i) r[i] += xj[i] * beta[j];
    }
  double l1 = 0.0;
  for (int j = 0; j < p; ++j) l1 += fabs(beta[j]);
  double P = 0.5 * col_dot(n, r, r) + lambda * l1;
  double yy = col_dot(n, y, y), d2 = 0.0;
  for (int i = 0; i < n; ++i) {
    double t = theta[i] - y[i] / lambda;
    d2 += t * t;
  }
  double D = 0.5 * yy - 0.5 * lambda * lambda * d2;
  free(r);
  if (P_out) *P_out = P;
  if (D_out) *D_out = D;
  return P - D;
}

/* ------------------------------------------------------- one screen pass */

typedef struct {
  double gap;        /* G_lambda(beta, theta) on the active set (R6)        */
  double alpha;      /* theta = alpha * rho                                 */
  double radius;     /* sqrt(2 max(G,0)) / lambda                           */
  double radius_inf; /* radius inflated by the rounding bound (R11)         */
  double M;          /* max_{j in A} |x_j^T rho|                            */
  double rho_norm2;  /* ||rho||^2                                           */
  double y_rho;      /* y^T rho                                             */
  double l1;         /* ||beta||_1                                          */
  double alpha_s;    /* alpha of the rounding-safe dual point (R11)         */
  double err_gap;    /* the rounding bound added to the gap (R11)           */
} orc_pass_info;

/* Residual rho = y - X beta, recomputed from scratch (Sec. 2.3). */
static void residual(int n, int p, int64_t ldx, const double* X, const double* y,
                     const double* beta, double* rho) {
  for (int i = 0; i < n; ++i) rho[i] = y[i];
  for (int j = 0; j < p; ++j)
    if (beta[j] != 0.0) {
      const double* xj = X + (int64_t)j * ldx;
      for (int i = 0; i < n; ++i) rho[i] -= beta[j] * xj[i];
    }
}

/* Support function of the dome D(c, r, a, w) = B(c, r) n {t: w^T (t - c) <= -a r}
 * (Sec. 3.2 dome tests; appendix "Dome test") at a vector x, given
 * cx = c^T x, wx = w^T x and xn = ||x||:  the ball's maximizer c + r x/||x||
 * lies in the half-space iff w^T x <= -a ||x||; otherwise the maximum is on
 * the circle where the plane cuts the sphere. */
static double dome_support(double cx, double wx, double xn, double r, double a) {
  if (wx <= -a * xn) return cx + r * xn;
  double s2 = (xn * xn - wx * wx) * (1.0 - a * a);
  return cx - r * a * wx + r * sqrt(s2 > 0.0 ? s2 : 0.0);
}

/* Dome parameters of one pass (R15), in terms of the pass scalars:
 *   R_hat^2   = ||alpha rho - y/lambda||^2 = alpha^2 R2 - 2 alpha Ry / lambda + yy / lambda^2
 *   r_check^2 = (yy - ||rho||^2 - 2 lambda l1)_+ / lambda^2       (Theorem 2)
 * center c = (y/lambda + theta)/2, radius R_hat/2, ratio 2 r_check^2/R_hat^2 - 1,
 * normal (y/lambda - theta)/R_hat.  For x_j:  c^T x_j = (x_j^T y/lambda +
 * alpha c_j)/2 and w^T x_j = (x_j^T y/lambda - alpha c_j)/R_hat, so the test
 * needs X^T y (computed once) and c_j: no further pass over X. */
double orc_dome_mu(double xty, double cj, double xn, double alpha, double lambda,
                   double Rh, double rc2);
static int dome_keep_exact(double xty, double cj, double xn, double alpha,
                           double lambda, double Rh, double rc2) {
  if (!(xn > 0.0)) return 0;
  if (!(Rh > 0.0)) return 1; /* theta = y/lambda: the dome is a point; no decision here */
  return orc_dome_mu(xty, cj, xn, alpha, lambda, Rh, rc2) >= 1.0;
}

/* mu_C(x_j) = max(sigma_C(x_j), sigma_C(-x_j)) of the GAP SAFE dome (exact
 * formula; exported for the tests). */
double orc_dome_mu(double xty, double cj, double xn, double alpha, double lambda,
                   double Rh, double rc2) {
  double r = 0.5 * Rh, a = 2.0 * rc2 / (Rh * Rh) - 1.0;
  double cx = 0.5 * (xty / lambda + alpha * cj);
  double wx = (xty / lambda - alpha * cj) / Rh;
  double mu_p = dome_support(cx, wx, xn, r, a);
  double mu_m = dome_support(-cx, -wx, xn, r, a);
  return mu_p > mu_m ? mu_p : mu_m;
}

/* The same test made safe for the rounding of its inputs (R11, R15): every
 * input is replaced by the bound that enlarges the dome (a larger ball, the
 * cutting plane moved outwards: r_check down, R_hat up), w^T x by a lower
 * bound (the support function does not increase with w^T x), c^T x by an
 * upper bound and ||x|| by an upper bound; a final margin covers the
 * evaluation itself.  e_cx, e_wn bound the errors of c^T x and of the
 * numerator x^T y/lambda - alpha c_j; Rlo, Rhi bracket R_hat; rc2lo is a
 * lower bound of r_check^2. */
static int dome_keep_safe(double xty, double cj, double xn_up, double alpha,
                          double lambda, double Rlo, double Rhi, double rc2lo,
                          double e_cx, double e_wn) {
  if (!(xn_up > 0.0)) return 0;
  if (!(Rhi > 0.0)) return 1;
  double r = 0.5 * Rhi;
  double a = 2.0 * rc2lo / (Rhi * Rhi) - 1.0;
  if (a < -1.0) a = -1.0;
  double cx = 0.5 * (xty / lambda + alpha * cj);
  double num = xty / lambda - alpha * cj;
  double mu = -INFINITY;
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    double cs = sgn * cx + e_cx;               /* upper bound of c^T (sgn x) */
    double ns = sgn * num - e_wn;              /* lower bound of the numerator */
    double wlo;                                /* lower bound of w^T (sgn x)  */
    if (ns >= 0.0) wlo = ns / Rhi;
    else wlo = (Rlo > 0.0) ? ns / Rlo : -INFINITY;
    double m = (wlo == -INFINITY) ? cs + r * xn_up : dome_support(cs, wlo, xn_up, r, a);
    if (m > mu) mu = m;
  }
  double scale = fabs(cx) + r * xn_up * 3.0 + 1.0;
  return mu >= 1.0 - 16.0 * ORC_U * scale;
}

/* Ingredients of the comparison rules (R16), computed once per problem. */
typedef struct {
  double lambda_max;   /* |x*^T y|                                         */
  double sstar;        /* sign of x*^T y                                   */
  double nstar;        /* ||x*||                                           */
  const double* g;     /* p: x_j^T x*                                      */
} orc_ref;

/* j* = first index of max |x_j^T y|; g_j = x_j^T x*. */
static void comparator_ingredients(int n, int p, int64_t ldx, const double* X,
                                   const double* xty, const double* nrm2, double* g,
                                   orc_ref* ref) {
  int js = 0;
  for (int j = 1; j < p; ++j)
    if (fabs(xty[j]) > fabs(xty[js])) js = j;
  const double* xs = X + (int64_t)js * ldx;
  for (int j = 0; j < p; ++j) g[j] = col_dot(n, X + (int64_t)j * ldx, xs);
  ref->lambda_max = fabs(xty[js]);
  ref->sstar = xty[js] >= 0.0 ? 1.0 : -1.0;
  ref->nstar = sqrt(nrm2[js]);
  ref->g = g;
}

/* One screening pass at (beta, lambda) over the active set A (q entries):
 *   c_j = x_j^T rho for j in A,  M = max |c_j|           (Sec. 4.1)
 *   alpha = min(max(y^T rho / (lambda ||rho||^2), -1/M), 1/M)   (Sec. 2.3)
 *   G = P(beta) - D(alpha rho)                           (Sec. 3.2)
 *   r = sqrt(2 G) / lambda                               (Proposition 1)
 *   keep j iff |x_j^T theta| + r ||x_j|| >= 1            (Sec. 2.1 sphere test)
 * keep_exact[k] / keep_safe[k] (k indexes A) receive the exact-formula test
 * and the rounding-inflated test (R11).  c_out (q) receives c_j.
 * rho (n) must hold y - X beta on entry (caller refreshes it). */
static void pass_on_residual(int n, int64_t ldx, const double* X, const double* y,
                             const double* beta, const double* nrm2,
                             const double* xty, int rule, const orc_ref* ref,
                             const int32_t* A, int q, int nnz, double lambda,
                             const double* rho, double* c_out,
                             uint8_t* keep_exact, uint8_t* keep_safe,
                             orc_pass_info* info) {
  double R2 = col_dot(n, rho, rho);
  double Ry = col_dot(n, y, rho);
  double M = 0.0, l1 = 0.0, xmax = 0.0, sum_bx = 0.0;
  for (int k = 0; k < q; ++k) {
    int j = A[k];
    const double* xj = X + (int64_t)j * ldx;
    c_out[k] = col_dot(n, xj, rho);
    if (fabs(c_out[k]) > M) M = fabs(c_out[k]);
    if (sqrt(nrm2[j]) > xmax) xmax = sqrt(nrm2[j]);
  }
  /* ||beta||_1 over A: coefficients outside A are zero (R5). */
  for (int k = 0; k < q; ++k) {
    int j = A[k];
    l1 += fabs(beta[j]);
    sum_bx += fabs(beta[j]) * sqrt(nrm2[j]);
  }

  /* Dual point, exact formula (R8). */
  double alpha;
  if (M > 0.0) {
    alpha = Ry / (lambda * R2);
    if (alpha < -1.0 / M) alpha = -1.0 / M;
    if (alpha > 1.0 / M) alpha = 1.0 / M;
  } else if (R2 > 0.0) {
    alpha = Ry / (lambda * R2);
  } else {
    alpha = 0.0;
  }

  /* Rounding bound (R11).  rho_tilde is the computed residual; e_c bounds
   * |c_hat_j - x_j^T rho_tilde| / ||x_j||.  M_plus makes alpha rho_tilde
   * exactly dual feasible on A. */
  double rnorm = sqrt(R2) * (1.0 + gamma_m(n + 2));
  double e_c = gamma_m(n + 1) * rnorm;
  double xmax_up = xmax * (1.0 + gamma_m(n + 2));
  double M_plus = (M + e_c * xmax_up) * (1.0 + 4.0 * ORC_U);
  double alpha_s;
  if (M_plus > 0.0) {
    alpha_s = (R2 > 0.0) ? Ry / (lambda * R2) : 0.0;
    if (alpha_s < -1.0 / M_plus) alpha_s = -1.0 / M_plus;
    if (alpha_s > 1.0 / M_plus) alpha_s = 1.0 / M_plus;
  } else {
    alpha_s = (R2 > 0.0) ? Ry / (lambda * R2) : 0.0; /* R8: no column bounds theta */
  }

  /* G = 1/2||rho||^2 + lambda||beta||_1 - (1/2||y||^2 - lambda^2/2
   * ||alpha rho - y/lambda||^2), expanded so that the 1/2||y||^2 terms cancel
   * analytically: G = 1/2 R2 + lambda l1 - lambda alpha Ry + 1/2 lambda^2
   * alpha^2 R2. */
  double G = 0.5 * R2 + lambda * l1 - lambda * alpha * Ry +
             0.5 * lambda * lambda * alpha * alpha * R2;
  double Gs = 0.5 * R2 + lambda * l1 - lambda * alpha_s * Ry +
              0.5 * lambda * lambda * alpha_s * alpha_s * R2;
  double yn = sqrt(col_dot(n, y, y)) * (1.0 + gamma_m(n + 2));
  double d_rho = gamma_m(nnz + 1) * (yn + sum_bx * (1.0 + gamma_m(n + 2)));
  /* The computed y^T rho carries an error of up to gamma_n ||y|| ||rho|| (a
   * dot product whose terms have both signs: its error is not relative to
   * its value); it enters G through lambda alpha y^T rho. */
  double errG = gamma_m(n + 6) * (0.5 * R2 + lambda * l1 +
                                  lambda * fabs(alpha_s * Ry) +
                                  0.5 * lambda * lambda * alpha_s * alpha_s * R2) +
                lambda * fabs(alpha_s) * gamma_m(n) * yn * rnorm +
                rnorm * d_rho + 0.5 * d_rho * d_rho;
  double Gp = (Gs > 0.0 ? Gs : 0.0) + errG;
  double radius = sqrt(2.0 * (G > 0.0 ? G : 0.0)) / lambda;
  double radius_s = sqrt(2.0 * Gp) / lambda * (1.0 + 4.0 * ORC_U);

  /* GAP SAFE dome (R15): exact parameters at (beta, alpha rho) and bounds
   * for the safe test at (beta, alpha_s rho). */
  double yy = col_dot(n, y, y);
  double Rh2 = alpha * alpha * R2 - 2.0 * alpha * Ry / lambda + yy / (lambda * lambda);
  double Rh = sqrt(Rh2 > 0.0 ? Rh2 : 0.0);
  double rc2 = (yy - R2 - 2.0 * lambda * l1) / (lambda * lambda);
  if (rc2 < 0.0) rc2 = 0.0;
  double Rs2 = alpha_s * alpha_s * R2 - 2.0 * alpha_s * Ry / lambda + yy / (lambda * lambda);
  double eR2 = gamma_m(n + 6) * (alpha_s * alpha_s * R2 + 2.0 * fabs(alpha_s * Ry) / lambda +
                                 yy / (lambda * lambda)) +
               2.0 * fabs(alpha_s) / lambda * gamma_m(n) * yn * rnorm;
  double Rhi = sqrt(Rs2 + eR2 > 0.0 ? Rs2 + eR2 : 0.0) * (1.0 + 4.0 * ORC_U);
  double Rlo = sqrt(Rs2 - eR2 > 0.0 ? Rs2 - eR2 : 0.0) * (1.0 - 4.0 * ORC_U);
  double rt = rnorm + d_rho; /* bounds ||y - X beta|| */
  double rc2lo = (yy * (1.0 - gamma_m(n + 2)) - rt * rt * (1.0 + 4.0 * ORC_U) -
                  2.0 * lambda * l1 * (1.0 + gamma_m(q + 2))) /
                 (lambda * lambda) * (1.0 - 4.0 * ORC_U);
  if (rc2lo < 0.0) rc2lo = 0.0;

  /* the comparison rules' spheres (R16): center term x_j^T c = xty_j/lambda
   * - shift * g_j, radius r; with the bounds of their rounding */
  double shift = 0.0, rad = 0.0, rad_s = 0.0, e_shift = 0.0;
  if (rule >= 2) {
    double lmx = ref->lambda_max;
    double e_lm = gamma_m(n + 1) * ref->nstar * yn;
    if (rule == 2) {
      rad = sqrt(yy) * fabs(1.0 / lambda - 1.0 / lmx);
      rad_s = yn * (fabs(1.0 / lambda - 1.0 / lmx) +
                    (lmx > e_lm ? e_lm / (lmx * (lmx - e_lm)) : INFINITY)) *
              (1.0 + 4.0 * ORC_U);
    } else if (rule == 3 || !(lambda < lmx)) {
      rad = Rh;
      rad_s = Rhi;
    } else {
      double ratio = lmx / lambda - 1.0;
      shift = ref->sstar * ratio / (ref->nstar * ref->nstar);
      double dd = ratio / ref->nstar;
      rad = sqrt(Rh * Rh - dd * dd > 0.0 ? Rh * Rh - dd * dd : 0.0);
      double dlo = ((lmx - e_lm) / lambda - 1.0) / (ref->nstar * (1.0 + gamma_m(n + 2)));
      if (dlo < 0.0) dlo = 0.0;
      double r2s = Rhi * Rhi * (1.0 + 4.0 * ORC_U) - dlo * dlo * (1.0 - 4.0 * ORC_U);
      rad_s = sqrt(r2s > 0.0 ? r2s : 0.0) * (1.0 + 4.0 * ORC_U);
      /* |error of the computed shift| times |g_j| <= ||x_j|| ||x*|| */
      e_shift = (e_lm / lambda / (ref->nstar * ref->nstar) + 8.0 * ORC_U * fabs(shift)) *
                ref->nstar;
    }
  }

  for (int k = 0; k < q; ++k) {
    int j = A[k];
    double xn = sqrt(nrm2[j]);
    double xn_up = xn * (1.0 + gamma_m(n + 2));
    if (rule >= 2) {
      double cx = xty[j] / lambda - shift * ref->g[j];
      keep_exact[k] = (nrm2[j] > 0.0 && fabs(cx) + rad * xn >= 1.0) ? 1 : 0;
      double e_cx = gamma_m(n + 1) * xn_up * yn / lambda + e_shift * xn_up +
                    fabs(shift) * gamma_m(n + 1) * xn_up * ref->nstar +
                    4.0 * ORC_U * (fabs(xty[j] / lambda) + fabs(shift * ref->g[j]));
      keep_safe[k] =
          (nrm2[j] > 0.0 && fabs(cx) + e_cx + rad_s * xn_up >= 1.0 - 4.0 * ORC_U) ? 1 : 0;
      continue;
    }
    double mu = fabs(alpha * c_out[k]) + radius * xn;
    keep_exact[k] = (nrm2[j] > 0.0 && mu >= 1.0) ? 1 : 0;
    double mu_s = fabs(alpha_s * c_out[k]) + fabs(alpha_s) * e_c * xn_up +
                  radius_s * xn_up;
    keep_safe[k] = (nrm2[j] > 0.0 && mu_s >= 1.0 - 4.0 * ORC_U) ? 1 : 0;
    if (rule == 1) {
      keep_exact[k] = keep_exact[k] && dome_keep_exact(xty[j], c_out[k], xn, alpha, lambda,
                                                        Rh, rc2);
      /* errors of x_j^T y / lambda and of alpha_s c_j */
      double e_y = gamma_m(n + 1) * xn_up * yn / lambda;
      double e_ac = fabs(alpha_s) * e_c * xn_up;
      double t1 = fabs(xty[j] / lambda), t2 = fabs(alpha_s * c_out[k]);
      double e_cx = 0.5 * (e_y + e_ac) + 4.0 * ORC_U * (t1 + t2);
      double e_wn = e_y + e_ac + 4.0 * ORC_U * (t1 + t2);
      keep_safe[k] = keep_safe[k] && dome_keep_safe(xty[j], c_out[k], xn_up, alpha_s, lambda,
                                                      Rlo, Rhi, rc2lo, e_cx, e_wn);
    }
  }
  info->gap = G;
  info->alpha = alpha;
  info->radius = radius;
  info->radius_inf = radius_s;
  info->M = M;
  info->rho_norm2 = R2;
  info->y_rho = Ry;
  info->l1 = l1;
  info->alpha_s = alpha_s;
  info->err_gap = errG;
}

/* Public single pass: the boundary's screen() call done plainly.
 * active_in may be NULL (all p).  Outputs (each sized q_in):
 *   c_out, keep_exact, keep_safe; plus scalars.  Returns q_in or <0. */
int orc_screen(int n, int p, int64_t ldx, const double* X, const double* y,
               const double* beta, double lambda, const int32_t* active_in,
               int q_in, int rule, double* c_out, uint8_t* keep_exact,
               uint8_t* keep_safe, double* scalars /* 10: see orc_pass_info */) {
  if (n <= 0 || p <= 0 || ldx < n || !(lambda > 0.0) || rule < 0 || rule > 4)
    return ORC_EINVAL;
  int q = active_in ? q_in : p;
  int32_t* A = (int32_t*)malloc(sizeof(int32_t) * (size_t)(q > 0 ? q : 1));
  double* rho = (double*)malloc(sizeof(double) * (size_t)n);
  double* nrm2 = (double*)malloc(sizeof(double) * (size_t)p);
  double* xty = (double*)malloc(sizeof(double) * (size_t)p);
  if (!A || !rho || !nrm2 || !xty) {
    free(A); free(rho); free(nrm2); free(xty);
    return ORC_ENOMEM;
  }
  for (int k = 0; k < q; ++k) A[k] = active_in ? active_in[k] : k;
  for (int j = 0; j < p; ++j) {
    const double* xj = X + (int64_t)j * ldx;
    nrm2[j] = col_dot(n, xj, xj);
    xty[j] = col_dot(n, xj, y);
  }
  double* g = (double*)malloc(sizeof(double) * (size_t)p);
  if (!g) {
    free(A); free(rho); free(nrm2); free(xty);
    return ORC_ENOMEM;
  }
  orc_ref ref;
  comparator_ingredients(n, p, ldx, X, xty, nrm2, g, &ref);
  int nnz = 0;
  for (int j = 0; j < p; ++j) nnz += beta[j] != 0.0;
  residual(n, p, ldx, X, y, beta, rho);
  orc_pass_info info;
  pass_on_residual(n, ldx, X, y, beta, nrm2, xty, rule, &ref, A, q, nnz, lambda, rho, c_out,
                   keep_exact, keep_safe, &info);
  scalars[0] = info.gap;
  scalars[1] = info.alpha;
  scalars[2] = info.radius;
  scalars[3] = info.radius_inf;
  scalars[4] = info.M;
  scalars[5] = info.rho_norm2;
  scalars[6] = info.y_rho;
  scalars[7] = info.l1;
  scalars[8] = info.alpha_s;
  scalars[9] = info.err_gap;
  free(A); free(rho); free(nrm2); free(xty); free(g);
  return q;
}

/* ------------------------------------------------------------ the path */

/* Algorithm 1 (Sec. 4.1): coordinate descent with GAP SAFE sphere screening
 * over a non-increasing lambda grid with warm starts.
 *
 * lambdas: T values, used as given (lambda_relative == 0) or as multiples of
 *   lambda_max (lambda_relative != 0); NULL gives the Sec. 3.3 grid with
 *   parameter delta (R12).
 * beta_init: optional start for the first lambda (NULL = 0, the solution at
 *   lambda_max).
 * Outputs: beta_out (p x T column-major), gap_out, epochs_out, nactive_out,
 *   status_out, passes_out (each T).  screened (optional, p x T bytes): 1 when
 *   j was screened out at some pass for lambda_t.  lambdas_out (optional, T).
 * Returns 0, ORC_NOT_CONVERGED if some lambda hit K epochs, or < 0. */
int orc_lasso_path(int n, int p, int64_t ldx, const double* X, const double* y,
                   int T, const double* lambdas, int lambda_relative,
                   double delta, double eps_rel, int f, int K, int rule,
                   const double* beta_init, double* beta_out, double* gap_out,
                   int32_t* epochs_out, int32_t* nactive_out,
                   int32_t* status_out, int32_t* passes_out, uint8_t* screened,
                   double* lambdas_out) {
  if (n <= 0 || p <= 0 || ldx < n || T <= 0 || f < 1 || K < 0 ||
      !(eps_rel > 0.0) || rule < 0 || rule > 4)
    return ORC_EINVAL;
  double *nrm2 = malloc(sizeof(double) * p), *xty = malloc(sizeof(double) * p);
  double *rho = malloc(sizeof(double) * n), *beta = malloc(sizeof(double) * p);
  double *c = malloc(sizeof(double) * p), *lam = malloc(sizeof(double) * T);
  int32_t* A = malloc(sizeof(int32_t) * p);
  uint8_t *ke = malloc(p), *ks = malloc(p);
  if (!nrm2 || !xty || !rho || !beta || !c || !lam || !A || !ke || !ks) {
    free(nrm2); free(xty); free(rho); free(beta); free(c); free(lam);
    free(A); free(ke); free(ks);
    return ORC_ENOMEM;
  }
  double lambda_max, ynorm2;
  orc_precompute(n, p, ldx, X, y, nrm2, xty, &lambda_max, &ynorm2);
  double* gst = malloc(sizeof(double) * p);
  if (!gst) {
    free(nrm2); free(xty); free(rho); free(beta); free(c); free(lam);
    free(A); free(ke); free(ks);
    return ORC_ENOMEM;
  }
  orc_ref ref;
  comparator_ingredients(n, p, ldx, X, xty, nrm2, gst, &ref);
  if (lambdas == NULL) {
    orc_grid(lambda_max, T, delta, lam);
  } else {
    for (int t = 0; t < T; ++t)
      lam[t] = lambda_relative ? lambdas[t] * lambda_max : lambdas[t];
  }
  int bad = 0;
  for (int t = 0; t < T; ++t) {
    if (!(lam[t] > 0.0) || !isfinite(lam[t])) bad = 1;
    if (t > 0 && lam[t] > lam[t - 1]) bad = 1;
  }
  if (bad) {
    free(nrm2); free(xty); free(rho); free(beta); free(c); free(lam);
    free(A); free(ke); free(ks); free(gst);
    return ORC_EINVAL;
  }
  if (lambdas_out) memcpy(lambdas_out, lam, sizeof(double) * T);
  const double eps = eps_rel * ynorm2; /* R1 */
  for (int j = 0; j < p; ++j) beta[j] = beta_init ? beta_init[j] : 0.0;
  if (screened) memset(screened, 0, (size_t)p * (size_t)T);
  int any_nc = 0;

  for (int t = 0; t < T; ++t) {
    const double lambda = lam[t];
    /* beta <- beta^{lambda_{t-1}} is implicit: beta is carried over. */
    int q = p;
    for (int j = 0; j < p; ++j) A[j] = j; /* R7 */
    int k = 0, passes = 0, status = ORC_NOT_CONVERGED;
    double G = INFINITY;
    for (;;) {
      if (k % f == 0 || k == K) { /* R2, R13 */
        int nnz = 0;
        for (int j = 0; j < p; ++j) nnz += beta[j] != 0.0;
        residual(n, p, ldx, X, y, beta, rho);
        orc_pass_info info;
        pass_on_residual(n, ldx, X, y, beta, nrm2, xty, rule, &ref, A, q, nnz, lambda, rho, c,
                         ke, ks, &info);
        ++passes;
        G = info.gap;
        if (G <= eps) { /* R3 */
          status = ORC_OK;
          break;
        }
        if (k == K) break; /* R13: budget exhausted, G certified for beta */
        /* Sphere test: drop j with mu < 1 (inflated, R11); zero dropped
         * nonzeros and update the residual (R5); compact A keeping order. */
        int q2 = 0;
        for (int kk = 0; kk < q; ++kk) {
          int j = A[kk];
          if (ks[kk]) {
            A[q2++] = j;
          } else {
            if (screened) screened[(size_t)t * p + j] = 1;
            if (beta[j] != 0.0) {
              const double* xj = X + (int64_t)j * ldx;
              for (int i = 0; i < n; ++i) rho[i] += beta[j] * xj[i];
              beta[j] = 0.0;
            }
          }
        }
        q = q2;
      }
      /* One CD epoch over A in ascending order (R14):
       * beta_j <- ST(lambda/||x_j||^2, beta_j - x_j^T(X beta - y)/||x_j||^2). */
      for (int kk = 0; kk < q; ++kk) {
        int j = A[kk];
        if (nrm2[j] == 0.0) continue; /* R8 */
        const double* xj = X + (int64_t)j * ldx;
        double z = beta[j] + col_dot(n, xj, rho) / nrm2[j];
        double b = soft_threshold(lambda / nrm2[j], z);
        if (b != beta[j]) {
          double d = b - beta[j];
          for (int i = 0; i < n; ++i) rho[i] -= d * xj[i];
          beta[j] = b;
        }
      }
      ++k;
    }
    if (status != ORC_OK) any_nc = 1;
    memcpy(beta_out + (size_t)t * p, beta, sizeof(double) * p);
    gap_out[t] = G;
    epochs_out[t] = k;
    nactive_out[t] = q;
    status_out[t] = status;
    if (passes_out) passes_out[t] = passes;
  }
  free(nrm2); free(xty); free(rho); free(beta); free(c); free(lam);
  free(A); free(ke); free(ks); free(gst);
  return any_nc ? ORC_NOT_CONVERGED : ORC_OK;
}
