/*
 * hot_oracle.c -- FP64 CPU oracle for HOT (arXiv 2408.00598).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke() check and
 * the benchmark's CPU-baseline leg, never by the product path.  It shares no
 * code with the GPU library.  Everything here is plain, sequential FP64 code
 * written for readability, not speed.
 *
 * Pins (what checks this file against something other than itself) live in
 * tests/test_oracle_*.py: a Kronecker-product construction of A from the
 * paper's definitions, a dense solve of A A^T y = R, a dense simplex cross-
 * checked against an independent LP solver, 1-D CDF closed forms, the
 * translation and separable closed forms, Prop. 1 on LP-exact flows, the
 * relative KKT residual (eq. kkt_res) and feasibility error recomputed with
 * numpy, and the restart rule replayed from the per-check trace.  Iteration
 * counts against the paper's tables are parity unpinned: its sigma and
 * restart rules are not printed.
 */
#include "hot_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Index helpers for the paper's vectorisation (Sec. 2.1, def:A1A2A3). */
/* ------------------------------------------------------------------ */

/* f1_{i,k,j}: flow from bin (i,j) to bin (k,j) */
/* Built with -fopenmp (the multi-core timing build), the loops marked here
 * run their independent iterations on several threads: each marked loop
 * writes disjoint outputs and computes every output with the same sequential
 * code as the serial build, so both builds give bit-identical results.  The
 * reductions (norms, inner products) stay sequential. */
#ifdef _OPENMP
#define OR_PARALLEL_FOR _Pragma("omp parallel for schedule(static)")
#else
#define OR_PARALLEL_FOR
#endif

static int64_t ix1(int32_t m, int32_t n, int32_t i, int32_t k, int32_t j) {
  (void)n;
  return ((int64_t)j * m + k) * m + i;
}
/* f2_{k,j,l}: flow from bin (k,j) to bin (k,l) */
static int64_t ix2(int32_t m, int32_t n, int32_t k, int32_t j, int32_t l) {
  return (int64_t)m * m * n + ((int64_t)l * n + j) * m + k;
}

void or_dims(int32_t m, int32_t n, int64_t *N, int64_t *M3) {
  *N = (int64_t)m * m * n + (int64_t)m * n * n;
  *M3 = 3 * (int64_t)m * n - 1;
}

/* Cost vector c = [c1; c2] (Sec. 2.1 item 3, eq. def:c with p = 2) for a
 * grid whose row i sits at u_i and column j at v_j:
 * c1_{i,k,j} = (u_k - u_i)^2, c2_{k,j,l} = (v_j - v_l)^2.  The squared
 * Euclidean distance between bins (i,j) and (k,l) splits into these two
 * terms for any such (possibly non-uniform) grid, which is what the
 * color-transfer application's K-means grid lines use (Sec. 4.2).
 * u == NULL means u_i = i, v == NULL means v_j = j (the uniform grid). */
void or_cost_xy(int32_t m, int32_t n, const double *u, const double *v, double *c) {
  for (int32_t j = 0; j < n; ++j)
    for (int32_t k = 0; k < m; ++k)
      for (int32_t i = 0; i < m; ++i) {
        const double d = u ? u[k] - u[i] : (double)k - (double)i;
        c[ix1(m, n, i, k, j)] = d * d;
      }
  for (int32_t k = 0; k < m; ++k)
    for (int32_t j = 0; j < n; ++j)
      for (int32_t l = 0; l < n; ++l) {
        const double d = v ? v[j] - v[l] : (double)j - (double)l;
        c[ix2(m, n, k, j, l)] = d * d;
      }
}

void or_cost(int32_t m, int32_t n, double *c) { or_cost_xy(m, n, NULL, NULL, c); }

/* b = [0_M; mu1; Ibar_M mu2] (eq. Mat:A&b), histograms ordered with the
 * row index fastest, as the Kronecker forms of A3 and A4 imply. */
void or_bvec(int32_t m, int32_t n, const double *mu1, const double *mu2,
             double *b) {
  const int64_t M = (int64_t)m * n;
  for (int64_t r = 0; r < M; ++r) b[r] = 0.0;
  for (int32_t j = 0; j < n; ++j)
    for (int32_t i = 0; i < m; ++i) b[M + (int64_t)j * m + i] = mu1[(int64_t)i * n + j];
  for (int32_t l = 0; l < n; ++l)
    for (int32_t k = 0; k < m; ++k) {
      if (l == n - 1 && k == m - 1) continue; /* row removed by Ibar */
      b[2 * M + (int64_t)l * m + k] = mu2[(int64_t)k * n + l];
    }
}

/* A x: the three constraint families of the reduced model (eq.
 * partite-graph), in the row order of eq. Mat:A&b. */
void or_A(int32_t m, int32_t n, const double *x, double *out) {
  const int64_t M = (int64_t)m * n;
  /* rows A1/A2: sum_i f1_{i,k,j} - sum_l f2_{k,j,l} for bin (k,j) */
  OR_PARALLEL_FOR
  for (int32_t j = 0; j < n; ++j)
    for (int32_t k = 0; k < m; ++k) {
      double acc = 0.0;
      for (int32_t i = 0; i < m; ++i) acc += x[ix1(m, n, i, k, j)];
      for (int32_t l = 0; l < n; ++l) acc -= x[ix2(m, n, k, j, l)];
      out[(int64_t)j * m + k] = acc;
    }
  /* rows A3: sum_k f1_{i,k,j} for bin (i,j) */
  OR_PARALLEL_FOR
  for (int32_t j = 0; j < n; ++j)
    for (int32_t i = 0; i < m; ++i) {
      double acc = 0.0;
      for (int32_t k = 0; k < m; ++k) acc += x[ix1(m, n, i, k, j)];
      out[M + (int64_t)j * m + i] = acc;
    }
  /* rows A4: sum_j f2_{k,j,l} for bin (k,l), last row dropped */
  OR_PARALLEL_FOR
  for (int32_t l = 0; l < n; ++l)
    for (int32_t k = 0; k < m; ++k) {
      if (l == n - 1 && k == m - 1) continue;
      double acc = 0.0;
      for (int32_t j = 0; j < n; ++j) acc += x[ix2(m, n, k, j, l)];
      out[2 * M + (int64_t)l * m + k] = acc;
    }
}

/* A^T y: every flow variable appears in exactly two rows of A. */
void or_AT(int32_t m, int32_t n, const double *y, double *out) {
  const int64_t M = (int64_t)m * n;
  OR_PARALLEL_FOR
  for (int32_t j = 0; j < n; ++j)
    for (int32_t k = 0; k < m; ++k)
      for (int32_t i = 0; i < m; ++i)
        out[ix1(m, n, i, k, j)] = y[(int64_t)j * m + k] + y[M + (int64_t)j * m + i];
  OR_PARALLEL_FOR
  for (int32_t k = 0; k < m; ++k)
    for (int32_t j = 0; j < n; ++j)
      for (int32_t l = 0; l < n; ++l) {
        double y3 = (l == n - 1 && k == m - 1) ? 0.0 : y[2 * M + (int64_t)l * m + k];
        out[ix2(m, n, k, j, l)] = -y[(int64_t)j * m + k] + y3;
      }
}

/* Solve A A^T y = R with the explicit formula of Prop. 3 (prop:linsol_OT),
 * in the paper's W-hat form:
 *   yhat1^j = (Rt1^j + Rt2^j + Rt3) / (m+n),
 *   ya      = (I + 11^T/n) What sum_j yhat1^j,
 *   y1^j = yhat1^j - ya,  y2^j = (R2^j - 1^T y1^j)/m,
 *   y3^l = (R3^l + sum_j y1^j)/n  (last block truncated by Ibar).
 * The block index of the sum over j inside y3 is a bound variable (the
 * statement reuses the letter j for it). */
void or_solve_aat(int32_t m, int32_t n, const double *R, double *y) {
  const int64_t M = (int64_t)m * n;
  const double dm = (double)m, dn = (double)n;
  const double *R1 = R, *R2 = R + M, *R3 = R + 2 * M;
  double *y1 = y, *y2 = y + M, *y3 = y + 2 * M;

  double *PR3 = (double *)calloc((size_t)m, sizeof(double));
  double *Y = (double *)calloc((size_t)m, sizeof(double));
  double *WY = (double *)calloc((size_t)m, sizeof(double));
  double *d = (double *)calloc((size_t)m, sizeof(double));
  double *t = (double *)calloc((size_t)m, sizeof(double));
  double *yh = (double *)calloc((size_t)M, sizeof(double));

  /* sum_{l<n} R3^l + Ibar^T R3^n, and 1^T R3 */
  double tot3 = 0.0;
  for (int32_t l = 0; l < n; ++l)
    for (int32_t k = 0; k < m; ++k) {
      if (l == n - 1 && k == m - 1) continue;
      PR3[k] += R3[(int64_t)l * m + k];
      tot3 += R3[(int64_t)l * m + k];
    }
  /* yhat1^j */
  for (int32_t j = 0; j < n; ++j) {
    double s1 = 0.0, s2 = 0.0;
    for (int32_t k = 0; k < m; ++k) s1 += R1[(int64_t)j * m + k];
    for (int32_t i = 0; i < m; ++i) s2 += R2[(int64_t)j * m + i];
    for (int32_t k = 0; k < m; ++k) {
      double Rt1 = R1[(int64_t)j * m + k] + s1 / dn;
      double Rt2 = -(1.0 / dm + 1.0 / dn) * s2;
      double Rt3 = PR3[k] / dn + tot3 / (dn * dn);
      yh[(int64_t)j * m + k] = (Rt1 + Rt2 + Rt3) / (dm + dn);
    }
  }
  /* What = -diag(d) - d d^T / w */
  for (int32_t k = 0; k < m; ++k) d[k] = 1.0 / dm;
  d[m - 1] = (1.0 - 1.0 / dn) / (dm + 1.0);
  const double w = 1.0 / dm - (1.0 - 1.0 / dn) / (dm + 1.0);
  for (int32_t j = 0; j < n; ++j)
    for (int32_t k = 0; k < m; ++k) Y[k] += yh[(int64_t)j * m + k];
  double dY = 0.0;
  for (int32_t k = 0; k < m; ++k) dY += d[k] * Y[k];
  double sWY = 0.0;
  for (int32_t k = 0; k < m; ++k) {
    WY[k] = -d[k] * Y[k] - d[k] * dY / w;
    sWY += WY[k];
  }
  /* y1^j = yhat1^j - (I + 11^T/n) What Y */
  for (int32_t j = 0; j < n; ++j)
    for (int32_t k = 0; k < m; ++k)
      y1[(int64_t)j * m + k] = yh[(int64_t)j * m + k] - (WY[k] + sWY / dn);
  /* y2^j = (R2^j - (1^T y1^j) 1)/m */
  for (int32_t j = 0; j < n; ++j) {
    double s = 0.0;
    for (int32_t k = 0; k < m; ++k) s += y1[(int64_t)j * m + k];
    for (int32_t i = 0; i < m; ++i)
      y2[(int64_t)j * m + i] = (R2[(int64_t)j * m + i] - s) / dm;
  }
  /* y3^l = (R3^l + sum_j y1^j)/n */
  for (int32_t j = 0; j < n; ++j)
    for (int32_t k = 0; k < m; ++k) t[k] += y1[(int64_t)j * m + k];
  for (int32_t l = 0; l < n; ++l)
    for (int32_t k = 0; k < m; ++k) {
      if (l == n - 1 && k == m - 1) continue;
      y3[(int64_t)l * m + k] = (R3[(int64_t)l * m + k] + t[k]) / dn;
    }
  free(PR3); free(Y); free(WY); free(d); free(t); free(yh);
}

static double nrm2(int64_t len, const double *v) {
  double s = 0.0;
  for (int64_t e = 0; e < len; ++e) s += v[e] * v[e];
  return sqrt(s);
}
static double dot(int64_t len, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t e = 0; e < len; ++e) s += a[e] * b[e];
  return s;
}

/* Relative KKT residual of eq. kkt_res, with the reduced (A, b) of
 * eq. Mat:A&b and the full cost vector c. */
void or_kkt(int32_t m, int32_t n, const double *mu1, const double *mu2,
            const double *x, const double *y, const double *z, or_result *res) {
  or_kkt_xy(m, n, NULL, NULL, mu1, mu2, x, y, z, res);
}

void or_kkt_xy(int32_t m, int32_t n, const double *cu, const double *cv,
               const double *mu1, const double *mu2, const double *x,
               const double *y, const double *z, or_result *res) {
  int64_t N, M3;
  or_dims(m, n, &N, &M3);
  double *c = (double *)malloc((size_t)N * sizeof(double));
  double *b = (double *)malloc((size_t)M3 * sizeof(double));
  double *v = (double *)malloc((size_t)N * sizeof(double));
  double *r = (double *)malloc((size_t)M3 * sizeof(double));
  or_cost_xy(m, n, cu, cv, c);
  or_bvec(m, n, mu1, mu2, b);
  or_AT(m, n, y, v);
  double dsum = 0.0, csum = 0.0;
  for (int64_t e = 0; e < N; ++e) {
    double dr = v[e] + z[e] - c[e];
    dsum += dr * dr;
    double mn = x[e] < z[e] ? x[e] : z[e];
    csum += mn * mn;
  }
  or_A(m, n, x, r);
  for (int64_t q = 0; q < M3; ++q) r[q] -= b[q];
  /* R(w) = (b - A x, z - Pi_+(z - x), c - A^T y - z); for z >= 0 the middle
   * block equals min(x, z) elementwise */
  double msum = 0.0;
  for (int64_t e = 0; e < N; ++e) {
    double pz = z[e] - x[e];
    pz = pz > 0.0 ? pz : 0.0;
    double v = z[e] - pz;
    msum += v * v;
  }
  const double rp2 = dot(M3, r, r);
  /* negative part of x for the feasibility error of Sec. 4.1 */
  double nsum = 0.0;
  for (int64_t e = 0; e < N; ++e)
    if (x[e] < 0.0) nsum += x[e] * x[e];
  res->kkt_abs = sqrt(rp2 + msum + dsum);
  res->res_dual = sqrt(dsum) / (1.0 + nrm2(N, c));
  res->res_comp = sqrt(csum) / (1.0 + nrm2(N, x) + nrm2(N, z));
  res->res_primal = nrm2(M3, r) / (1.0 + nrm2(M3, b));
  double k = res->res_dual;
  if (res->res_comp > k) k = res->res_comp;
  if (res->res_primal > k) k = res->res_primal;
  res->kkt = k;
  {
    const double fneg = sqrt(nsum) / (1.0 + nrm2(N, x));
    res->feaserr = fneg > res->res_primal ? fneg : res->res_primal;
  }
  res->primal_obj = dot(N, c, x);
  res->dual_obj = dot(M3, b, y);
  free(c); free(b); free(v); free(r);
}

/* Algorithm 2 (alg:HOT) in the variables w = (y, z, x).  On the dual of the
 * reduced model (maximise b^T y subject to A^T y + z = c, z >= 0), x is the
 * multiplier of the equality and sigma its penalty; with the augmented
 * Lagrangian -b^T y + <x, A^T y + z - c> + (sigma/2) ||A^T y + z - c||^2:
 *   Step 1 minimises it over y (z, x held): setting its gradient to zero
 *     gives A A^T y_bar = b/sigma - A(x/sigma + z - c) (eq. update:y),
 *     solved by Prop. 3;
 *   Step 2 moves the multiplier along the residual at (y_bar, z):
 *     x_bar = x + sigma (A^T y_bar + z - c);
 *   Step 3 minimises it over z >= 0 with the new multiplier: the free
 *     minimiser c - A^T y_bar - x_bar/sigma, projected onto z >= 0;
 *   Step 4 averages the pass's output with the epoch's anchor w^0
 *     (Halpern weight 1/(k+2)).
 * Readings where the paper is silent: w^0 = 0; sigma = ||b||/||c|| unless
 * given; the check runs every T iterations of the current epoch (k % T == 0)
 * and evaluates eq. kkt_res at w_bar^k; with restarts on, the epoch restarts
 * (w^0 <- w_bar^k, w^k <- w_bar^k, k <- 0) when the fixed-point residual
 * r = 2 ||(x^k - x_bar^k)/sigma + z^k - z_bar^k|| falls to 0.2 of its value at
 * the epoch's start, or to 0.8 of it while having grown since the last check.
 * Returns 1 if converged, 0 otherwise. */
int32_t or_hot(int32_t m, int32_t n, const double *mu1, const double *mu2,
               const or_params *p, double *xbar, double *ybar, double *zbar,
               double *s_state, or_result *res) {
  int64_t N, M3;
  or_dims(m, n, &N, &M3);
  double *c = (double *)malloc((size_t)N * sizeof(double));
  double *b = (double *)malloc((size_t)M3 * sizeof(double));
  double *x = (double *)calloc((size_t)N, sizeof(double));
  double *z = (double *)calloc((size_t)N, sizeof(double));
  double *y = (double *)calloc((size_t)M3, sizeof(double));
  double *x0 = (double *)calloc((size_t)N, sizeof(double));
  double *z0 = (double *)calloc((size_t)N, sizeof(double));
  double *y0 = (double *)calloc((size_t)M3, sizeof(double));
  double *tmp = (double *)malloc((size_t)N * sizeof(double));
  double *aty = (double *)malloc((size_t)N * sizeof(double));
  double *R = (double *)malloc((size_t)M3 * sizeof(double));
  or_cost_xy(m, n, p->coord_row, p->coord_col, c);
  or_bvec(m, n, mu1, mu2, b);
  /* sigma = ||b||/||c||; on a 1 x 1 grid every cost is zero and the ratio is
   * undefined, so sigma = 1 there. */
  const double nb = nrm2(M3, b), nc = nrm2(N, c);
  double sigma = p->sigma > 0 ? p->sigma : ((nc > 0 && nb > 0) ? nb / nc : 1.0);
  /* optional re-balancing of sigma at restarts: x_bar and y_bar of the last
   * restart (the initial point 0 before the first) */
  double *Xr = p->sigma_update ? (double *)calloc((size_t)N, sizeof(double)) : NULL;
  double *Yr = p->sigma_update ? (double *)calloc((size_t)M3, sizeof(double)) : NULL;
  const int32_t T = p->check_every > 0 ? p->check_every : 1;
  const int32_t fixed = p->fixed_iters > 0 ? p->fixed_iters : 0;

  int32_t k = 0, it = 0, restarts = 0, converged = 0, ntrace = 0;
  double r_start = 0.0, r_prev = 0.0, r_last = 0.0;
  memset(res, 0, sizeof(*res));
  /* one record per check: (it, k, r, restarted) */
#define OR_TRACE(flag)                                   \
  do {                                                   \
    if (p->trace && ntrace < p->trace_cap) {             \
      double *t_ = p->trace + 4 * (int64_t)ntrace;       \
      t_[0] = (double)it;                                \
      t_[1] = (double)k;                                 \
      t_[2] = r_last;                                    \
      t_[3] = (flag);                                    \
      ++ntrace;                                          \
    }                                                    \
  } while (0)
  for (;;) {
    /* Step 1: A A^T y_bar = b/sigma - A(x/sigma + z - c) */
    OR_PARALLEL_FOR
    for (int64_t e = 0; e < N; ++e) tmp[e] = x[e] / sigma + z[e] - c[e];
    or_A(m, n, tmp, R);
    for (int64_t q = 0; q < M3; ++q) R[q] = b[q] / sigma - R[q];
    or_solve_aat(m, n, R, ybar);
    /* Step 2 */
    or_AT(m, n, ybar, aty);
    OR_PARALLEL_FOR
    for (int64_t e = 0; e < N; ++e) xbar[e] = x[e] + sigma * (aty[e] + z[e] - c[e]);
    /* Step 3 */
    OR_PARALLEL_FOR
    for (int64_t e = 0; e < N; ++e) {
      double v = c[e] - aty[e] - xbar[e] / sigma;
      zbar[e] = v > 0.0 ? v : 0.0;
    }
    if (fixed) {
      if (it == fixed) break;
    } else {
      int32_t last = (it >= p->max_iter);
      if (k % T == 0 || last) {
        or_kkt_xy(m, n, p->coord_row, p->coord_col, mu1, mu2, xbar, ybar, zbar, res);
        double acc = 0.0;
        for (int64_t e = 0; e < N; ++e) {
          double v = (x[e] - xbar[e]) / sigma + (z[e] - zbar[e]);
          acc += v * v;
        }
        r_last = 2.0 * sqrt(acc);
        const double crit = p->abs_kkt ? res->kkt_abs : res->kkt;
        const int32_t restart_now =
            p->restart && !(p->admm_rho > 0) && k > 0 &&
            (r_last <= 0.2 * r_start || (r_last <= 0.8 * r_start && r_last > r_prev));
        const int32_t stop = (p->tol > 0 && crit <= p->tol) || last;
        OR_TRACE((!stop && restart_now) ? 1.0 : 0.0);
        if (p->tol > 0 && crit <= p->tol) {
          converged = 1;
          break;
        }
        if (last) break;
        if (p->restart && !(p->admm_rho > 0)) {
          if (k == 0) {
            r_start = r_last;
            r_prev = r_last;
          } else if (restart_now) {
            if (p->sigma_update) {
              /* primal / dual displacement over the epoch that ends here:
               * dx = ||x_bar - X||, dy = ||A^T (y_bar - Y)||; the ratio puts
               * both on the same scale (sigma carries mass / cost units) */
              double dx2 = 0.0;
              for (int64_t e = 0; e < N; ++e) {
                const double d = xbar[e] - Xr[e];
                dx2 += d * d;
              }
              for (int64_t q = 0; q < M3; ++q) R[q] = ybar[q] - Yr[q];
              or_AT(m, n, R, tmp);
              const double dy = nrm2(N, tmp), dx = sqrt(dx2);
              if (dx > 0.0 && dy > 0.0 && isfinite(dx / dy)) sigma = dx / dy;
              memcpy(Xr, xbar, (size_t)N * sizeof(double));
              memcpy(Yr, ybar, (size_t)M3 * sizeof(double));
            }
            memcpy(x, xbar, (size_t)N * sizeof(double));
            memcpy(z, zbar, (size_t)N * sizeof(double));
            memcpy(y, ybar, (size_t)M3 * sizeof(double));
            memcpy(x0, xbar, (size_t)N * sizeof(double));
            memcpy(z0, zbar, (size_t)N * sizeof(double));
            memcpy(y0, ybar, (size_t)M3 * sizeof(double));
            k = 0;
            ++it;
            ++restarts;
            continue;
          } else {
            r_prev = r_last;
          }
        }
      }
    }
    if (p->admm_rho > 0) {
      /* generalized ADMM baseline of the experiments (Sec. 4.1): Step 4
       * replaced by w^{k+1} = (1 - rho) w^k + rho w_bar^k */
      const double rho = p->admm_rho;
      OR_PARALLEL_FOR
      for (int64_t e = 0; e < N; ++e) {
        x[e] = (1.0 - rho) * x[e] + rho * xbar[e];
        z[e] = (1.0 - rho) * z[e] + rho * zbar[e];
      }
      for (int64_t q = 0; q < M3; ++q) y[q] = (1.0 - rho) * y[q] + rho * ybar[q];
    } else {
      /* Step 4: w^{k+1} = w^0/(k+2) + (k+1)/(k+2) (2 w_bar - w) */
      const double a = 1.0 / (double)(k + 2), bb = (double)(k + 1) / (double)(k + 2);
      OR_PARALLEL_FOR
      for (int64_t e = 0; e < N; ++e) {
        x[e] = a * x0[e] + bb * (2.0 * xbar[e] - x[e]);
        z[e] = a * z0[e] + bb * (2.0 * zbar[e] - z[e]);
      }
      for (int64_t q = 0; q < M3; ++q) y[q] = a * y0[q] + bb * (2.0 * ybar[q] - y[q]);
    }
    ++k;
    ++it;
  }
  if (fixed) or_kkt_xy(m, n, p->coord_row, p->coord_col, mu1, mu2, xbar, ybar, zbar, res);
  if (s_state)
    for (int64_t e = 0; e < N; ++e) s_state[e] = x[e] / sigma + z[e];
  res->sigma = sigma;
  res->fp_res = r_last;
  res->iters = it;
  res->restarts = restarts;
  res->converged = converged;
  res->ntrace = ntrace;
#undef OR_TRACE
  free(c); free(b); free(x); free(z); free(y); free(x0); free(z0); free(y0);
  free(tmp); free(aty); free(R); free(Xr); free(Yr);
  return converged;
}

/* The plan of Algorithm 1 (alg:transportplan) from the clipped flows
 * f = max(x, 0).  Bin (k,j) receives the mass f1_{i,k,j} from each source
 * bin (i,j) of its column and sends f2_{k,j,l} to each target bin (k,l) of
 * its row; flow conservation at the bin (Prop. 1) makes the two totals
 * equal for an optimal flow.  Algorithm 1 pairs the two sequences greedily
 * in their natural order, i ascending against l ascending, always moving
 * the smaller of the two amounts still unmatched: the monotone
 * (north-west-corner) coupling of the two sequences.  It is walked here
 * with one cursor on each side; a source (target) whose amount is used up
 * moves its cursor on, and a pair of cursors with no mass left on one side
 * exchanges nothing, so the walk makes exactly the algorithm's nonzero
 * matches, in its order and with its subtractions.  Entries with positive
 * mass are written as (source bin i*n+j, target bin k*n+l, mass).  Returns
 * the number of entries (which may exceed cap: then only the first cap
 * entries are stored). */
int64_t or_recover(int32_t m, int32_t n, const double *x, int64_t cap,
                   int32_t *src, int32_t *dst, double *mass) {
  int64_t N, M3;
  or_dims(m, n, &N, &M3);
  double *in = (double *)malloc((size_t)m * sizeof(double));   /* column of the bin */
  double *out = (double *)malloc((size_t)n * sizeof(double));  /* row of the bin */
  int64_t nnz = 0;
  for (int32_t k = 0; k < m; ++k)
    for (int32_t j = 0; j < n; ++j) {
      for (int32_t i = 0; i < m; ++i) {
        const double v = x[ix1(m, n, i, k, j)];
        in[i] = v > 0.0 ? v : 0.0;
      }
      for (int32_t l = 0; l < n; ++l) {
        const double v = x[ix2(m, n, k, j, l)];
        out[l] = v > 0.0 ? v : 0.0;
      }
      int32_t i = 0, l = 0;
      while (i < m && l < n) {
        const double moved = in[i] < out[l] ? in[i] : out[l];
        in[i] -= moved;
        out[l] -= moved;
        if (moved > 0.0) {
          if (nnz < cap) {
            src[nnz] = i * n + j;
            dst[nnz] = k * n + l;
            mass[nnz] = moved;
          }
          ++nnz;
        }
        /* the side left with nothing moves on (both when both are used up) */
        const int32_t adv_i = !(in[i] > 0.0), adv_l = !(out[l] > 0.0);
        i += adv_i;
        l += adv_l;
      }
    }
  free(in);
  free(out);
  return nnz;
}

void or_marginals(int32_t m, int32_t n, int64_t nnz, const int32_t *src,
                  const int32_t *dst, const double *mass, double *row,
                  double *col) {
  const int64_t M = (int64_t)m * n;
  for (int64_t q = 0; q < M; ++q) row[q] = col[q] = 0.0;
  for (int64_t e = 0; e < nnz; ++e) {
    row[src[e]] += mass[e];
    col[dst[e]] += mass[e];
  }
}

/* Marginal repair of a plan recovered from an approximate flow (the paper
 * states Algorithm 1 for optimal flows only): scale down the rows whose sum
 * exceeds mu1, then the columns whose sum exceeds mu2, and couple the
 * remaining deficits of rows and columns with the north-west-corner rule in
 * bin order.  Appends the coupling entries; returns the new entry count
 * (entries beyond cap are counted, not stored). */
int64_t or_repair(int32_t m, int32_t n, const double *mu1, const double *mu2,
                  int64_t nnz, int64_t cap, int32_t *src, int32_t *dst,
                  double *mass) {
  const int64_t M = (int64_t)m * n;
  double *row = (double *)malloc((size_t)M * sizeof(double));
  double *col = (double *)malloc((size_t)M * sizeof(double));
  int64_t stored = nnz < cap ? nnz : cap;
  or_marginals(m, n, stored, src, dst, mass, row, col);
  for (int64_t e = 0; e < stored; ++e)
    if (row[src[e]] > mu1[src[e]]) mass[e] *= mu1[src[e]] / row[src[e]];
  or_marginals(m, n, stored, src, dst, mass, row, col);
  for (int64_t e = 0; e < stored; ++e)
    if (col[dst[e]] > mu2[dst[e]]) mass[e] *= mu2[dst[e]] / col[dst[e]];
  or_marginals(m, n, stored, src, dst, mass, row, col);
  for (int64_t q = 0; q < M; ++q) {
    double er = mu1[q] - row[q], ec = mu2[q] - col[q];
    row[q] = er > 0.0 ? er : 0.0; /* row deficit */
    col[q] = ec > 0.0 ? ec : 0.0; /* column deficit */
  }
  int64_t out = nnz;
  int64_t i = 0, l = 0;
  while (i < M && l < M) {
    double t = row[i] < col[l] ? row[i] : col[l];
    if (t > 0.0) {
      if (out < cap) {
        src[out] = (int32_t)i;
        dst[out] = (int32_t)l;
        mass[out] = t;
      }
      ++out;
    }
    row[i] -= t;
    col[l] -= t;
    if (row[i] <= 0.0) ++i;
    if (l < M && col[l] <= 0.0) ++l;
  }
  free(row);
  free(col);
  return out;
}

/* ------------------------------------------------------------------ */
/* Dense two-phase simplex with Bland's rule: min c^T x, A x = b, x >= 0.  */
/* Used only to pin the oracle to exact LP optima on tiny grids.            */
/* Returns 0 optimal, 1 infeasible, 2 unbounded, 3 iteration limit.         */
/* ------------------------------------------------------------------ */
static void pivot(int32_t rows, int32_t width, double *T, double *rhs,
                  int32_t pr, int32_t pc) {
  double *prow = T + (int64_t)pr * width;
  const double inv = 1.0 / prow[pc];
  for (int32_t q = 0; q < width; ++q) prow[q] *= inv;
  prow[pc] = 1.0;
  rhs[pr] *= inv;
  for (int32_t r = 0; r < rows; ++r) {
    if (r == pr) continue;
    double *row = T + (int64_t)r * width;
    const double f = row[pc];
    if (f == 0.0) continue;
    for (int32_t q = 0; q < width; ++q) row[q] -= f * prow[q];
    row[pc] = 0.0;
    rhs[r] -= f * rhs[pr];
  }
}

static int32_t bland_phase(int32_t rows, int32_t width, int32_t allowed,
                           double *T, double *rhs, int32_t *basis,
                           const char *dead, const double *cost) {
  const double eps = 1e-11;
  double *rc = (double *)malloc((size_t)width * sizeof(double));
  int32_t status = 3;
  for (int64_t iter = 0; iter < 1000000; ++iter) {
    for (int32_t q = 0; q < width; ++q) rc[q] = cost[q];
    for (int32_t r = 0; r < rows; ++r) {
      if (dead[r]) continue;
      const double cb = cost[basis[r]];
      if (cb == 0.0) continue;
      const double *row = T + (int64_t)r * width;
      for (int32_t q = 0; q < width; ++q) rc[q] -= cb * row[q];
    }
    int32_t enter = -1;
    for (int32_t q = 0; q < allowed; ++q)
      if (rc[q] < -eps) {
        enter = q;
        break;
      }
    if (enter < 0) {
      status = 0;
      break;
    }
    int32_t leave = -1;
    double best = 0.0;
    for (int32_t r = 0; r < rows; ++r) {
      if (dead[r]) continue;
      const double a = T[(int64_t)r * width + enter];
      if (a <= 1e-12) continue;
      const double ratio = rhs[r] / a;
      if (leave < 0 || ratio < best - 1e-14 ||
          (ratio <= best + 1e-14 && basis[r] < basis[leave])) {
        if (leave < 0 || ratio < best - 1e-14) best = ratio;
        leave = r;
      }
    }
    if (leave < 0) {
      status = 2;
      break;
    }
    pivot(rows, width, T, rhs, leave, enter);
    basis[leave] = enter;
  }
  free(rc);
  return status;
}

int32_t or_simplex(int32_t rows, int32_t cols, const double *A, const double *b,
                   const double *c, double *x, double *obj) {
  const int32_t width = cols + rows;
  double *T = (double *)calloc((size_t)rows * width, sizeof(double));
  double *rhs = (double *)malloc((size_t)rows * sizeof(double));
  double *cost = (double *)calloc((size_t)width, sizeof(double));
  int32_t *basis = (int32_t *)malloc((size_t)rows * sizeof(int32_t));
  char *dead = (char *)calloc((size_t)rows, 1);
  for (int32_t r = 0; r < rows; ++r) {
    const double sgn = b[r] < 0 ? -1.0 : 1.0;
    for (int32_t q = 0; q < cols; ++q)
      T[(int64_t)r * width + q] = sgn * A[(int64_t)r * cols + q];
    T[(int64_t)r * width + cols + r] = 1.0;
    rhs[r] = sgn * b[r];
    basis[r] = cols + r;
  }
  /* phase 1: minimise the sum of artificials */
  for (int32_t q = cols; q < width; ++q) cost[q] = 1.0;
  int32_t st = bland_phase(rows, width, width, T, rhs, basis, dead, cost);
  double infeas = 0.0;
  for (int32_t r = 0; r < rows; ++r)
    if (basis[r] >= cols) infeas += rhs[r];
  if (st != 0 || infeas > 1e-9) {
    free(T); free(rhs); free(cost); free(basis); free(dead);
    return st != 0 ? st : 1;
  }
  /* drive remaining (zero-level) artificials out of the basis */
  for (int32_t r = 0; r < rows; ++r) {
    if (basis[r] < cols) continue;
    int32_t q;
    for (q = 0; q < cols; ++q)
      if (fabs(T[(int64_t)r * width + q]) > 1e-9) break;
    if (q < cols) {
      pivot(rows, width, T, rhs, r, q);
      basis[r] = q;
    } else {
      dead[r] = 1; /* redundant equality */
    }
  }
  /* phase 2 */
  for (int32_t q = 0; q < width; ++q) cost[q] = q < cols ? c[q] : 0.0;
  st = bland_phase(rows, width, cols, T, rhs, basis, dead, cost);
  for (int32_t q = 0; q < cols; ++q) x[q] = 0.0;
  for (int32_t r = 0; r < rows; ++r)
    if (!dead[r] && basis[r] < cols) x[basis[r]] = rhs[r];
  double o = 0.0;
  for (int32_t q = 0; q < cols; ++q) o += c[q] * x[q];
  *obj = o;
  free(T); free(rhs); free(cost); free(basis); free(dead);
  return st;
}

/* Squared 2-Wasserstein distance between two histograms on 0..n-1 (mass
 * sums equal): the quantile coupling, i.e. the overlap of the CDF steps
 * [F_{j-1}, F_j) and [G_{l-1}, G_l) times (j-l)^2, summed over all pairs. */
double or_w2_1d(int32_t n, const double *a, const double *b) {
  double total = 0.0, Fj_1 = 0.0;
  for (int32_t j = 0; j < n; ++j) {
    const double Fj = Fj_1 + a[j];
    double Gl_1 = 0.0;
    for (int32_t l = 0; l < n; ++l) {
      const double Gl = Gl_1 + b[l];
      const double lo = Fj_1 > Gl_1 ? Fj_1 : Gl_1;
      const double hi = Fj < Gl ? Fj : Gl;
      if (hi > lo) total += (hi - lo) * (double)(j - l) * (double)(j - l);
      Gl_1 = Gl;
    }
    Fj_1 = Fj;
  }
  return total;
}
