/*
 * hot_oracle.h -- FP64 CPU oracle for HOT (Halpern accelerating method for
 * optimal transport, arXiv 2408.00598).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * package's smoke() check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Conventions follow the paper's standard-form LP (Sec. 2.1, eqs. standLP0,
 * def:A1A2A3, Mat:A&b, def:A4), written 0-based:
 *   grid m x n, M = m n, N = m^2 n + m n^2, M3 = 3M - 1;
 *   x = [f1; f2],  f1_{i,k,j} at x[(j*m + k)*m + i],
 *                  f2_{k,j,l} at x[m*m*n + (l*n + j)*m + k];
 *   y = [y1; y2; y3], y1 row (j,k) at j*m+k (conservation at bin (k,j)),
 *                     y2 row (j,i) at M + j*m+i (source marginal of bin (i,j)),
 *                     y3 row (l,k) at 2M + l*m+k (target marginal of bin (k,l)),
 *                     the row (l,k) = (n-1,m-1) is dropped (def:A4);
 *   histograms are row-major images: mu[i*n + j] is the mass of bin (i,j).
 */
#ifndef HOT_ORACLE_H
#define HOT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double tol;        /* stop when the relative KKT residual (eq. kkt_res) <= tol; <=0: never */
  int32_t max_iter;  /* hard cap on iterations */
  int32_t check_every; /* check cadence T (>=1) */
  double sigma;      /* > 0: use it; <= 0: sigma = ||b|| / ||c|| */
  int32_t restart;   /* 1: restart rule on, 0: Algorithm 2 verbatim */
  int32_t fixed_iters; /* > 0: run exactly this many updates, no stop test */
  double admm_rho;   /* > 0: Step 4 replaced by w <- (1-rho) w + rho w_bar (no restarts) */
  int32_t abs_kkt;   /* 1: stop on the absolute residual ||R(w_bar)|| instead of eq. kkt_res */
  const double *coord_row; /* m grid-line positions u_i, or NULL for u_i = i */
  const double *coord_col; /* n grid-line positions v_j, or NULL for v_j = j */
  int32_t sigma_update; /* 1: at every restart, sigma <- ||x_bar - X|| / ||A^T (y_bar - Y)||
                           with (X, Y) the w_bar of the previous restart (w^0 = 0 at first) */
  double *trace;       /* nullable: 4 doubles per check (iteration count it, epoch
                          counter k, fixed-point residual r, 1 if the check
                          restarts the epoch else 0), at most trace_cap checks */
  int32_t trace_cap;
} or_params;

typedef struct {
  double primal_obj;   /* <c, xbar> */
  double dual_obj;     /* <b, ybar> */
  double kkt;          /* max of the three relative residuals */
  double res_dual;     /* ||A^T ybar + zbar - c|| / (1 + ||c||) */
  double res_comp;     /* ||min(xbar, zbar)|| / (1 + ||xbar|| + ||zbar||) */
  double res_primal;   /* ||A xbar - b|| / (1 + ||b||) */
  double sigma;
  double fp_res;       /* ||s - shat|| with s = x/sigma + z: fixed-point residual */
  double kkt_abs;      /* ||R(w_bar)||: the residual map of the complexity proposition */
  double feaserr;      /* max(||min(xbar, 0)|| / (1 + ||xbar||), res_primal): the
                          relative primal feasibility error of the experiments (Sec. 4.1) */
  int32_t iters;       /* number of updates performed */
  int32_t restarts;
  int32_t converged;
  int32_t ntrace;      /* checks recorded in or_params.trace */
} or_result;

void or_dims(int32_t m, int32_t n, int64_t *N, int64_t *M3);
void or_cost(int32_t m, int32_t n, double *c);
void or_cost_xy(int32_t m, int32_t n, const double *u, const double *v, double *c);
void or_bvec(int32_t m, int32_t n, const double *mu1, const double *mu2, double *b);
void or_A(int32_t m, int32_t n, const double *x, double *out);
void or_AT(int32_t m, int32_t n, const double *y, double *out);
void or_solve_aat(int32_t m, int32_t n, const double *R, double *y);
void or_kkt(int32_t m, int32_t n, const double *mu1, const double *mu2,
            const double *x, const double *y, const double *z, or_result *res);
void or_kkt_xy(int32_t m, int32_t n, const double *cu, const double *cv,
               const double *mu1, const double *mu2, const double *x,
               const double *y, const double *z, or_result *res);
int32_t or_hot(int32_t m, int32_t n, const double *mu1, const double *mu2,
               const or_params *p, double *xbar, double *ybar, double *zbar,
               double *s_state, or_result *res);
int64_t or_recover(int32_t m, int32_t n, const double *x, int64_t cap,
                   int32_t *src, int32_t *dst, double *mass);
int64_t or_repair(int32_t m, int32_t n, const double *mu1, const double *mu2,
                  int64_t nnz, int64_t cap, int32_t *src, int32_t *dst,
                  double *mass);
void or_marginals(int32_t m, int32_t n, int64_t nnz, const int32_t *src,
                  const int32_t *dst, const double *mass, double *row,
                  double *col);
int32_t or_simplex(int32_t rows, int32_t cols, const double *A, const double *b,
                   const double *c, double *x, double *obj);
double or_w2_1d(int32_t n, const double *a, const double *b);

#ifdef __cplusplus
}
#endif
#endif
