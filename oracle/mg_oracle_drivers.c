/*
 * Plain CPU reference ("oracle"): coarsest-grid solve, norms and the outer
 * solve loops (plain FP64 and mixed precision).
 *
 * TEST INFRASTRUCTURE ONLY (see mg_oracle.h).  FP64 throughout; the mixed
 * loop calls the FP32 build of the V-cycle.  Build with -ffp-contract=off.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "mg_oracle.h"

/* Dense Gaussian elimination with partial pivoting, a (m x m, row-major) and
 * b are overwritten; the solution is returned in x. */
static void gauss_solve(int m, double* a, double* b, double* x) {
  for (int k = 0; k < m; ++k) {
    int piv = k;
    for (int i = k + 1; i < m; ++i)
      if (fabs(a[i * m + k]) > fabs(a[piv * m + k])) piv = i;
    if (piv != k) {
      for (int j = 0; j < m; ++j) {
        const double t = a[k * m + j];
        a[k * m + j] = a[piv * m + j];
        a[piv * m + j] = t;
      }
      const double t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
    for (int i = k + 1; i < m; ++i) {
      const double l = a[i * m + k] / a[k * m + k];
      for (int j = k; j < m; ++j) a[i * m + j] -= l * a[k * m + j];
      b[i] -= l * b[k];
    }
  }
  for (int i = m - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < m; ++j) s -= a[i * m + j] * x[j];
    x[i] = s / a[i * m + i];
  }
}

/* Coarsest grid, n = 5, h = 1/4.  The paper relaxes there (appendix V-cycle);
 * this build solves directly instead.
 *   Dirichlet: the 3 x 3 interior system A u = f, assembled and eliminated.
 *   Periodic:  the 4 x 4 torus; A is singular with the constants as null
 *   space, so the answer is the minimum-norm (zero-mean) solution of
 *   A u = f - mean(f), obtained as the unique solution of
 *   (A + c 1 1^T) u = f - mean(f) for any c > 0 (here c = 1). */
void orc_coarse_direct(int bc, const double* f, double* u) {
  const int n = 5;
  const double inv_h2 = 16.0;
  memset(u, 0, sizeof(double) * 25);
  if (bc == ORC_DIRICHLET) {
    double a[81], b[9], x[9];
    memset(a, 0, sizeof a);
    for (int i = 1; i <= 3; ++i)
      for (int j = 1; j <= 3; ++j) {
        const int k = (i - 1) * 3 + (j - 1);
        a[k * 9 + k] = 4.0 * inv_h2;
        const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
        for (int t = 0; t < 4; ++t) {
          const int ii = i + di[t], jj = j + dj[t];
          if (ii < 1 || ii > 3 || jj < 1 || jj > 3) continue; /* boundary value 0 */
          a[k * 9 + (ii - 1) * 3 + (jj - 1)] -= inv_h2;
        }
        b[k] = f[i * n + j];
      }
    gauss_solve(9, a, b, x);
    for (int i = 1; i <= 3; ++i)
      for (int j = 1; j <= 3; ++j) u[i * n + j] = x[(i - 1) * 3 + (j - 1)];
  } else {
    double a[256], b[16], x[16];
    memset(a, 0, sizeof a);
    double mean = 0.0;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) mean += f[i * n + j];
    mean /= 16.0;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        const int k = i * 4 + j;
        a[k * 16 + k] += 4.0 * inv_h2;
        const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
        for (int t = 0; t < 4; ++t) {
          const int ii = (i + di[t] + 4) % 4, jj = (j + dj[t] + 4) % 4;
          a[k * 16 + ii * 4 + jj] -= inv_h2;
        }
        b[k] = f[i * n + j] - mean;
      }
    for (int k = 0; k < 256; ++k) a[k] += 1.0;
    gauss_solve(16, a, b, x);
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) u[i * n + j] = x[(i % 4) * 4 + (j % 4)];
  }
}

/* Euclidean norm over the unknown nodes (Dirichlet interior, periodic unique
 * nodes), summed in natural order. */
double orc_norm2(int n, int bc, const double* a) {
  const int lo = bc == ORC_DIRICHLET ? 1 : 0;
  double s = 0.0;
  for (int i = lo; i <= n - 2; ++i)
    for (int j = lo; j <= n - 2; ++j) s += a[(size_t)i * n + j] * a[(size_t)i * n + j];
  return sqrt(s);
}

/* ||f - A u|| / ||f|| over the unknown nodes (the stopping measure; the paper
 * stops on the change between iterates instead, Section 4.2). */
double orc_relres(int n, int bc, const double* u, const double* f) {
  double* r = (double*)malloc(sizeof(double) * (size_t)n * n);
  orc_residual_f64(n, bc, u, f, r);
  const double rn = orc_norm2(n, bc, r);
  free(r);
  const double fn = orc_norm2(n, bc, f);
  return fn > 0.0 ? rn / fn : rn;
}

/* Repeat FP64 V-cycles from the given u until relres <= rtol or max_cycles.
 * hist (length max_cycles + 1, may be NULL) receives relres before the first
 * and after every cycle.  Returns the number of cycles done. */
int orc_solve_f64(int n, int bc, int nu1, int nu2, double* u, const double* f,
                  double rtol, int max_cycles, double* hist) {
  double rr = orc_relres(n, bc, u, f);
  if (hist) hist[0] = rr;
  int c = 0;
  while (c < max_cycles && !(rr <= rtol)) {
    orc_vcycle_f64(n, bc, nu1, nu2, u, f);
    ++c;
    rr = orc_relres(n, bc, u, f);
    if (hist) hist[c] = rr;
  }
  return c;
}

/* One step of FP64 iterative refinement around FP32 V-cycles:
 *   r = f - A u in FP64, rounded to FP32;
 *   e = 0, then `inner` FP32 V-cycles on A e = r (coarsest solve in FP64);
 *   u += e in FP64. */
void orc_refine_step(int n, int bc, int nu1, int nu2, int inner, double* u, const double* f) {
  const size_t nn = (size_t)n * n;
  double* r = (double*)malloc(sizeof(double) * nn);
  float* r32 = (float*)malloc(sizeof(float) * nn);
  float* e32 = (float*)calloc(nn, sizeof(float));
  orc_residual_f64(n, bc, u, f, r);
  for (size_t k = 0; k < nn; ++k) r32[k] = (float)r[k];
  for (int s = 0; s < inner; ++s) orc_vcycle_f32(n, bc, nu1, nu2, e32, r32);
  for (size_t k = 0; k < nn; ++k) u[k] += (double)e32[k];
  free(e32);
  free(r32);
  free(r);
}

/* Refinement loop: same contract as orc_solve_f64, counting refinement steps. */
int orc_solve_mixed(int n, int bc, int nu1, int nu2, int inner, double* u,
                    const double* f, double rtol, int max_steps, double* hist) {
  double rr = orc_relres(n, bc, u, f);
  if (hist) hist[0] = rr;
  int c = 0;
  while (c < max_steps && !(rr <= rtol)) {
    orc_refine_step(n, bc, nu1, nu2, inner, u, f);
    ++c;
    rr = orc_relres(n, bc, u, f);
    if (hist) hist[c] = rr;
  }
  return c;
}

/* Two-level solve of the paper's controlled experiment (Section 4.1): the
 * initial grid is relaxed n_pre times (N_smooth,pre on an initially random
 * grid, Table 1), then two-level iterations run until the change between
 * successive iterates, ||p_i - p_(i-1)||_2 over the unique nodes, is at most
 * tol (the paper's stopping rule, Section 4.2; it names no norm). */
int orc_twolevel_solve(int n, int F, int n_smooth, int coarse_sweeps, int n_pre, double* p,
                       const double* f, double tol, int max_iter, double* hist) {
  const size_t nn = (size_t)n * n;
  double* prev = (double*)malloc(sizeof(double) * nn);
  for (int s = 0; s < n_pre; ++s) {
    orc_relax_f64(n, ORC_PERIODIC, p, f, ORC_RED);
    orc_relax_f64(n, ORC_PERIODIC, p, f, ORC_BLACK);
  }
  int it = 0;
  while (it < max_iter) {
    memcpy(prev, p, sizeof(double) * nn);
    orc_twolevel_f64(n, F, n_smooth, coarse_sweeps, p, f);
    for (size_t k = 0; k < nn; ++k) prev[k] = p[k] - prev[k];
    const double change = orc_norm2(n, ORC_PERIODIC, prev);
    if (hist) hist[it] = change;
    ++it;
    if (change <= tol) break;
  }
  free(prev);
  return it;
}
