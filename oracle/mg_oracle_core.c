/*
 * Plain CPU reference ("oracle") for the 2-D Poisson multigrid V-cycle:
 * the per-level steps and the recursive cycle.
 *
 * TEST INFRASTRUCTURE ONLY (see mg_oracle.h).  Parity status: every function
 * here is pinned by tests that do not reuse this code (closed forms, library
 * routines, dense linear algebra, invariants); none is "parity unpinned".
 *
 * This file is compiled twice: with REAL=double, SFX=f64 (the FP64 path) and
 * with REAL=float, SFX=f32 (emulation of the FP32 inner cycle of the mixed
 * path).  Loops are plain and in natural order; there is no blocking, fusion
 * or reordering.  Build with -ffp-contract=off so that every operation rounds.
 * Loops whose iterations write disjoint outputs and read nothing written in
 * the same loop (one colour of a half-sweep, the residual, the restriction,
 * independent spline lines) may run on several OpenMP threads; results are
 * bitwise independent of the thread count.  Sums stay serial.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "mg_oracle.h"

#ifndef REAL
#error "REAL must be defined"
#endif
#define PASTE_(a, b) a##_##b
#define PASTE(a, b) PASTE_(a, b)
#define FN(name) PASTE(name, SFX)

typedef REAL real;

static int wrap_index(int i, int m) { return ((i % m) + m) % m; }

/* Value of grid function a at node (i, j).  Periodic grids wrap over the
 * n-1 unique nodes; zero-Dirichlet grids are only ever asked for nodes in
 * 0..n-1, whose boundary entries hold 0. */
static real at(const real* a, int n, int bc, int i, int j) {
  if (bc == ORC_PERIODIC) {
    i = wrap_index(i, n - 1);
    j = wrap_index(j, n - 1);
  }
  return a[(size_t)i * n + j];
}

/* First unknown index per direction; the last is n-2 for both conditions. */
static int first_unknown(int bc) { return bc == ORC_DIRICHLET ? 1 : 0; }

/* Periodic storage: row and column n-1 repeat row and column 0. */
static void refresh_seam(real* a, int n, int bc) {
  if (bc != ORC_PERIODIC) return;
  for (int j = 0; j < n; ++j) a[(size_t)(n - 1) * n + j] = a[j];
  for (int i = 0; i < n; ++i) a[(size_t)i * n + (n - 1)] = a[(size_t)i * n];
}

static real neighbour_sum(const real* u, int n, int bc, int i, int j) {
  return at(u, n, bc, i - 1, j) + at(u, n, bc, i + 1, j) + at(u, n, bc, i, j - 1) +
         at(u, n, bc, i, j + 1);
}

/* One Gauss-Seidel half-sweep over the nodes of one colour (Section 2.2
 * names Gauss-Seidel relaxation and red-black ordering; the V-cycle of the
 * appendix relaxes before and after the coarse correction).  Each node of
 * the colour solves its own row of A u = f exactly with its four neighbours,
 * which all have the other colour, held fixed:
 *     u_ij <- (h^2 f_ij + u_{i-1,j} + u_{i+1,j} + u_{i,j-1} + u_{i,j+1}) / 4. */
void FN(orc_relax)(int n, int bc, real* u, const real* f, int colour) {
  const double hd = 1.0 / (double)(n - 1);
  const real h2 = (real)(hd * hd);
  const int lo = first_unknown(bc);
#pragma omp parallel for schedule(static)
  for (int i = lo; i <= n - 2; ++i)
    for (int j = lo; j <= n - 2; ++j) {
      if (((i + j) & 1) != colour) continue;
      const real s = neighbour_sum(u, n, bc, i, j);
      u[(size_t)i * n + j] = (h2 * f[(size_t)i * n + j] + s) * (real)0.25;
    }
  refresh_seam(u, n, bc);
}

/* Residual r = f - A u with A u = (4 u_ij - sum of the four neighbours)/h^2
 * (the appendix's V-cycle forms r = f - A p before restricting).  Zero at
 * Dirichlet boundary nodes. */
void FN(orc_residual)(int n, int bc, const real* u, const real* f, real* r) {
  const real inv_h2 = (real)((double)(n - 1) * (double)(n - 1));
  const int lo = first_unknown(bc);
  memset(r, 0, sizeof(real) * (size_t)n * n);
#pragma omp parallel for schedule(static)
  for (int i = lo; i <= n - 2; ++i)
    for (int j = lo; j <= n - 2; ++j) {
      const real s = neighbour_sum(u, n, bc, i, j);
      const real au = ((real)4 * u[(size_t)i * n + j] - s) * inv_h2;
      r[(size_t)i * n + j] = f[(size_t)i * n + j] - au;
    }
  refresh_seam(r, n, bc);
}

/* Full-weighting restriction to the grid of spacing 2h (node (I, J) sits on
 * fine node (2I, 2J)):
 *     f_c = (4 r_centre + 2 (sum of 4 edge neighbours) + (sum of 4 corners)) / 16.
 * The paper's restriction is described only loosely (Section 2.2); full
 * weighting is the reading used here.  Coarse Dirichlet boundary nodes are 0. */
void FN(orc_restrict)(int n, int bc, const real* r, real* fc) {
  const int nc = (n - 1) / 2 + 1;
  const int lo = first_unknown(bc);
  memset(fc, 0, sizeof(real) * (size_t)nc * nc);
#pragma omp parallel for schedule(static)
  for (int I = lo; I <= nc - 2; ++I)
    for (int J = lo; J <= nc - 2; ++J) {
      const int i = 2 * I, j = 2 * J;
      const real centre = at(r, n, bc, i, j);
      const real edges = at(r, n, bc, i - 1, j) + at(r, n, bc, i + 1, j) +
                         at(r, n, bc, i, j - 1) + at(r, n, bc, i, j + 1);
      const real corners = at(r, n, bc, i - 1, j - 1) + at(r, n, bc, i - 1, j + 1) +
                           at(r, n, bc, i + 1, j - 1) + at(r, n, bc, i + 1, j + 1);
      fc[(size_t)I * nc + J] = ((real)4 * centre + (real)2 * edges + corners) / (real)16;
    }
  refresh_seam(fc, nc, bc);
}

/* Thomas algorithm for the constant tridiagonal system
 *     x_{k-1} + 4 x_k + x_{k+1} = d_k,  k = 0..m-1,  x_{-1} = x_m = 0.
 * d is overwritten; cp is workspace of length m. */
static void solve_141(int m, real* d, real* cp, real* x) {
  if (m <= 0) return;
  cp[0] = (real)1 / (real)4;
  d[0] = d[0] / (real)4;
  for (int k = 1; k < m; ++k) {
    const real denom = (real)4 - cp[k - 1];
    cp[k] = (real)1 / denom;
    d[k] = (d[k] - d[k - 1]) / denom;
  }
  x[m - 1] = d[m - 1];
  for (int k = m - 2; k >= 0; --k) x[k] = d[k] - cp[k] * x[k + 1];
}

/* Tridiagonal solve with unit off-diagonals, diagonal b0 on row 0, bl on
 * row p-1 and 4 elsewhere.  src is read, dst written; rhs and cp are
 * workspace of length p. */
static void thomas_ends(int p, real b0, real bl, const real* src, real* dst, real* rhs, real* cp) {
  for (int k = 0; k < p; ++k) rhs[k] = src[k];
  real diag = b0;
  cp[0] = (real)1 / diag;
  rhs[0] = rhs[0] / diag;
  for (int k = 1; k < p; ++k) {
    diag = (k == p - 1 ? bl : (real)4) - cp[k - 1];
    cp[k] = (real)1 / diag;
    rhs[k] = (rhs[k] - rhs[k - 1]) / diag;
  }
  dst[p - 1] = rhs[p - 1];
  for (int k = p - 2; k >= 0; --k) dst[k] = rhs[k] - cp[k] * dst[k + 1];
}

/* Cyclic version: x_{k-1} + 4 x_k + x_{k+1} = d_k with indices mod p (p >= 3),
 * by the Sherman-Morrison correction of a tridiagonal solve: the cyclic
 * matrix is T + u v^T with u = (g, 0, .., 0, 1), v = (1, 0, .., 0, 1/g), so T
 * is tridiagonal with diagonal 4 - g on row 0 and 4 - 1/g on row p-1.
 * w is workspace of length 5p. */
static void solve_141_cyclic(int p, const real* d, real* w, real* x) {
  real* y = w;
  real* z = w + p;
  real* uvec = w + 2 * p;
  real* rhs = w + 3 * p;
  real* cp = w + 4 * p;
  const real g = (real)-4;
  const real b0 = (real)4 - g, bl = (real)4 - (real)1 / g;
  thomas_ends(p, b0, bl, d, y, rhs, cp);
  for (int k = 0; k < p; ++k) uvec[k] = 0;
  uvec[0] = g;
  uvec[p - 1] = 1;
  thomas_ends(p, b0, bl, uvec, z, rhs, cp);
  const real vy = y[0] + y[p - 1] / g;
  const real vz = z[0] + z[p - 1] / g;
  const real fac = vy / ((real)1 + vz);
  for (int k = 0; k < p; ++k) x[k] = y[k] - fac * z[k];
}

/* Interpolating cubic spline through y_0..y_{m-1} at unit spacing, evaluated
 * at the 2m-1 points of half spacing (the spline is invariant under scaling
 * of x, so the coarse spacing is taken as 1).  Textbook second-derivative
 * (moment) form: on each interval the spline is the cubic with end values
 * y_k, y_{k+1} and second derivatives M_k, M_{k+1}, and continuity of the
 * first derivative gives  M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k+1} - 2 y_k + y_{k-1}).
 * At the midpoint the cubic equals (y_k + y_{k+1})/2 - (M_k + M_{k+1})/16.
 *   natural  (bc = Dirichlet): M_0 = M_{m-1} = 0;
 *   periodic (bc = periodic):  y_{m-1} = y_0 and indices wrap over m-1 nodes.
 * This is the bivariate-spline prolongation of Section 2.2 read as a tensor
 * product of 1-D interpolating cubic splines. */
static void spline_line(int m, int bc, const real* y, real* out, real* work) {
  real* M = work;          /* m */
  real* d = work + m;      /* m */
  real* w = work + 2 * m;  /* 5m */
  if (bc == ORC_DIRICHLET) {
    const int q = m - 2; /* unknown moments M_1..M_{m-2} */
    for (int k = 1; k <= m - 2; ++k) d[k - 1] = (real)6 * (y[k + 1] - (real)2 * y[k] + y[k - 1]);
    M[0] = 0;
    M[m - 1] = 0;
    solve_141(q, d, w, M + 1);
  } else {
    const int p = m - 1;
    for (int k = 0; k < p; ++k) {
      const real ym = y[(k - 1 + p) % p], y0 = y[k], yp = y[(k + 1) % p];
      d[k] = (real)6 * (yp - (real)2 * y0 + ym);
    }
    solve_141_cyclic(p, d, w, M);
    M[m - 1] = M[0];
  }
  for (int k = 0; k < m; ++k) out[2 * k] = y[k];
  for (int k = 0; k + 1 < m; ++k)
    out[2 * k + 1] = (y[k] + y[k + 1]) / (real)2 - (M[k] + M[k + 1]) / (real)16;
}

/* Prolongation of a coarse grid function (nc per side) to the fine grid
 * (n = 2 nc - 1): cubic-spline interpolation along x for every coarse row,
 * then along y for every fine column.  Returns P e_c (not added). */
void FN(orc_prolong)(int nc, int bc, const real* ec, real* ef) {
  const int n = 2 * (nc - 1) + 1;
  real* tmp = (real*)malloc(sizeof(real) * (size_t)nc * n);
#pragma omp parallel
  {
    real* work = (real*)malloc(sizeof(real) * (size_t)7 * (nc + 2));
    real* col = (real*)malloc(sizeof(real) * (size_t)nc);
    real* fcol = (real*)malloc(sizeof(real) * (size_t)n);
#pragma omp for schedule(static)
    for (int I = 0; I < nc; ++I)
      spline_line(nc, bc, ec + (size_t)I * nc, tmp + (size_t)I * n, work);
#pragma omp for schedule(static)
    for (int j = 0; j < n; ++j) {
      for (int I = 0; I < nc; ++I) col[I] = tmp[(size_t)I * n + j];
      spline_line(nc, bc, col, fcol, work);
      for (int i = 0; i < n; ++i) ef[(size_t)i * n + j] = fcol[i];
    }
    free(fcol);
    free(col);
    free(work);
  }
  free(tmp);
}

/* Coarsest grid (n = 5): direct solve in FP64 whatever the cycle precision. */
void FN(orc_coarse)(int bc, const real* f, real* u) {
  double fd[25], ud[25];
  for (int k = 0; k < 25; ++k) fd[k] = (double)f[k];
  orc_coarse_direct(bc, fd, ud);
  for (int k = 0; k < 25; ++k) u[k] = (real)ud[k];
}

/* One V(nu1, nu2) cycle on A u = f (appendix: multigrid algorithm with
 * V-cycle structure; Section 2.2), recursing down to the 5 x 5 grid:
 *   relax nu1 times (red then black half-sweep each time),
 *   r = f - A u, f_c = R r, u_c = 0, recurse on (u_c, f_c),
 *   u += P u_c (cubic spline), relax nu2 times.
 * u is updated in place; f is not modified. */
void FN(orc_vcycle)(int n, int bc, int nu1, int nu2, real* u, const real* f) {
  if (n == 5) {
    FN(orc_coarse)(bc, f, u);
    return;
  }
  const int nc = (n - 1) / 2 + 1;
  for (int s = 0; s < nu1; ++s) {
    FN(orc_relax)(n, bc, u, f, ORC_RED);
    FN(orc_relax)(n, bc, u, f, ORC_BLACK);
  }
  real* r = (real*)malloc(sizeof(real) * (size_t)n * n);
  real* fc = (real*)malloc(sizeof(real) * (size_t)nc * nc);
  real* uc = (real*)calloc((size_t)nc * nc, sizeof(real));
  FN(orc_residual)(n, bc, u, f, r);
  FN(orc_restrict)(n, bc, r, fc);
  FN(orc_vcycle)(nc, bc, nu1, nu2, uc, fc);
  real* ef = r; /* reuse */
  FN(orc_prolong)(nc, bc, uc, ef);
  const int lo = first_unknown(bc);
#pragma omp parallel for schedule(static)
  for (int i = lo; i <= n - 2; ++i)
    for (int j = lo; j <= n - 2; ++j) u[(size_t)i * n + j] += ef[(size_t)i * n + j];
  refresh_seam(u, n, bc);
  for (int s = 0; s < nu2; ++s) {
    FN(orc_relax)(n, bc, u, f, ORC_RED);
    FN(orc_relax)(n, bc, u, f, ORC_BLACK);
  }
  free(uc);
  free(fc);
  free(r);
}

/* ---------------------------------------------------------------------------
 * The paper's controlled two-level experiment (Section 4.1; Table 1: N_grid,
 * r_min, N_step, N_smooth, N_smooth,pre; appendix V-CYCLE with the coarse
 * level relaxed rather than solved).  Periodic grids only (the paper's
 * fields are biperiodic), n = N + 1 stored nodes per side with the seam, N
 * divisible by the coarsening factor F = 2^N_step and N/F even (red-black
 * colouring agrees across the wrap only on even sides).
 * ------------------------------------------------------------------------- */

/* Restriction by the factor F: the tensor product of the 1-D weights
 * w_a = (F - |a|) / F^2 for |a| < F, centred on the fine node F*I under coarse
 * node I.  For F = 2 these are (1/4, 1/2, 1/4), i.e. full weighting; for any F
 * the 1-D operator is the transpose of linear interpolation by F divided by
 * F, so constants are kept and sums are kept up to the factor F per axis.
 * The paper coarsens 192 -> 12 in one step (Section 4.1) and names no
 * weights; this is full weighting widened to the step.  Applied along x for
 * every fine row, then along y; each sum runs over a = -(F-1) .. F-1 in
 * increasing order. */
void FN(orc_restrict_factor)(int n, int F, const real* r, real* fc) {
  const int N = n - 1, Nc = N / F, nc = Nc + 1;
  real* s = (real*)malloc(sizeof(real) * (size_t)N * Nc);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < N; ++i)
    for (int J = 0; J < Nc; ++J) {
      real acc = 0;
      for (int a = -(F - 1); a <= F - 1; ++a) {
        const real w = (real)(F - abs(a)) / (real)(F * F);
        acc += w * r[(size_t)i * n + wrap_index(F * J + a, N)];
      }
      s[(size_t)i * Nc + J] = acc;
    }
#pragma omp parallel for schedule(static)
  for (int I = 0; I < Nc; ++I)
    for (int J = 0; J < Nc; ++J) {
      real acc = 0;
      for (int a = -(F - 1); a <= F - 1; ++a) {
        const real w = (real)(F - abs(a)) / (real)(F * F);
        acc += w * s[(size_t)wrap_index(F * I + a, N) * Nc + J];
      }
      fc[(size_t)I * nc + J] = acc;
    }
  refresh_seam(fc, nc, ORC_PERIODIC);
  free(s);
}

/* Periodic interpolating cubic spline through y_0..y_{m-1} (y_{m-1} = y_0)
 * at unit spacing, evaluated at the F points t = q/F, q = 0..F-1, of every
 * interval: out[F k + q], k = 0..m-2, and out[F (m-1)] = y_0.  Moments M from
 * the cyclic system of spline_line; on [k, k+1] the spline is the textbook
 *   S(t) = (1-t) y_k + t y_{k+1} + (((1-t)^3 - (1-t)) M_k + (t^3 - t) M_{k+1}) / 6. */
static void spline_line_factor(int m, int F, const real* y, real* out, real* work) {
  real* M = work;          /* m */
  real* d = work + m;      /* m */
  real* w = work + 2 * m;  /* 5m */
  const int p = m - 1;
  for (int k = 0; k < p; ++k) {
    const real ym = y[(k - 1 + p) % p], y0 = y[k], yp = y[(k + 1) % p];
    d[k] = (real)6 * (yp - (real)2 * y0 + ym);
  }
  solve_141_cyclic(p, d, w, M);
  M[m - 1] = M[0];
  for (int k = 0; k < p; ++k)
    for (int q = 0; q < F; ++q) {
      const real t = (real)q / (real)F, u = (real)1 - t;
      out[F * k + q] = u * y[k] + t * y[k + 1] +
                       ((u * u * u - u) * M[k] + (t * t * t - t) * M[k + 1]) / (real)6;
    }
  out[F * p] = y[0];
}

/* Prolongation by the factor F of a periodic coarse grid function (nc per
 * side, seam included) to the fine grid n = F (nc - 1) + 1: the tensor cubic
 * spline (Section 2.2's bivariate spline, periodic), along x for every coarse
 * row, then along y for every fine column.  Returns P e_c (not added). */
void FN(orc_prolong_factor)(int nc, int F, const real* ec, real* ef) {
  const int n = F * (nc - 1) + 1;
  real* tmp = (real*)malloc(sizeof(real) * (size_t)nc * n);
#pragma omp parallel
  {
    real* work = (real*)malloc(sizeof(real) * (size_t)7 * (nc + 2));
    real* col = (real*)malloc(sizeof(real) * (size_t)nc);
    real* fcol = (real*)malloc(sizeof(real) * (size_t)n);
#pragma omp for schedule(static)
    for (int I = 0; I < nc; ++I)
      spline_line_factor(nc, F, ec + (size_t)I * nc, tmp + (size_t)I * n, work);
#pragma omp for schedule(static)
    for (int j = 0; j < n; ++j) {
      for (int I = 0; I < nc; ++I) col[I] = tmp[(size_t)I * n + j];
      spline_line_factor(nc, F, col, fcol, work);
      for (int i = 0; i < n; ++i) ef[(size_t)i * n + j] = fcol[i];
    }
    free(fcol);
    free(col);
    free(work);
  }
  free(tmp);
}

/* One iteration of the two-level method (appendix V-CYCLE with a single
 * coarse level, Section 4.1's set-up): relax n_smooth times on the fine grid
 * (red then black half-sweep each), r = f - A p, r_c = R_F r, delta_c = 0,
 * relax coarse_sweeps times on A_c delta_c = r_c (the coarse operator is the
 * 5-point one rediscretised at spacing F h; the coarsest level is relaxed,
 * not solved), then p += P_F delta_c.  The paper relaxes only at the start
 * of an iteration (N_smooth is the smoothing between iterations), so there
 * is no post-smoothing.  p is updated in place (seam rewritten). */
void FN(orc_twolevel)(int n, int F, int n_smooth, int coarse_sweeps, real* p, const real* f) {
  const int nc = (n - 1) / F + 1;
  for (int s = 0; s < n_smooth; ++s) {
    FN(orc_relax)(n, ORC_PERIODIC, p, f, ORC_RED);
    FN(orc_relax)(n, ORC_PERIODIC, p, f, ORC_BLACK);
  }
  real* r = (real*)malloc(sizeof(real) * (size_t)n * n);
  real* rc = (real*)malloc(sizeof(real) * (size_t)nc * nc);
  real* dc = (real*)calloc((size_t)nc * nc, sizeof(real));
  FN(orc_residual)(n, ORC_PERIODIC, p, f, r);
  FN(orc_restrict_factor)(n, F, r, rc);
  for (int s = 0; s < coarse_sweeps; ++s) {
    FN(orc_relax)(nc, ORC_PERIODIC, dc, rc, ORC_RED);
    FN(orc_relax)(nc, ORC_PERIODIC, dc, rc, ORC_BLACK);
  }
  real* ef = r; /* reuse */
  FN(orc_prolong_factor)(nc, F, dc, ef);
  const int N = n - 1;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) p[(size_t)i * n + j] += ef[(size_t)i * n + j];
  refresh_seam(p, n, ORC_PERIODIC);
  free(dc);
  free(rc);
  free(r);
}

