/*
 * Plain CPU reference ("oracle") for the 2-D Poisson multigrid V-cycle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no source with the HIP
 * library.
 *
 * Conventions (all functions):
 *   n      nodes per side, n - 1 = 4 * 2^k, n >= 5; h = 1/(n-1).
 *   bc     ORC_DIRICHLET (zero boundary values, unknowns 1..n-2) or
 *          ORC_PERIODIC (unknowns 0..n-2, row/column n-1 repeats 0).
 *   arrays n*n row-major, a[i*n + j], i = y index, j = x index.
 *   The operator is A = -Delta_h (5-point), so A u = f is the paper's
 *   Poisson equation (Section 2.2) with the sign flipped to make A SPD.
 */
#ifndef MG_ORACLE_H
#define MG_ORACLE_H

#define ORC_DIRICHLET 0
#define ORC_PERIODIC 1
#define ORC_RED 0   /* (i + j) even */
#define ORC_BLACK 1 /* (i + j) odd  */

#define ORC_DECLARE(SFX, REAL)                                                     \
  void orc_relax_##SFX(int n, int bc, REAL* u, const REAL* f, int colour);          \
  void orc_residual_##SFX(int n, int bc, const REAL* u, const REAL* f, REAL* r);   \
  void orc_restrict_##SFX(int n, int bc, const REAL* r, REAL* fc);                 \
  void orc_prolong_##SFX(int nc, int bc, const REAL* ec, REAL* ef);                \
  void orc_coarse_##SFX(int bc, const REAL* f, REAL* u);                           \
  void orc_vcycle_##SFX(int n, int bc, int nu1, int nu2, REAL* u, const REAL* f);    \
  void orc_restrict_factor_##SFX(int n, int F, const REAL* r, REAL* fc);             \
  void orc_prolong_factor_##SFX(int nc, int F, const REAL* ec, REAL* ef);            \
  void orc_twolevel_##SFX(int n, int F, int n_smooth, int coarse_sweeps, REAL* p,    \
                          const REAL* f);

ORC_DECLARE(f64, double)
ORC_DECLARE(f32, float)

/* FP64 direct solve on the 5x5 coarsest grid (both precisions call it). */
void orc_coarse_direct(int bc, const double* f, double* u);

double orc_norm2(int n, int bc, const double* a);
double orc_relres(int n, int bc, const double* u, const double* f);
int orc_solve_f64(int n, int bc, int nu1, int nu2, double* u, const double* f,
                  double rtol, int max_cycles, double* hist);
void orc_refine_step(int n, int bc, int nu1, int nu2, int inner, double* u, const double* f);
/* Two-level solve of the paper's controlled experiment: n_pre sweeps on the
 * initial grid p, then iterations of orc_twolevel_f64 until the change
 * ||p_i - p_(i-1)||_2 over the unique nodes is <= tol (Section 4.2's
 * criterion) or max_iter iterations; hist[k] = the change of iteration k+1
 * (max_iter entries).  Returns the iteration count. */
int orc_twolevel_solve(int n, int F, int n_smooth, int coarse_sweeps, int n_pre, double* p,
                       const double* f, double tol, int max_iter, double* hist);
int orc_solve_mixed(int n, int bc, int nu1, int nu2, int inner, double* u,
                    const double* f, double rtol, int max_steps, double* hist);

#endif
