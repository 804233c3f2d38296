/*
 * mg.h -- C ABI of the MI355X (gfx950) geometric-multigrid library for the
 * 2-D Poisson equation.
 *
 * What is solved.  The paper solves the pressure-Poisson equation
 * "Laplacian p = f" (Section 2.2, the Poisson equation; Section 2.5 for the
 * pressure source) with a geometric multigrid V-cycle (Section 2.2; appendix,
 * algorithm "Multigrid algorithm with V-Cycle structure").  This library
 * solves A u = f with A = -Delta_h, the 5-point negative Laplacian, which is
 * symmetric positive (semi-)definite; the paper's p is -u.
 *
 * Grids.  A grid has n nodes per side on the unit square, n - 1 = 4 * 2^k
 * (n = 5, 9, 17, 33, 65, 129, ...), spacing h = 1/(n-1).  Arrays are row
 * major with a row pitch given in elements: element (i, j) of a grid stored
 * at `a` with pitch p is a[i * p + j], i the y index, j the x index.
 *   MG_BC_DIRICHLET0: zero boundary values.  Unknowns are 1 <= i, j <= n-2;
 *     boundary entries of u must hold 0 and are never written.
 *   MG_BC_PERIODIC: the unit torus.  Unknowns are 0 <= i, j <= n-2; row and
 *     column n-1 duplicate row and column 0 (the "seam").  The seam of an
 *     input is ignored; the seam of an output is rewritten from node 0.
 *     f must have (numerically) zero mean.
 * The hierarchy halves the spacing down to n = 5 (level 0 is the finest).
 *
 * The V(nu_pre, nu_post) cycle, per level: nu_pre red-black Gauss-Seidel
 * sweeps (red = (i+j) even first), residual r = f - A u, full-weighting
 * restriction of r to the next coarser level, recursion from a zero guess,
 * correction u += P u_c with P the tensor-product interpolating cubic spline
 * (natural for Dirichlet, periodic for periodic grids), nu_post sweeps.  The
 * 5 x 5 level is solved directly (Dirichlet: inverse of the 9 x 9 system;
 * periodic: pseudo-inverse of the 16 x 16 system, zero-mean result).
 *
 * Precision.  MG_FP64 runs every step in FP64.  MG_MIXED runs FP64
 * iterative refinement around FP32 cycles: r = f - A u in FP64 (stored as
 * FP32), `inner_cycles` FP32 V-cycles on A e = r from e = 0 with the 5 x 5
 * solve in FP64, then u += e in FP64.
 *
 * Memory and streams.  All array arguments of the solve calls are DEVICE
 * pointers (hipMalloc'd or torch-allocated on the current device), FP64,
 * owned by the caller; the library never keeps them past a call.  The
 * library owns every workspace it allocates in mg_setup and frees it in
 * mg_destroy.  Work is queued on the HIP stream given to mg_setup (NULL =
 * the default stream) and is asynchronous unless a call says it
 * synchronises.  A context is not thread-safe; distinct contexts are
 * independent.
 *
 * Errors.  Every function returns an mg_status and never aborts or throws
 * across the ABI.  mg_last_error() gives a thread-local detail string for
 * the last failing call on this thread.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Exported from the shared library (which hides everything else). */
#define MG_API __attribute__((visibility("default")))

typedef struct mg_ctx_s* mg_ctx;

typedef enum {
  MG_OK = 0,
  MG_ERR_INVALID_ARG = -1,      /* bad size, NULL pointer, out-of-range index */
  MG_ERR_UNSUPPORTED = -2,      /* valid but not provided (e.g. SR-CNN on Dirichlet) */
  MG_ERR_OOM = -3,              /* device allocation failed */
  MG_ERR_HIP = -4,              /* a HIP runtime call failed; see mg_last_error() */
  MG_ERR_INCOMPATIBLE_RHS = -5, /* periodic f with |sum f| > 1e-10 * N * rms(f) */
  MG_ERR_NOT_CONVERGED = -6,    /* max_cycles reached above rtol (u is valid) */
  MG_ERR_STAGNATED = -7,        /* residual stopped decreasing above rtol (u is valid) */
  MG_ERR_NONFINITE = -8         /* NaN or Inf in the residual norm (u may be garbage) */
} mg_status;

enum { MG_BC_DIRICHLET0 = 0, MG_BC_PERIODIC = 1 };
enum { MG_FP64 = 0, MG_MIXED = 1 };
enum { MG_PROLONG_SPLINE = 0, MG_PROLONG_SRCNN = 1 };
enum { MG_DT_F64 = 0, MG_DT_F32 = 1 };

/* One problem: n nodes per side, boundary condition, row pitch of the
 * caller's level-0 arrays in elements (0 means n). */
typedef struct {
  int32_t n;
  int32_t bc;
  int32_t pitch;
} mg_grid;

/* Solver options (parameter set of the paper's Table 1, reduced to what this
 * cycle uses).  Fill with mg_options_default() and override fields. */
typedef struct {
  int32_t precision;          /* MG_FP64 (default) or MG_MIXED */
  int32_t nu_pre, nu_post;    /* red-black sweeps before / after the correction (2, 2) */
  int32_t inner_cycles;       /* MG_MIXED: FP32 cycles per refinement step (1) */
  int32_t prolong;            /* MG_PROLONG_SPLINE (default) or MG_PROLONG_SRCNN */
  int32_t cnn_levels;         /* SR-CNN on this many finest prolongations (2) */
  const void* cnn_weights;    /* host blob of SR-CNN weights, copied at setup:
                                 MG_SRCNN_WEIGHT_COUNT float32 values (see below) */
  size_t cnn_weights_bytes;   /* 4 * MG_SRCNN_WEIGHT_COUNT */
  int32_t check_every;        /* mg_solve: cycles between norm checks; 0 = auto */
  int32_t use_graph;          /* capture each cycle into a hipGraph (1) */
  const char* tune_cache_path; /* autotuner cache file; NULL = built-in choices */
  int32_t kernel_path;        /* 0: fused register-streaming passes (default);
                                 1: one launch per operation (reference schedule);
                                 2: fused LDS-tiled passes.  Same arithmetic. */
  int32_t schedule;           /* 0: auto (autotuned at setup, cached in tune_cache_path);
                                 1: per problem, one graph of per-level kernels per cycle;
                                 2: one persistent launch per cycle for the whole batch
                                 (all problems must share the boundary condition; needs
                                 kernel_path 0, nu_pre = nu_post = 2, inner_cycles = 1);
                                 3: as 2, but one launch per phase of the cycle (per level
                                 and pass, over every problem), each kernel holding only
                                 its phase's code; no device-wide barrier. */
  double cnn_max_ratio;       /* mg_solve with SR-CNN: after a network-prolongated cycle whose
                                 residual ratio exceeds this (0.5), use the spline from then on */
  double cnn_min_relres;      /* ... and likewise once the relative residual is <= this (1e-7) */
  double n_gan;               /* mg_solve with SR-CNN: the hybrid schedule of Table 1 and the
                                 appendix's V-CYCLE in place of the rule above.  0 (default):
                                 off.  >= 1: N = round(n_gan) network prolongations, then one
                                 spline one; in (0, 1): N = round(1 / n_gan) spline ones, then
                                 one network one (cycle i = 1, 2, ... of the call takes the
                                 second operator when i is a multiple of N + 1). */
  double s_thres;             /* with n_gan: once a cycle changes u by at most this,
                                 ||u_i - u_(i-1)||_2 over the unknowns, the next cycle takes
                                 the second operator (Section 4); 0 (default): never. */
} mg_options;

/* SR-CNN weights (Section 3.1, generator after Ledig et al.; no biases):
 * float32, PyTorch (out, in, ky, kx) order, concatenated as
 *   stem 64x1x3x3, then for each of 8 residual blocks conv1 64x64x3x3 and
 *   conv2 64x64x3x3, then 256x64x3x3 (followed by the x2 pixel shuffle:
 *   channel 4c + 2a + b -> channel c at fine offset (a, b)), then 1x64x3x3.
 * The library rounds them to bfloat16 (nearest even) at setup. */
#define MG_SRCNN_WEIGHT_COUNT 738432

/* Fill *opt with the defaults listed above.  No-op on NULL. */
MG_API void mg_options_default(mg_options* opt);

/* Create a context for `batch` problems grids[0..batch-1] (host array).
 * The multigrid parameters of Table 1 map to it as follows: the grid side
 * N_grid is grids[b].n; the hierarchy halves the side per level (N_step =
 * 1) down to the coarsest side r_min = 5, solved directly; the sweeps per
 * level are nu_pre and nu_post (N_smooth); N_GAN and S_thres are n_gan
 * and s_thres of the options.
 * Allocates every device workspace (per problem: the coarse levels of the
 * hierarchy, and for MG_MIXED the FP32 hierarchy including level 0) and the
 * 5 x 5 inverses, computed in FP64 on the host.  hip_stream is a
 * hipStream_t (NULL = default stream) used by every later call.
 * Errors: INVALID_ARG (NULL out/grids/opt, batch <= 0, n not 4*2^k+1,
 * pitch < n, bad enum, nu_pre/nu_post outside 0..8, inner_cycles outside
 * 1..8, SR-CNN weights of the wrong size), UNSUPPORTED (SR-CNN requested
 * without weights, on Dirichlet grids, or with a network level whose coarse
 * side is below 129), OOM, HIP.  On error *out is set to NULL and nothing is leaked. */
MG_API int32_t mg_setup(const mg_grid* grids, int32_t batch, const mg_options* opt,
                 void* hip_stream, mg_ctx* out);

/* Run `ncycles` cycles (MG_FP64: V-cycles; MG_MIXED: refinement steps) on
 * every problem of the batch.  u[b], f[b] (host arrays of device pointers)
 * are FP64 level-0 arrays with the pitch given at setup; u[b] is both the
 * initial guess and the result (in place), f[b] is read only.  The
 * appendix's V-CYCLE(p, r) is one call with ncycles = 1.  If relres_out is
 * not NULL (host array [batch]) the call synchronises and writes
 * ||f - A u||_2 / ||f||_2 over the unknowns after the last cycle; otherwise
 * it returns after queueing.  Periodic seams of u are rewritten.  With
 * MG_PROLONG_SRCNN every cycle uses the network on the cnn_levels finest
 * prolongations.  On the persistent schedule (option `schedule`) the call
 * always synchronises before it returns, to read the device-wide barrier's
 * status: a barrier that timed out makes the call return MG_ERR_HIP (u is
 * then partly updated).
 * Errors: INVALID_ARG (NULL ctx/u/f or entries, ncycles < 0), HIP,
 * NONFINITE (only when relres_out is given). */
MG_API int32_t mg_vcycle(mg_ctx ctx, double* const* u, const double* const* f, int32_t ncycles,
                  double* relres_out);

/* Iterate cycles from the given u until ||f - A u|| / ||f|| <= rtol
 * (the paper iterates to a tolerance, Section 4.2).  Norms are checked every
 * check_every cycles (auto: after the first cycle, then at predicted
 * crossings).  Synchronises at every check.  When the level-0 down pass
 * streams (and, mixed, with one inner cycle and a streaming level-0 up
 * pass; no network), a check of a single-problem context is the next step's
 * level-0 down pass, which measures the residual of the iterate it reads
 * and leaves it unchanged, and the rest of that step runs only if the
 * problem goes on (mixed batches likewise, with every down phase).  On exit periodic u has zero mean and a rewritten seam; its
 * relative residual is the one measured before that mean was removed (the
 * same up to rounding: constants are the null space of A).  cycles_out / relres_out (host arrays [batch],
 * may be NULL) receive per-problem cycle counts and final relative residuals.
 * Returns OK when every problem converged, else the first failure among
 * NOT_CONVERGED (max_cycles hit), STAGNATED (ratio > 0.9 over 3 checks),
 * NONFINITE, INCOMPATIBLE_RHS (periodic f with nonzero mean; nothing run).
 * Problems that converge stop cycling while others continue.  With
 * MG_PROLONG_SRCNN each problem starts with network-prolongated cycles,
 * checked after every cycle, and falls back to the spline for the rest of
 * the solve after a cycle whose residual ratio exceeds cnn_max_ratio or
 * once the relative residual is <= cnn_min_relres (a minimal form of the
 * paper's switching threshold S_thres); with n_gan > 0 the choice per cycle
 * follows the hybrid schedule instead (N_GAN and S_thres, Table 1 and the
 * appendix's V-CYCLE), and with s_thres > 0 every cycle is checked. */
MG_API int32_t mg_solve(mg_ctx ctx, double* const* u, const double* const* f, double rtol,
                 int32_t max_cycles, int32_t* cycles_out, double* relres_out);

/* Per-cycle record of the last mg_solve for problem `problem`: prolong_out[k]
 * (MG_PROLONG_SPLINE or MG_PROLONG_SRCNN) is the prolongation cycle k + 1
 * used, diff_out[k] the change it made, ||u_(k+1) - u_k||_2 over the
 * unknowns, when the hybrid schedule tracks it (n_gan > 0 and s_thres > 0),
 * else NaN.  At most `cap` entries are written (either output may be NULL);
 * *count_out receives the number of cycles.  Host only, no device work.
 * Errors: INVALID_ARG (NULL ctx or count_out, bad problem, cap < 0). */
MG_API int32_t mg_solve_history(mg_ctx ctx, int32_t problem, int32_t cap, int32_t* prolong_out,
                         double* diff_out, int32_t* count_out);

/* Prolongation operator on its own (the appendix's SR-Prolongation and the
 * spline prolongation of Section 2.2): fine = P coarse for problem
 * `problem`, from level `coarse_level` (>= 1) to level coarse_level - 1.
 * coarse and fine are device arrays of that problem's level sides, pitch =
 * side, dtype MG_DT_F64 or MG_DT_F32.  kind MG_PROLONG_SPLINE interpolates
 * with the cubic spline; MG_PROLONG_SRCNN applies the SR-CNN (the coarse
 * unique side nc - 1 must be a multiple of 32, at least 32).  The result
 * is written, not added; periodic seams are written.  Asynchronous.
 * Errors: INVALID_ARG, UNSUPPORTED (SRCNN without weights at setup, or a
 * coarse side the network kernels do not tile), HIP. */
MG_API int32_t mg_prolong(mg_ctx ctx, int32_t problem, int32_t coarse_level, int32_t kind,
                   const void* coarse, void* fine, int32_t dtype);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * spline prolongation of mg_prolong (kind MG_PROLONG_SPLINE), same kernels
 * and bitwise the same result, with no context.  fine = P coarse from a grid
 * of nc nodes per side (nc - 1 = 4 * 2^k, 5 <= nc <= 1025) to the grid of
 * 2 nc - 1; coarse and fine are caller-owned device arrays of the current
 * device, pitch = side, dtype MG_DT_F64 or MG_DT_F32; bc as in mg_grid.
 * The result is written, not added; periodic seams are written.
 * Asynchronous on hip_stream (NULL: the null stream), which must belong to
 * the current device.  Its scratch (the prefilter's intermediate and the
 * B-spline coefficients, 16.8 MB) is a static device array, one per GPU,
 * held until the process ends; the call allocates nothing, and its first
 * call on a device looks that array's address up once.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race.
 * Errors: INVALID_ARG (bad nc, bc or dtype, NULL or aliased arrays),
 * UNSUPPORTED (nc above 1025), HIP. */
MG_API int32_t mg_prolong_noalloc(int32_t nc, int32_t bc, const void* coarse, void* fine,
                                  int32_t dtype, void* hip_stream);

/* The steps either side of the pressure solve in a time step of the
 * incompressible flow (Section 2.1's momentum system; Section 2.3's source
 * with zero viscosity), on one periodic n x n grid with the duplicated seam
 * (n - 1 = 4 * 2^k, 5 <= n <= 16385; spacing h = 1/(n-1); x along the
 * columns, y along the rows).  Every derivative is the second-order central
 * difference of the nodal values, (a[j+1] - a[j-1]) / (2h).
 *   mg_ns_rhs:    f = -div((u . grad) u), the source of the pressure-Poisson
 *                 equation Laplacian p = f (mean zero up to rounding); seam
 *                 written.
 *   mg_ns_update: (ux_out, uy_out) = u - dt ((u . grad) u + grad p), one
 *                 explicit Euler step of the momentum equation; seams
 *                 written.  The pressure is passed as q, the solution that
 *                 mg_solve returns for the source f of mg_ns_rhs: mg_solve
 *                 solves -Laplacian_h q = f, so q = -p, and the step is
 *                 evaluated as u - dt ((u . grad) u - grad q).  A time step
 *                 is therefore mg_ns_rhs -> mg_solve -> mg_ns_update with
 *                 the solver's output handed over unchanged.  The outputs
 *                 must not alias the inputs or each other.
 * All arrays are device arrays of dtype MG_DT_F64 or MG_DT_F32 with row
 * pitch `pitch` (>= n) elements, owned by the caller; only the unique nodes
 * of the inputs are read.  Asynchronous on hip_stream (NULL: the null
 * stream); no context needed.  Errors: INVALID_ARG (bad n, pitch or dtype,
 * NULL or aliased arrays, non-finite dt), HIP. */
MG_API int32_t mg_ns_rhs(int32_t n, const void* ux, const void* uy, void* f, int32_t pitch,
                  int32_t dtype, void* hip_stream);
MG_API int32_t mg_ns_update(int32_t n, const void* ux, const void* uy, const void* q, double dt,
                     void* ux_out, void* uy_out, int32_t pitch, int32_t dtype,
                     void* hip_stream);

/* Single steps of the cycle on caller arrays, for operator-level checks.
 * Arrays are device arrays of level `level` of problem `problem`, pitch =
 * side, in dtype MG_DT_F64 or MG_DT_F32.  All are asynchronous.
 *   mg_relax:        `count` red-black half-sweeps starting with `colour`
 *                    (0 red, 1 black), alternating (Section 2.2: Gauss-Seidel).
 *   mg_residual:     r = f - A u (appendix V-cycle), zero on Dirichlet
 *                    boundary nodes, seam written.
 *   mg_restrict:     fc = full weighting of r onto level + 1.
 *   mg_coarse_solve: u = direct solution on the 5 x 5 level (FP64 inside).
 * Errors: INVALID_ARG (bad indices or NULL), HIP. */
MG_API int32_t mg_relax(mg_ctx ctx, int32_t problem, int32_t level, void* u, const void* f,
                 int32_t colour, int32_t count, int32_t dtype);
MG_API int32_t mg_residual(mg_ctx ctx, int32_t problem, int32_t level, const void* u, const void* f,
                    void* r, int32_t dtype);
MG_API int32_t mg_restrict(mg_ctx ctx, int32_t problem, int32_t level, const void* r, void* fc,
                    int32_t dtype);
MG_API int32_t mg_coarse_solve(mg_ctx ctx, int32_t problem, const void* f, void* u, int32_t dtype);

/* The paper's controlled two-level experiment (Section 4.1: a 192 x 192
 * periodic grid coarsened directly to 12 x 12, N_step = 4 and r_min = 12 in
 * Table 1; the appendix's V-CYCLE with one coarse level, which is relaxed 10
 * times rather than solved), for a batch of problems.  One iteration:
 * n_smooth red-black Gauss-Seidel sweeps (red = (i+j) even first) on
 * A p = f, r = f - A p, r_c = R r with R the tensor product of the 1-D
 * weights (F - |a|) / F^2, |a| < F (full weighting widened to the factor F;
 * the paper names no weights), coarse_sweeps red-black sweeps from d_c = 0 on
 * the 5-point system of spacing F h, then p += P d_c with P the periodic
 * tensor cubic spline (Section 2.2) by the factor F.  There is no
 * post-smoothing: the paper relaxes at the start of each iteration.
 * Grids: N = n_unique nodes per side on the unit torus (h = 1/N), stored
 * with the seam as (N+1) x (N+1); p and f are device arrays of `batch`
 * such grids back to back ([batch][N+1][N+1], FP64), owned by the caller;
 * p is updated in place (seams rewritten), f must have zero mean.  One
 * workgroup runs each problem, the whole solve in one launch.
 *   mg_twolevel_setup: N in {64, 128, 192}; factor F = 2^N_step in
 *     {4, 8, 16, 32} with N/F even (the coarse side r_min = N/F); n_smooth
 *     and coarse_sweeps in 0..1000 (the paper: 20 and 10).  Allocates the
 *     workspaces (packed h^2 f, the smoothed iterate and the residual: 3
 *     arrays of batch N^2 doubles).  Errors: INVALID_ARG, UNSUPPORTED (N),
 *     OOM, HIP.
 *   mg_twolevel_smooth: `sweeps` red-black sweeps on every problem (the
 *     paper's N_smooth,pre sweeps on the initial random grid).  Asynchronous.
 *   mg_twolevel_cycle: `ncycles` iterations on every problem; with
 *     change_out (host [batch]) the call synchronises and writes the last
 *     iteration's ||p_i - p_(i-1)||_2 over the unique nodes, else it is
 *     asynchronous.  NONFINITE if a change is NaN or infinite.
 *   mg_twolevel_solve: n_pre sweeps, then iterations until a problem's change
 *     is <= tol (the paper's stopping rule, Section 4.2) or max_iter; each
 *     problem stops on its own, on the device.  Synchronises once at the
 *     end; iters_out / change_out (host [batch], may be NULL) receive the
 *     iteration count and the last change.  Returns OK when every problem
 *     converged, else NOT_CONVERGED or NONFINITE (outputs filled).
 *   mg_twolevel_destroy: frees the context (NULL accepted).
 * A context is not thread-safe.  Errors of the run calls: INVALID_ARG (NULL
 * context or arrays, p == f, negative counts, tol not >= 0), HIP. */
typedef struct mg_twolevel_s* mg_twolevel;
MG_API int32_t mg_twolevel_setup(int32_t n_unique, int32_t factor, int32_t batch,
                                 int32_t n_smooth, int32_t coarse_sweeps, void* hip_stream,
                                 mg_twolevel* out);
MG_API int32_t mg_twolevel_smooth(mg_twolevel ctx, double* p, const double* f, int32_t sweeps);
MG_API int32_t mg_twolevel_cycle(mg_twolevel ctx, double* p, const double* f, int32_t ncycles,
                                 double* change_out);
MG_API int32_t mg_twolevel_solve(mg_twolevel ctx, double* p, const double* f, int32_t n_pre,
                                 double tol, int32_t max_iter, int32_t* iters_out,
                                 double* change_out);
MG_API int32_t mg_twolevel_destroy(mg_twolevel ctx);

/* Kernel classes for the timing diagnostics below. */
enum {
  MG_K_RELAX = 0,          /* one red-black half-sweep */
  MG_K_RESIDUAL = 1,       /* r = f - A u */
  MG_K_RESTRICT = 2,       /* full weighting */
  MG_K_PREFILTER = 3,      /* spline coefficients (both axes) */
  MG_K_PROLONG = 4,        /* spline evaluation and correction */
  MG_K_COARSE = 5,         /* 5 x 5 direct solve */
  MG_K_RESIDUAL_MIXED = 6, /* FP64 residual stored as FP32 */
  MG_K_UPDATE_MIXED = 7,   /* u += e */
  MG_K_RESNORM = 8,        /* residual norm partial sums */
  MG_K_ZERO = 9,           /* zero fill */
  MG_K_DOWN = 10,          /* fused: 2 sweeps + residual + restriction */
  MG_K_UP = 11,            /* fused: spline correction + 2 sweeps */
  MG_K_TAIL = 12,          /* fused: all levels <= 65 x 65 in one workgroup */
  MG_K_PERSISTENT = 13,    /* persistent schedule: one whole step of the batch */
  MG_K_CNN = 14,           /* SR-CNN 64-channel convolutions (matrix cores) */
  MG_K_CNN_AUX = 15,       /* SR-CNN scale, stem and final convolution */
  MG_K_PHASED = 16,        /* phased schedule: one whole step of the batch, a launch per phase */
  MG_K_COUNT = 17
};

/* Diagnostics: while enabled, cycles run without graph capture and every
 * kernel launch is bracketed by HIP events on the context's stream.
 * Enabling clears earlier records.  Errors: INVALID_ARG, HIP. */
MG_API int32_t mg_timing_enable(mg_ctx ctx, int32_t enable);

/* Totals over the launches recorded since timing was enabled, for kernel
 * class `kind` on level `level` (-1 = all levels): number of launches,
 * summed event time in milliseconds and summed algorithmic bytes (the bytes
 * the operation must read and write at its arithmetic precision, counted
 * once per array element).  Synchronises the context's stream.
 * Errors: INVALID_ARG, HIP. */
MG_API int32_t mg_timing_read(mg_ctx ctx, int32_t kind, int32_t level, int64_t* launches,
                              double* total_ms, double* bytes);

/* Static name of a kernel class ("?" if unknown). */
MG_API const char* mg_kernel_name(int32_t kind);

/* Diagnostics: how many times the context has captured a step into a
 * hipGraph and instantiated one (all problems, since setup).  With the
 * default kernels (nu_pre = nu_post = 2, kernel_path not per-operation, no
 * SR-CNN prolongation) a step's graph reads u[b] and f[b] from a device
 * slot of the problem that each call rewrites when the arrays differ from
 * the last call's, so calls on new arrays reuse the graph; the other
 * configurations capture the step again when its arrays change.  Either
 * output may be NULL.  Errors: INVALID_ARG (NULL ctx). */
MG_API int32_t mg_graph_stats(mg_ctx ctx, int64_t* captures, int64_t* instantiations);

/* Diagnostics for callers' error handling: marks the persistent schedule's
 * device-wide barrier as timed out, exactly as a barrier that waited past
 * its spin limit does.  The next persistent launch then exits at entry
 * without touching any array, and the mg_vcycle or mg_solve call that
 * queued it returns MG_ERR_HIP and clears the mark.  Synchronises the
 * context's stream.  Errors: INVALID_ARG (NULL ctx), UNSUPPORTED (the
 * context does not run the persistent schedule, or runs it as one launch
 * per phase: schedule 3 has no device-wide barrier), HIP. */
MG_API int32_t mg_persistent_mark_timeout(mg_ctx ctx);

/* Number of levels of problem `problem` (>= 1), or a negative mg_status. */
MG_API int32_t mg_num_levels(mg_ctx ctx, int32_t problem);

/* Free every device and host resource of the context (waits for its stream).
 * NULL is accepted. */
MG_API int32_t mg_destroy(mg_ctx ctx);

/* Static description of a status code (never NULL). */
MG_API const char* mg_status_string(int32_t status);

/* Thread-local detail of the last error on this thread ("" if none). */
MG_API const char* mg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MG_H */
