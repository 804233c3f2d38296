// Internal declarations shared by the host runtime and the kernel launchers.
// Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mg {

constexpr int kDirichlet = 0;
constexpr int kPeriodic = 1;

// Half-width of the truncated spline prefilter (see spline_taps): the
// neglected weights sum to below the unit roundoff of FP64 (|z|^28 ~ 1e-16)
// and to ~1/300 of that of FP32 (|z|^18 ~ 2e-10).  Chunked recursions that
// start from a zero state K nodes out leave steps of that relative size at
// chunk edges, which the 5-point operator amplifies; at |z|^14 ~ 1e-8 they
// showed in FP32 residual norms.
constexpr int kPrefilterHalfTapsF64 = 28;
constexpr int kPrefilterHalfTapsF32 = 18;
constexpr int kMaxPrefilterTaps = 64;

// Levels with at most this many nodes per side run inside the single-
// workgroup tail kernel.
constexpr int kTailMaxSide = 65;

// Tap table of the B-spline prefilter for one level (see spline_taps).
struct PrefilterTaps {
  int count;   // number of taps
  int offset;  // tap t multiplies e_ext(i + t - offset)
  int period;  // period of the extended sequence (periodic: n-1, Dirichlet: 2(n-1))
  double w[kMaxPrefilterTaps];
};

// Records the detail string mg_last_error() returns on this thread, and
// returns `status` (for entry points defined outside the runtime unit).
int32_t set_last_error(int32_t status, const char* why);

// True for a grid side of the form 4 * 2^k + 1 in 5 .. 16385.
bool valid_side(int n);

// Builds the prefilter table for a level with `nc` nodes per side.
void spline_taps(int nc, int bc, int half_taps, PrefilterTaps* out);

// Inverse (Dirichlet, 9 x 9) or pseudo-inverse (periodic, 16 x 16) of the
// 5 x 5 level's operator, row-major, from its eigen-decomposition.
void coarsest_inverse(int bc, double* out /* 256 */);

// The prefilter of the tail sides 5, 9, 17 and 33 as dense nc x nc matrices
// (c = M e along one axis, every extension folded onto the stored nodes),
// stored after the coarsest inverse in the same device table.
constexpr int kTailMatOffset = 256;                  // doubles before the first matrix
constexpr int kTailMatElems = 25 + 81 + 289 + 1089;  // sides 5, 9, 17, 33
__host__ __device__ constexpr int tail_mat_offset(int nc) {
  return nc == 5 ? 0 : (nc == 9 ? 25 : (nc == 17 ? 106 : 395));
}
void prefilter_matrix(int nc, int bc, double* out /* nc * nc */);

// The caller's level-0 arrays of one problem, in device memory.  A
// captured step reads them from here (`ca` of the launchers below, when not
// null), so that one graph serves any u and f: the table is rewritten in
// stream order before a launch whose arrays differ from the last ones.
struct CallerArgs {
  double* u;
  const double* f;
};
hipError_t launch_bind_caller(hipStream_t s, CallerArgs* slot, double* u, const double* f);

// ---- launchers (mg_kernels.hip); all asynchronous on `s` -------------------
// Every array is a level array with `n` nodes per side and the given pitch.

template <typename T>
hipError_t launch_zero(hipStream_t s, int n, T* a, int pa);
// ca (FP64 only): a = ca->u.
template <typename T>
hipError_t launch_seam(hipStream_t s, int n, T* a, int pa, const CallerArgs* ca = nullptr);
template <typename T>
hipError_t launch_relax(hipStream_t s, int bc, int n, T* u, int pu, const T* f, int pf,
                        int colour, int count);
template <typename T>
hipError_t launch_residual(hipStream_t s, int bc, int n, const T* u, int pu, const T* f, int pf,
                           T* r, int pr);
template <typename T>
hipError_t launch_restrict(hipStream_t s, int bc, int n, const T* r, int pr, T* fc, int pfc);
// c = B-spline coefficients of e on a level with nc nodes; tmp is workspace
// of the same shape.
template <typename T>
hipError_t launch_prefilter(hipStream_t s, int bc, int nc, const PrefilterTaps& taps, const T* e,
                            int pe, T* tmp, int pt, T* c, int pc);
// Fine level with n nodes: u (+)= spline evaluated from coefficients c of
// the next coarser level.  add = false writes instead of adding.
template <typename T>
hipError_t launch_prolong(hipStream_t s, int bc, int n, T* u, int pu, const T* c, int pc, bool add);
template <typename T>
hipError_t launch_coarse(hipStream_t s, int bc, const T* f, int pf, T* u, int pu,
                         const double* inv);

// Mixed path, level 0: r32 = fl32(f - A u) computed in FP64, with per-block
// partial sums of r^2 (FP64) in partials[0 .. blocks).
// ca: u = ca->u, f = ca->f.
hipError_t launch_residual_mixed(hipStream_t s, int bc, int n, const double* u, int pu,
                                 const double* f, int pf, float* r32, int pr, double* partials,
                                 int* nblocks, const CallerArgs* ca = nullptr);
// u += e (FP64 += FP32) over the unknowns; ca: u = ca->u.
hipError_t launch_update_mixed(hipStream_t s, int bc, int n, double* u, int pu, const float* e,
                               int pe, const CallerArgs* ca = nullptr);
// Per-block partial sums of (f - A u)^2 and, if with_f, of f^2 (stored at
// partials[nblocks + b]).
hipError_t launch_resnorm(hipStream_t s, int bc, int n, const double* u, int pu, const double* f,
                          int pf, double* partials, bool with_f, int* nblocks);
// Per-block partial sums of f and f^2 for the RHS checks.
hipError_t launch_rhs_moments(hipStream_t s, int bc, int n, const double* f, int pf,
                              double* partials, int* nblocks);
// Per-block partial sums of (u - prev)^2 over the unknowns in
// partials[0 .. nblocks), and prev = u there.
hipError_t launch_diffnorm(hipStream_t s, int bc, int n, const double* u, int pu, double* prev,
                           int pp, double* partials, int* nblocks);
// Pressure-projection steps on a periodic n x n grid with seam, arrays of
// row pitch `pitch`: f = -div((u . grad) u), and (ox, oy) = u - dt ((u .
// grad) u - grad q) with q = -p the Poisson solve's solution for f
// (outputs distinct from the inputs).
template <typename T>
hipError_t launch_ns_rhs(hipStream_t s, int n, const T* ux, const T* uy, T* f, int pitch);
template <typename T>
hipError_t launch_ns_update(hipStream_t s, int n, const T* ux, const T* uy, const T* q, double dt,
                            T* ox, T* oy, int pitch);
// out[k] = sum of partials[k * stride + 0 .. count) for k < groups, in a
// fixed order (single workgroup per group).
hipError_t launch_reduce(hipStream_t s, const double* partials, int count, int stride, int groups,
                         double* out);
// Periodic: subtract mean (given on device as sum/(N^2)) from the unknowns
// and rewrite the seam.
hipError_t launch_remove_mean(hipStream_t s, int n, double* u, int pu, const double* sum);
hipError_t launch_sum(hipStream_t s, int bc, int n, const double* a, int pa, double* partials,
                      int* nblocks);

int blocks_for(int n, int bc);

// ---- fused launchers (mg_fused.hip) -----------------------------------------
// Sets the LDS limits of the tail kernels; call once per process/device.
hipError_t fused_init();
// Down pass of one level (n > kTailMaxSide): 2 red-black sweeps from uin
// (nullptr = zero guess) written to uout (must differ from uin), then
// fc = full weighting of f - A u on the next level.
// ca (FP64 level 0): uin = ca->u (when uin is not null), f = ca->f.
template <typename T>
hipError_t launch_down(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout, int puo,
                       const T* f, int pf, T* fc, int pfc, const CallerArgs* ca = nullptr);
// Up pass: uout = uin + P c (c = prefiltered coarse correction), then 2
// red-black sweeps.  uout must differ from uin.  pre: c is the coarse
// correction itself, prefiltered by each tile on its own support.
// ca (FP64 level 0): uout = ca->u, f = ca->f.
template <typename T>
hipError_t launch_up(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout, int puo,
                     const T* f, int pf, const T* c, int pc,
                     bool pre = false, const CallerArgs* ca = nullptr);
// Register-streaming versions of the two passes (mg_stream.hip); same
// contracts.  hs = rows per wavefront segment (even, 4..128; 0 = chosen per level).
template <typename T>
hipError_t launch_down_stream(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout,
                              int puo, const T* f, int pf, T* fc, int pfc, int hs,
                              const CallerArgs* ca = nullptr, double* partials = nullptr,
                              int nparts = 0, int* nitems = nullptr);
// partials (FP64, uin given): also one sum of r^2 per wavefront into
// partials[0 .. *nitems) for ||f - A uin||, the residual of the iterate the
// pass starts from; hipErrorInvalidValue when *nitems exceeds nparts.
// u64 (nullable): instead of writing uout, add the result to this FP64
// array (pitch p64) over the unknowns (the mixed path's refinement update);
// ca: u64 = ca->u (FP32 with u64), or uout = ca->u and f = ca->f (FP64).
template <typename T>
hipError_t launch_up_stream(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout, int puo,
                            const T* f, int pf, const T* c, int pc, int hs,
                            double* u64 = nullptr, int p64 = 0, const CallerArgs* ca = nullptr);
// c = spline coefficients of e (level with nc nodes), via tmp.
template <typename T>
hipError_t launch_prefilter_iir(hipStream_t s, int bc, int nc, const T* e, int pe, T* tmp, int pt,
                                T* c, int pc);
// Whole cycle from side nt (<= kTailMaxSide) down to 5 in one workgroup.
// uin: initial guess (nullptr = zero); uout (nullable): result; cout
// (nullable): prefiltered result; taps: device table for levels nt, .., 5.
// ca (FP64 level 0): uin and uout = ca->u where not null, f = ca->f.
template <typename T>
hipError_t launch_tail(hipStream_t s, int bc, int nt, const T* uin, int pui, T* uout, int puo,
                       const T* f, int pf, T* cout, int pco, const double* inv,
                       const PrefilterTaps* taps, const CallerArgs* ca = nullptr);

// ---- SR-CNN prolongation (mg_srcnn.hip) ------------------------------------
// Activations are bf16 (stored as unsigned short) in NHWC order with 64
// channels; N = unique nodes per side of the coarse level (a multiple of 32).
constexpr int kCnnBlocks = 8;
constexpr int kCnnWidth = 64;
constexpr int kCnnConvSet = 9 * kCnnWidth * kCnnWidth;  // bf16 values of one 64x64 conv
hipError_t cnn_init();  // LDS limits of the convolution kernels
int cnn_partials();     // floats of the max-abs partials buffer
// partials <- per-block max |e|; h = bf16(relu(stem(bf16(e / s)))) with
// s = max |e| also stored in scale[0].  stem_w: [64][9] floats.
template <typename T>
hipError_t launch_cnn_head(hipStream_t s, int N, const T* e, int pe, float* partials,
                           const float* stem_w, unsigned short* h, float* scale);
// mode 0: out = bf16(relu(conv(in))); 1: out = bf16(skip + conv(in)) (out
// may alias skip); 2: the 64 -> 256 conv followed by the x2 pixel shuffle and
// ReLU into out [2N][2N][64], w holding 4 sets (one per sub-pixel offset).
// w: [9 taps][64 out][64 in] bf16 per set.
hipError_t launch_cnn_conv(hipStream_t s, int mode, int N, const unsigned short* in,
                           const unsigned short* w, unsigned short* out, const unsigned short* skip);
// uout = uin (nullable: 0) + scale[0] * conv_fin(z) on the (2N+1)^2 fine grid,
// seam included.  fin_w: [9][64] floats.
template <typename T>
hipError_t launch_cnn_final(hipStream_t s, int N, const unsigned short* z, const float* fin_w,
                            const float* scale, const T* uin, int pui, T* uout, int puo);

// ---- persistent cycle kernel (mg_persist.hip) -------------------------------
constexpr int kMaxLevels = 13;   // 16385 -> 5
constexpr int kPersistThreads = 512;
constexpr int kRowsPerItem = 8;  // rows of an update item
constexpr int kResSegRows = 32;  // rows of a residual item (one band of columns)

// One level of one problem as the persistent kernel sees it.  Arrays are of
// the cycle's precision except where noted.
struct PLevel {
  void* u;    // final u of the level (level 0: the correction e, or the caller's u in FP64)
  void* f;    // right-hand side (level 0 in mixed: the FP32 residual)
  void* b;    // pre-smoothed u (written by the down pass, read by the up pass)
  void* c;    // spline coefficients of u (levels >= 1)
  void* tmp;  // x-filtered u (levels >= 1)
  int n, pitch;        // side; pitch of b, c, tmp (and of u, f above level 0)
  int pitch_u, pitch_f;  // pitches of u and f (differ at level 0 in FP64)
  int hs_down, nb_down, hs_up, nb_up;  // streaming-pass geometry
};

struct PProblem {
  int levels, tail, bc, active;
  double* u64;          // caller's FP64 u (mixed: refined in place)
  const double* f64;    // caller's FP64 f
  int pitch64, zero_guess;  // zero_guess: level-0 down pass starts from u = 0
  // Mixed path, level 0 above the tail: the level-0 down items (global item
  // indices nfirst .. nfirst + ncount) each write the sum of r^2 over the
  // unknowns they own to npart[item - nfirst].
  double* npart;
  int nfirst, ncount;
  PLevel lv[kMaxLevels];
};

enum PKind : int {
  kItemRes = 0,   // FP64 residual -> FP32 right-hand side (a = band, b = segment)
  kItemDown = 1,  // a = band, b = segment
  kItemTail = 2,  // workgroup item
  kItemPre = 3,   // workgroup item: prefilter tile a of b tiles along x
  kItemUp = 5,    // a = band, b = segment
  kItemUpd = 6    // u64 += e rows (a = first row)
};

struct PItem {
  int prob, level, a, b;
};

struct PPhase {
  int kind, first, count, pad;
};

struct PBarrier {
  unsigned count, gen, error, pad;
};

// One launch of phases [ph_begin, ph_end) of the list.  T = cycle
// precision.
template <typename T>
hipError_t launch_persistent(hipStream_t s, int bc, const PProblem* probs, const PPhase* phases,
                             int ph_begin, int ph_end, const PItem* items, PBarrier* bar,
                             const double* inv, int blocks, size_t lds);
// Per problem, the sum of the partials its level-0 down items wrote
// (PProblem::npart, the sum of r^2) into sums[b], in a fixed order; 0 for a
// problem without such items.
hipError_t launch_reduce_norms(hipStream_t s, const PProblem* probs, int nprob, double* sums);
// One phase of the table alone (its record passed by value), by a kernel
// that holds only the code of its kind; blocks of kPersistThreads threads,
// `lds` bytes of dynamic LDS (tail and prefilter phases).
template <typename T>
hipError_t launch_phase(hipStream_t s, int bc, const PPhase& phase, const PProblem* probs,
                        const PItem* items, const double* inv, int blocks, size_t lds);
// Wavefronts of the phase kernel of `kind` (kItemDown or kItemUp) that the
// current device holds at once.
template <typename T>
hipError_t phase_wave_slots(int bc, int kind, long* slots);
// Largest number of co-resident workgroups of the persistent kernel.
template <typename T>
hipError_t persistent_blocks(int bc, size_t lds, int* blocks);
hipError_t persistent_init(size_t lds64, size_t lds32);
// Batched helpers over a device problem table: per-problem partial sums of
// (f - A u)^2 and f^2 at level 0 (FP64), then their fixed-order reduction.
hipError_t launch_resnorm_batched(hipStream_t s, int bc, const PProblem* probs, int nprob,
                                  double* partials, int slots, double* sums);
hipError_t launch_seam_batched(hipStream_t s, const PProblem* probs, int nprob);
// Per-problem sums of f (use_u: of u) and of its square over the unknowns
// (sums[2 b], sums[2 b + 1]); zeros for inactive problems.
hipError_t launch_moments_batched(hipStream_t s, const PProblem* probs, int nprob,
                                  double* partials, int slots, double* sums, bool use_u);
// Active periodic problems: u minus its mean over the unknowns (sums[2 b] =
// the sum of u there), then the seams rewritten.
hipError_t launch_remove_mean_batched(hipStream_t s, const PProblem* probs, int nprob,
                                      const double* sums);
// Mixed path, level 0, from e = 0: the streaming down pass whose
// right-hand side r32 = fl32(f64 - A u64) it computes itself (and stores on
// the rows and columns it owns, for the up pass): no separate residual pass.
// ca: u64 = ca->u, f64 = ca->f.
hipError_t launch_down_res_stream(hipStream_t s, int bc, int n, const double* u64, int p64,
                                  const double* f64, int pf64, float* r32, int pr, float* uout,
                                  int puo, float* fc, int pfc, int hs,
                                  const CallerArgs* ca = nullptr, double* partials = nullptr,
                                  int nparts = 0, int* nitems = nullptr);
// uout == nullptr: the pre-smoothed iterate is not stored; the level's up
// pass must then be launch_up_pre_stream, which makes it again from r32.
// partials (with uout == nullptr): also one sum of r^2 per wavefront into
// partials[0 .. *nitems) and one of f64^2 into partials[*nitems .. 2
// *nitems), for ||f64 - A u64|| of the iterate the pass starts from and
// ||f64||; hipErrorInvalidValue when 2 *nitems exceeds nparts.
// Mixed path, level 0, after launch_down_res_stream without uout: the up
// pass that re-makes the pre-smoothed iterate from r32 (same values) and
// adds the result into u64.
// ca: u64 = ca->u.
hipError_t launch_up_pre_stream(hipStream_t s, int bc, int n, const float* f, int pf,
                                const float* c, int pc, int hs, double* u64, int p64,
                                const CallerArgs* ca = nullptr);
// Segment rows / band count of the streaming passes for a level.
int stream_segment_rows(int n, int bc, int owned_cols);
// Rows per segment at which every item of a streaming pass over a level is
// resident on the current device at once: the smallest even height whose
// item count fits the wave slots the kernel's occupancy allows (0: none up
// to the grid's extent).  A candidate for the autotuner.
enum StreamPass { kFitDown, kFitDownIn, kFitDownRes, kFitUp, kFitUpPre };
template <typename T>
int stream_fit_rows(StreamPass pass, int bc, int n);
int stream_down_owned();
int stream_up_owned();
int stream_res_owned();

}  // namespace mg
