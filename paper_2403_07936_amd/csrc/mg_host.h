// Host-side state of a multigrid context and the helpers that the runtime's
// translation units share: mg_runtime.hip (set-up, teardown, host math and
// the C ABI), mg_cycle.hip (cycles, solves and single steps), mg_batch.hip
// (the batch schedules) and mg_tune.hip (the autotuner).

#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mg.h"
#include "mg_internal.h"

namespace mg {

// --------------------------------------------------------------- context ----

template <typename T>
struct Hierarchy {
  // Level 0 holds only the scratch array r (and, in FP32, every array);
  // the FP64 level-0 u and f belong to the caller.
  std::vector<T*> u, f, r, c, tmp;
};

struct Problem {
  int n = 0, bc = 0, pitch0 = 0, levels = 0;
  std::vector<int> side, pitch;
  std::vector<PrefilterTaps> taps64, taps32;
  PrefilterTaps* taps64_dev = nullptr;  // device copies (read by the tail kernel)
  PrefilterTaps* taps32_dev = nullptr;
  int tail = 0;                         // first level handled by the tail kernel
  Hierarchy<double> h64;
  Hierarchy<float> h32;
  double* partials = nullptr;  // 2 * blocks_for(n) doubles
  double* sums = nullptr;      // 4 doubles of reduced results
  int nblocks = 0;
  // Hybrid prolongation schedule with a switch threshold: the previous
  // iterate (n x n, pitch n), and the last mg_solve's per-cycle record.
  double* uprev = nullptr;
  std::vector<int> hist_op;
  std::vector<double> hist_diff;
  // Captured step per variant (bit 0: SR-CNN prolongation, bit 1: mixed
  // step whose FP64 residual is already in place) and the caller arrays it
  // was captured with.
  hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  const double* graph_u[4] = {nullptr, nullptr, nullptr, nullptr};
  const double* graph_f[4] = {nullptr, nullptr, nullptr, nullptr};
  // Device slot of the caller's arrays read by captured steps that take
  // them from there, and the arrays last written to it.
  CallerArgs* caller = nullptr;
  double* bound_u = nullptr;
  const double* bound_f = nullptr;
  // Kernel choice per level (autotuned): variant 0 = register streaming with
  // `hs` rows per segment (0 = default), 1 = LDS tiles.
  std::vector<int> down_var, down_hs, up_var, up_hs;
};

struct TimingRec {
  int kind, level;
  double bytes;
  hipEvent_t a, b;
};

// State of the persistent schedule (one launch per step for the batch).
struct Persist {
  bool on = false;
  int bc = 0;
  std::vector<PProblem> h_probs;
  PProblem* d_probs = nullptr;
  bool dirty = true;
  PPhase* d_phases = nullptr;
  int nphases = 0;
  PItem* d_items = nullptr;
  PBarrier* d_bar = nullptr;
  int blocks = 0;
  size_t lds = 0;
  // Captured launches of the whole step, of its head and of its rest
  // (StepPart).
  hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
  // Mixed path with level 0 above the tail for every problem: the level-0
  // down items write each problem's norm partials (d_npart), so a
  // convergence check is the head of the next step, phases [0, head_end)
  // (every down phase), and the rest follows only for unconverged problems.
  bool split = false;
  int head_end = 0;
  double* d_npart = nullptr;
  double* d_nsums = nullptr;  // per problem: the sum of r^2
  // One launch per phase instead of one launch with device-wide barriers
  // (schedule 3): per phase, its kind, grid and dynamic LDS.
  bool phased = false;
  std::vector<PPhase> h_phases;
  size_t lds_tail = 0, lds_pre = 0;
  double* d_partials = nullptr;
  double* d_sums = nullptr;
  int slots = 32;
  // Algorithmic bytes of one launch (every problem active): the bytes each
  // pass of the step must read and write at its precision, as the
  // per-problem schedule counts them.
  double bytes = 0.0;
};

// SR-CNN prolongation state: weights (bf16 sets for the 64-channel convs,
// bf16-valued floats for the stem and the final conv) and activation
// buffers sized for the largest coarse level of the batch.
struct Cnn {
  bool on = false;   // weights loaded
  int levels = 0;    // finest prolongations that use the network in cycles
  unsigned short* w = nullptr;  // 2 * kCnnBlocks body sets, then 4 sub-pixel sets
  float* stem = nullptr;        // [64][9]
  float* fin = nullptr;         // [9][64]
  unsigned short *h = nullptr, *t = nullptr, *z = nullptr;
  float* partials = nullptr;
  float* scale = nullptr;
  int max_n = 0;  // largest coarse unique side the buffers hold
};

}  // namespace mg

struct mg_ctx_s {
  mg::Persist ps;
  mg::Cnn cnn;
  bool timing = false;
  std::vector<mg::TimingRec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t capture = nullptr;
  mg_options opt{};
  std::vector<mg::Problem> probs;
  double* inv[2] = {nullptr, nullptr};
  std::vector<void*> owned;
  double* host = nullptr;  // pinned host slots for norm readback
  int64_t graph_captures = 0, graph_instantiations = 0;
};

namespace mg {

// Records `why` as the thread's last-error detail and returns `status`.
int32_t fail(int32_t status, const std::string& why);

#define MG_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(MG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define MG_TRY(expr)                  \
  do {                                \
    int32_t st_ = (expr);             \
    if (st_ != MG_OK) return st_;     \
  } while (0)

inline hipEvent_t take_event(mg_ctx_s* ctx) {
  if (ctx->pool_used < ctx->pool.size()) return ctx->pool[ctx->pool_used++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  ctx->pool.push_back(e);
  ctx->pool_used++;
  return e;
}

// Runs `launch` (returning hipError_t); while timing is enabled and the work
// goes to the context's own stream, brackets it with a pair of events.
template <class Launch>
int32_t timed(mg_ctx_s* ctx, hipStream_t s, int kind, int level, double bytes, Launch&& launch) {
  if (!ctx->timing || s != ctx->stream) {
    MG_HIP(launch());
    return MG_OK;
  }
  hipEvent_t a = take_event(ctx), b = take_event(ctx);
  if (!a || !b) return fail(MG_ERR_HIP, "hipEventCreate failed");
  MG_HIP(hipEventRecord(a, s));
  MG_HIP(launch());
  MG_HIP(hipEventRecord(b, s));
  ctx->recs.push_back({kind, level, bytes, a, b});
  return MG_OK;
}

// Unknowns per side of a level (Dirichlet: the interior; periodic: the
// nodes without the seam).
inline double unknowns_side(int n, int bc) { return bc == kDirichlet ? n - 2 : n - 1; }

// Row pitch (elements) of the library's level arrays.
inline int pitch_for(int n) { return (n + 63) / 64 * 64; }

template <typename T>
int32_t alloc_level(mg_ctx_s* ctx, int n, int pitch, T** out) {
  void* p = nullptr;
  const size_t bytes = sizeof(T) * (size_t)n * pitch;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MG_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  ctx->owned.push_back(p);
  MG_HIP(hipMemsetAsync(p, 0, bytes, ctx->stream));
  *out = static_cast<T*>(p);
  return MG_OK;
}

template <typename T>
const Hierarchy<T>& hier(const Problem& p);
template <>
inline const Hierarchy<double>& hier<double>(const Problem& p) {
  return p.h64;
}
template <>
inline const Hierarchy<float>& hier<float>(const Problem& p) {
  return p.h32;
}

inline bool cnn_cycles(const mg_ctx_s* ctx) { return ctx->cnn.on && ctx->cnn.levels > 0; }

// ---- mg_cycle.hip
bool use_fused(const mg_ctx_s* ctx);
int32_t run_step(mg_ctx_s* ctx, Problem& p, double* u, const double* f, bool cnn = false,
                 bool have_res = false);
int32_t vcycle_impl(mg_ctx ctx, double* const* u, const double* const* f, int32_t ncycles,
                    double* relres_out);
int32_t solve_impl(mg_ctx ctx, double* const* u, const double* const* f, double rtol,
                   int32_t max_cycles, int32_t* cycles_out, double* relres_out);
// SR-CNN prolongation of a coarse correction ec (N x N unique nodes of a
// periodic level, pitch pec) onto fine level `level`: uout = uin + network
// output (uin nullable).
template <typename T>
int32_t enqueue_cnn(mg_ctx_s* ctx, hipStream_t s, int level, int N, const T* ec, int pec,
                    const T* uin, int pui, T* uout, int puo);

// ---- mg_batch.hip
bool persistent_eligible(const mg_ctx_s* ctx, std::string* why);
template <typename T>
int32_t build_persistent(mg_ctx_s* ctx);
int32_t persistent_bind(mg_ctx_s* ctx, double* const* u, const double* const* f,
                        const std::vector<int>& active);
// Which part of a step a launch queues: all of it, its head (the phases
// up to the tail: for a split step, the level-0 down passes that make the
// FP64 residual and its norms, the iterate untouched) or the rest.
enum StepPart { kWhole = 0, kHead = 1, kRest = 2 };
int32_t persistent_launch(mg_ctx_s* ctx, StepPart part = kWhole);
// Split batches: the head of a step for the bound active problems, and
// each problem's sum of r^2 (B doubles) read back (synchronises).
int32_t persistent_head(mg_ctx_s* ctx, double* sums);
void persistent_drop_graphs(Persist& P);
int32_t persistent_check(mg_ctx_s* ctx);
int32_t persistent_relres(mg_ctx_s* ctx, double* rel);

// ---- mg_tune.hip
int32_t autotune(mg_ctx_s* ctx);
int32_t tune_schedule(mg_ctx_s* ctx);

}  // namespace mg
