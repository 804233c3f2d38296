// Host runtime and C ABI of the multigrid library (declared in include/mg.h).
//
// A context owns, per problem, the grid hierarchy down to 5 x 5, the
// per-level work arrays, the prefilter tables and, optionally, hipGraphs of
// one cycle.  The caller owns the finest-level u and f.

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
#include "mg_tail_dev.h"

namespace mg {

// ------------------------------------------------------------ host math ----

// Inverse of S = (1, 4, 1)/6 on a periodic sequence of period Q (Dirichlet
// grids use the odd extension of period 2(nc-1), periodic grids period
// nc-1).  With z = sqrt(3) - 2 the bi-infinite inverse is sqrt(3) z^|k|;
// folded onto one period it is
//   c_i = sqrt(3) / (1 - z^Q) * sum_{m=0}^{Q-1} (z^m + z^(Q-m)) e_{i+m}.
// When Q <= 2 * half_taps + 1 the whole period is used (exact); otherwise
// the taps |k| <= half_taps are kept, whose neglected tail is below the
// unit roundoff of the working precision.
void spline_taps(int nc, int bc, int half_taps, PrefilterTaps* out) {
  const int Q = bc == kPeriodic ? nc - 1 : 2 * (nc - 1);
  const double z = std::sqrt(3.0) - 2.0;
  auto zpow = [&](int m) {
    double p = 1.0;
    for (int k = 0; k < m; ++k) p *= z;
    return p;
  };
  const double zq = zpow(Q);
  auto G = [&](int m) { return std::sqrt(3.0) * (zpow(m) + zpow(Q - m)) / (1.0 - zq); };
  out->period = Q;
  if (Q <= 2 * half_taps + 1) {
    out->count = Q;
    out->offset = 0;
    for (int t = 0; t < Q; ++t) out->w[t] = G(t);
  } else {
    out->count = 2 * half_taps + 1;
    out->offset = half_taps;
    for (int t = 0; t < out->count; ++t) {
      const int m = ((t - half_taps) % Q + Q) % Q;
      out->w[t] = G(m);
    }
  }
}

// The period is at most 64 nodes for nc <= 33, so the table of spline_taps
// holds the whole period and M is the exact inverse: M[q][k] sums the taps
// w[t] whose extended node q + t is stored node k (with the odd extension's
// sign).  Dirichlet rows 0 and nc-1 (boundary coefficients) are 0; the
// periodic seam row repeats row 0.
void prefilter_matrix(int nc, int bc, double* out) {
  PrefilterTaps tp;
  spline_taps(nc, bc, kMaxPrefilterTaps / 2, &tp);
  const int Q = tp.period;
  for (int i = 0; i < nc * nc; ++i) out[i] = 0.0;
  for (int q = 0; q < nc; ++q) {
    if (bc == kDirichlet && (q == 0 || q == nc - 1)) continue;
    for (int t = 0; t < tp.count; ++t) {
      const int x = ((q + t - tp.offset) % Q + Q) % Q;
      int node = x;
      double sign = 1.0;
      if (bc == kDirichlet && x > nc - 1) {
        node = Q - x;
        sign = -1.0;
      }
      out[q * nc + node] += sign * tp.w[t];
    }
  }
  if (bc == kPeriodic)
    for (int k = 0; k < nc; ++k) out[(nc - 1) * nc + k] = out[k];
}

// 5 x 5 level (h = 1/4) from the eigen-decomposition of the 5-point operator.
// Dirichlet: orthonormal sine vectors phi_a(i) = sqrt(1/2) sin(a pi i / 4),
// eigenvalues 64 (sin^2(a pi/8) + sin^2(b pi/8)).  Periodic: Fourier modes
// on the 4 x 4 torus, eigenvalues 64 (sin^2(pi k/4) + sin^2(pi l/4)); the
// zero mode is dropped, which gives the pseudo-inverse.
void coarsest_inverse(int bc, double* out) {
  const double pi = 3.14159265358979323846;
  std::memset(out, 0, sizeof(double) * 256);
  if (bc == kDirichlet) {
    double phi[4][4];
    for (int a = 1; a <= 3; ++a)
      for (int i = 1; i <= 3; ++i) phi[a][i] = std::sqrt(0.5) * std::sin(a * pi * i / 4.0);
    for (int i = 1; i <= 3; ++i)
      for (int j = 1; j <= 3; ++j)
        for (int ii = 1; ii <= 3; ++ii)
          for (int jj = 1; jj <= 3; ++jj) {
            double s = 0.0;
            for (int a = 1; a <= 3; ++a)
              for (int b = 1; b <= 3; ++b) {
                const double sa = std::sin(a * pi / 8.0), sb = std::sin(b * pi / 8.0);
                const double lam = 64.0 * (sa * sa + sb * sb);
                s += phi[a][i] * phi[b][j] * phi[a][ii] * phi[b][jj] / lam;
              }
            out[((i - 1) * 3 + (j - 1)) * 9 + (ii - 1) * 3 + (jj - 1)] = s;
          }
  } else {
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        for (int ii = 0; ii < 4; ++ii)
          for (int jj = 0; jj < 4; ++jj) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k)
              for (int l = 0; l < 4; ++l) {
                if (k == 0 && l == 0) continue;
                const double sk = std::sin(pi * k / 4.0), sl = std::sin(pi * l / 4.0);
                const double lam = 64.0 * (sk * sk + sl * sl);
                s += std::cos(2.0 * pi * (k * (i - ii) + l * (j - jj)) / 4.0) / lam;
              }
            out[(i * 4 + j) * 16 + ii * 4 + jj] = s / 16.0;
          }
  }
}

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

}  // namespace mg

namespace mg {
struct TimingRec {
  int kind, level;
  double bytes;
  hipEvent_t a, b;
};
}  // namespace mg

namespace mg {
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
  hipGraphExec_t graph = nullptr;
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
}  // namespace mg

namespace mg {
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
namespace {

thread_local std::string g_last_error;

int32_t fail(int32_t status, const std::string& why) {
  g_last_error = why;
  return status;
}
}  // namespace

int32_t set_last_error(int32_t status, const char* why) {
  g_last_error = why ? why : "";
  return status;
}

namespace {

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

hipEvent_t take_event(mg_ctx_s* ctx) {
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

double unknowns_side(int n, int bc) { return bc == kDirichlet ? n - 2 : n - 1; }

// SR-CNN prolongation of a coarse correction ec (N x N unique nodes of a
// periodic level, pitch pec) onto fine level `level`: uout = uin + network
// output (uin nullable).  Uses the context's activation buffers.
template <typename T>
int32_t enqueue_cnn(mg_ctx_s* ctx, hipStream_t s, int level, int N, const T* ec, int pec,
                    const T* uin, int pui, T* uout, int puo) {
  const mg::Cnn& c = ctx->cnn;
  const double px = (double)N * N, conv = 2.0 * px * kCnnWidth * kCnnWidth * 9;
  MG_TRY(timed(ctx, s, MG_K_CNN_AUX, level, 2.0 * px * 2 * sizeof(T) + px * 128, [&] {
    return launch_cnn_head<T>(s, N, ec, pec, c.partials, c.stem, c.h, c.scale);
  }));
  for (int b = 0; b < kCnnBlocks; ++b) {
    const unsigned short* w1 = c.w + (size_t)(2 * b) * kCnnConvSet;
    const unsigned short* w2 = w1 + kCnnConvSet;
    MG_TRY(timed(ctx, s, MG_K_CNN, level, conv,
                 [&] { return launch_cnn_conv(s, 0, N, c.h, w1, c.t, nullptr); }));
    MG_TRY(timed(ctx, s, MG_K_CNN, level, conv,
                 [&] { return launch_cnn_conv(s, 1, N, c.t, w2, c.h, c.h); }));
  }
  MG_TRY(timed(ctx, s, MG_K_CNN, level, 4 * conv, [&] {
    return launch_cnn_conv(s, 2, N, c.h, c.w + (size_t)(2 * kCnnBlocks) * kCnnConvSet, c.z,
                           nullptr);
  }));
  MG_TRY(timed(ctx, s, MG_K_CNN_AUX, level, 4 * px * (128 + 2 * sizeof(T)), [&] {
    return launch_cnn_final<T>(s, N, c.z, c.fin, c.scale, uin, pui, uout, puo);
  }));
  return MG_OK;
}

}  // namespace

bool valid_side(int n) {
  if (n < 5 || n > 16385) return false;
  const int m = (n - 1) / 4;
  return (n - 1) % 4 == 0 && (m & (m - 1)) == 0;
}

namespace {

int pitch_for(int n) { return (n + 63) / 64 * 64; }

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
int32_t enqueue_cycle(mg_ctx_s* ctx, const Problem& p, const Hierarchy<T>& h,
                      const std::vector<PrefilterTaps>& taps, T* u0, int pu0, const T* f0,
                      int pf0, hipStream_t s, bool cnn) {
  const int L = p.levels;
  const double* inv = ctx->inv[p.bc];
  auto U = [&](int l) { return l == 0 ? u0 : h.u[l]; };
  auto F = [&](int l) { return l == 0 ? f0 : (const T*)h.f[l]; };
  auto PU = [&](int l) { return l == 0 ? pu0 : p.pitch[l]; };
  auto PF = [&](int l) { return l == 0 ? pf0 : p.pitch[l]; };
  const int nu1 = ctx->opt.nu_pre, nu2 = ctx->opt.nu_post;
  const double sz = sizeof(T);
  const int bc = p.bc;
  if (L == 1) {
    return timed(ctx, s, MG_K_COARSE, 0, 50 * sz,
                 [&] { return launch_coarse<T>(s, bc, f0, pf0, u0, pu0, inv); });
  }
  auto sweeps = [&](int l, int count) -> int32_t {
    const int n = p.side[l];
    const double m = unknowns_side(n, bc);
    for (int k = 0; k < count; ++k)
      MG_TRY(timed(ctx, s, MG_K_RELAX, l, 1.5 * m * m * sz, [&] {
        return launch_relax<T>(s, bc, n, U(l), PU(l), F(l), PF(l), k & 1, 1);
      }));
    return MG_OK;
  };
  for (int l = 0; l + 1 < L; ++l) {
    const int n = p.side[l], nc = p.side[l + 1];
    const double nn = (double)n * n;
    if (l > 0)
      MG_TRY(timed(ctx, s, MG_K_ZERO, l, nn * sz, [&] { return launch_zero<T>(s, n, U(l), PU(l)); }));
    MG_TRY(sweeps(l, 2 * nu1));
    MG_TRY(timed(ctx, s, MG_K_RESIDUAL, l, 3 * nn * sz, [&] {
      return launch_residual<T>(s, bc, n, U(l), PU(l), F(l), PF(l), h.r[l], p.pitch[l]);
    }));
    MG_TRY(timed(ctx, s, MG_K_RESTRICT, l, (nn + (double)nc * nc) * sz, [&] {
      return launch_restrict<T>(s, bc, n, h.r[l], p.pitch[l], h.f[l + 1], p.pitch[l + 1]);
    }));
  }
  MG_TRY(timed(ctx, s, MG_K_COARSE, L - 1, 50 * sz, [&] {
    return launch_coarse<T>(s, bc, h.f[L - 1], p.pitch[L - 1], h.u[L - 1], p.pitch[L - 1], inv);
  }));
  for (int l = L - 2; l >= 0; --l) {
    const int n = p.side[l], nc = p.side[l + 1], pc = p.pitch[l + 1];
    const double m = unknowns_side(n, bc), ncc = (double)nc * nc;
    if (cnn && l < ctx->cnn.levels) {
      MG_TRY(enqueue_cnn<T>(ctx, s, l, nc - 1, h.u[l + 1], pc, U(l), PU(l), U(l), PU(l)));
    } else {
      MG_TRY(timed(ctx, s, MG_K_PREFILTER, l + 1, 4 * ncc * sz, [&] {
        return launch_prefilter<T>(s, bc, nc, taps[l + 1], h.u[l + 1], pc, h.tmp[l + 1], pc,
                                   h.c[l + 1], pc);
      }));
      MG_TRY(timed(ctx, s, MG_K_PROLONG, l, (2 * m * m + ncc) * sz, [&] {
        return launch_prolong<T>(s, bc, n, U(l), PU(l), h.c[l + 1], pc, true);
      }));
    }
    MG_TRY(sweeps(l, 2 * nu2));
  }
  return MG_OK;
}

// The fused schedule: down passes to the first level of at most 65 x 65,
// the tail kernel, then prefilter + up passes back to level 0.  Level l's
// pre-smoothed u goes to h.r[l] (ping-pong against h.u[l] / u0).
template <typename T>
int32_t enqueue_cycle_fused(mg_ctx_s* ctx, const Problem& p, const Hierarchy<T>& h,
                            const PrefilterTaps* taps_dev, T* u0, int pu0, const T* f0, int pf0,
                            bool zero_guess, hipStream_t s, bool cnn, double* u64 = nullptr,
                            int p64 = 0, bool* added = nullptr, const double* res_u = nullptr,
                            const double* res_f = nullptr, int res_p = 0, T* r_out = nullptr,
                            const CallerArgs* ca = nullptr) {
  const int t = p.tail, bc = p.bc;
  // ca: the caller's FP64 arrays are read from the device table.  They are
  // level 0's u0 and f0 on the FP64 path, u64 / res_u / res_f on the mixed
  // path's.
  constexpr bool f64 = sizeof(T) == sizeof(double);
  auto ca_at = [&](int l) { return (f64 && l == 0) ? ca : nullptr; };
  const double sz = sizeof(T);
  auto F = [&](int l) { return l == 0 ? f0 : (const T*)h.f[l]; };
  auto PF = [&](int l) { return l == 0 ? pf0 : p.pitch[l]; };
  // Level l's up pass is a tiled kernel (variant 1, LDS tiles; variant 2,
  // tiles that prefilter their own coarse support) rather than a stream.
  auto up_tiled = [&](int l) {
    return ctx->opt.kernel_path == 2 || p.up_var[l] == 1 || (p.up_var[l] == 2 && l + 1 < t);
  };
  // Mixed level 0 whose down pass makes the residual from e = 0 and whose
  // up pass streams into the FP64 iterate: the up pass makes the
  // pre-smoothed iterate again from r32, so the down pass does not store it.
  const bool remake0 = res_u && u64 && t > 0 && !up_tiled(0) && !(cnn && ctx->cnn.levels > 0);
  for (int l = 0; l < t; ++l) {
    const int n = p.side[l];
    const double m = unknowns_side(n, bc), mc = unknowns_side(p.side[l + 1], bc);
    const T* uin = (l == 0 && !zero_guess) ? u0 : nullptr;
    const double bytes = ((uin ? 3 : 2) * m * m + mc * mc) * sz;
    if constexpr (sizeof(T) == sizeof(float)) {
      if (l == 0 && res_u) {
        // Mixed level 0: the right-hand side is made from the FP64 iterate
        // inside the down pass (and stored for the up pass).
        MG_TRY(timed(ctx, s, MG_K_DOWN, 0, (16 + 4 + (remake0 ? 0 : 4)) * m * m + 4 * mc * mc, [&] {
          return launch_down_res_stream(s, bc, n, res_u, res_p, res_f, res_p, r_out, pf0,
                                        remake0 ? nullptr : h.r[0], p.pitch[0], h.f[1],
                                        p.pitch[1], p.down_hs[0], ca);
        }));
        continue;
      }
    }
    MG_TRY(timed(ctx, s, MG_K_DOWN, l, bytes, [&] {
      if (ctx->opt.kernel_path == 2 || p.down_var[l] == 1)
        return launch_down<T>(s, bc, n, uin, pu0, h.r[l], p.pitch[l], F(l), PF(l), h.f[l + 1],
                              p.pitch[l + 1], ca_at(l));
      return launch_down_stream<T>(s, bc, n, uin, pu0, h.r[l], p.pitch[l], F(l), PF(l),
                                   h.f[l + 1], p.pitch[l + 1], p.down_hs[l], ca_at(l));
    }));
  }
  {
    const int nt = p.side[t];
    const T* uin = (t == 0 && !zero_guess) ? u0 : nullptr;
    T* uout = t == 0 ? u0 : nullptr;
    T* cout = t == 0 ? nullptr : h.c[t];
    const double nn = (double)nt * nt;
    MG_TRY(timed(ctx, s, MG_K_TAIL, t, (uin ? 3 : 2) * nn * sz, [&] {
      return launch_tail<T>(s, bc, nt, uin, pu0, uout, pu0, F(t), PF(t), cout, p.pitch[t],
                            ctx->inv[bc], taps_dev + t, ca_at(t));
    }));
  }
  for (int l = t - 1; l >= 0; --l) {
    const int n = p.side[l], nc = p.side[l + 1], pc = p.pitch[l + 1];
    const double m = unknowns_side(n, bc), ncc = (double)nc * nc;
    T* uout = l == 0 ? u0 : h.u[l];
    const int puo = l == 0 ? pu0 : p.pitch[l];
    if (cnn && l < ctx->cnn.levels) {
      // Network prolongation of the coarse result (level l + 1 lies above
      // the tail, so its values are in h.u), added to the pre-smoothed u,
      // then the post-smoothing sweeps.
      MG_TRY(enqueue_cnn<T>(ctx, s, l, nc - 1, h.u[l + 1], pc, h.r[l], p.pitch[l], uout, puo));
      MG_TRY(timed(ctx, s, MG_K_RELAX, l, 3 * m * m * sz * ctx->opt.nu_post, [&] {
        return launch_relax<T>(s, bc, n, uout, puo, F(l), PF(l), 0, 2 * ctx->opt.nu_post);
      }));
      continue;
    }
    // Variant 2: the tiled up pass prefilters its own coarse support (no
    // prefilter pass over level l + 1).
    const bool pre = ctx->opt.kernel_path != 2 && p.up_var[l] == 2 && l + 1 < t;
    if (l + 1 < t && !pre)
      MG_TRY(timed(ctx, s, MG_K_PREFILTER, l + 1, 4 * ncc * sz, [&] {
        return launch_prefilter_iir<T>(s, bc, nc, h.u[l + 1], pc, h.tmp[l + 1], pc, h.c[l + 1], pc);
      }));
    // Level 0 of the mixed path's last inner cycle: the streaming up pass
    // adds its result straight into the FP64 iterate (no separate update).
    const bool tile = ctx->opt.kernel_path == 2 || p.up_var[l] == 1 || pre;
    const bool add = l == 0 && u64 && !tile;
    if (add && added) *added = true;
    if (l == 0 && remake0) {
      MG_TRY(timed(ctx, s, MG_K_UP, 0, (4 + 8 + 8) * m * m + ncc * sz, [&] {
        return launch_up_pre_stream(s, bc, n, (const float*)F(0), PF(0), (const float*)h.c[1], pc,
                                    p.up_hs[0], u64, p64, ca);
      }));
      continue;
    }
    MG_TRY(timed(ctx, s, MG_K_UP, l, (3 * m * m + ncc) * sz + (add ? 16 * m * m - 4 * m * m : 0), [&] {
      if (tile)
        return launch_up<T>(s, bc, n, h.r[l], p.pitch[l], uout, puo, F(l), PF(l),
                            pre ? h.u[l + 1] : h.c[l + 1], pc, pre, ca_at(l));
      return launch_up_stream<T>(s, bc, n, h.r[l], p.pitch[l], uout, puo, F(l), PF(l),
                                 h.c[l + 1], pc, p.up_hs[l], add ? u64 : nullptr, p64,
                                 add ? ca : ca_at(l));
    }));
  }
  return MG_OK;
}

bool use_fused(const mg_ctx_s* ctx) {
  return ctx->opt.kernel_path != 1 && ctx->opt.nu_pre == 2 && ctx->opt.nu_post == 2;
}

// One step of the outer iteration for one problem: an FP64 V-cycle, or one
// refinement step around inner FP32 cycles.
// One step for problem p: an FP64 V-cycle, or one mixed refinement step
// (FP64 residual, FP32 inner cycles, FP64 update).  have_res: the mixed
// step's residual of this u is already in the level-0 right-hand side (left
// there by enqueue_check_mixed), so the step starts with the inner cycles.
int32_t enqueue_step(mg_ctx_s* ctx, const Problem& p, double* u, const double* f,
                     hipStream_t s, bool cnn, bool have_res = false,
                     const CallerArgs* ca = nullptr) {
  const double m = unknowns_side(p.n, p.bc), nn = (double)p.n * p.n;
  const bool fused = use_fused(ctx);
  if (ctx->opt.precision == MG_FP64) {
    if (fused)
      MG_TRY(enqueue_cycle_fused<double>(ctx, p, p.h64, p.taps64_dev, u, p.pitch0, f, p.pitch0,
                                         false, s, cnn, nullptr, 0, nullptr, nullptr, nullptr, 0,
                                         nullptr, ca));
    else
      MG_TRY(enqueue_cycle<double>(ctx, p, p.h64, p.taps64, u, p.pitch0, f, p.pitch0, s, cnn));
  } else {
    int nb = 0;
    float* e0 = p.h32.u[0];
    float* r0 = p.h32.f[0];
    // The first inner cycle's streaming down pass can make the residual
    // itself when level 0 lies above the tail and both level-0 passes stream
    // (the up pass reads only rows and columns that down pass stores).
    const bool res_in_down = fused && !have_res && p.tail > 0 && ctx->opt.kernel_path != 2 &&
                             p.down_var[0] == 0 && p.up_var[0] == 0;
    if (!have_res && !res_in_down)
      MG_TRY(timed(ctx, s, MG_K_RESIDUAL_MIXED, 0, 20 * nn, [&] {
        return launch_residual_mixed(s, p.bc, p.n, u, p.pitch0, f, p.pitch0, r0, p.pitch[0],
                                     p.partials, &nb, ca);
      }));
    bool added = false;
    if (fused) {
      const int K = ctx->opt.inner_cycles;
      for (int k = 0; k < K; ++k) {
        const bool rd = res_in_down && k == 0;
        MG_TRY(enqueue_cycle_fused<float>(ctx, p, p.h32, p.taps32_dev, e0, p.pitch[0], r0,
                                          p.pitch[0], k == 0, s, cnn, k == K - 1 ? u : nullptr,
                                          p.pitch0, &added, rd ? u : nullptr, rd ? f : nullptr,
                                          p.pitch0, r0, ca));
      }
    } else {
      MG_TRY(timed(ctx, s, MG_K_ZERO, 0, 4 * nn,
                   [&] { return launch_zero<float>(s, p.n, e0, p.pitch[0]); }));
      for (int k = 0; k < ctx->opt.inner_cycles; ++k)
        MG_TRY(enqueue_cycle<float>(ctx, p, p.h32, p.taps32, e0, p.pitch[0], r0, p.pitch[0], s,
                                    cnn));
    }
    if (!added)
      MG_TRY(timed(ctx, s, MG_K_UPDATE_MIXED, 0, 20 * m * m, [&] {
        return launch_update_mixed(s, p.bc, p.n, u, p.pitch0, e0, p.pitch[0], ca);
      }));
  }
  if (p.bc == kPeriodic) MG_HIP(launch_seam<double>(s, p.n, u, p.pitch0, ca));
  return MG_OK;
}

int32_t run_step(mg_ctx_s* ctx, Problem& p, double* u, const double* f, bool cnn = false,
                 bool have_res = false) {
  if (!ctx->opt.use_graph || ctx->timing)
    return enqueue_step(ctx, p, u, f, ctx->stream, cnn, have_res);
  const int k = (cnn ? 1 : 0) + (have_res ? 2 : 0);
  // The fused schedule's kernels read the caller's arrays from the
  // problem's device slot: one captured graph serves every u and f, and a
  // change of arrays only rewrites the slot (in stream order, before the
  // launch).  The per-operation and SR-CNN schedules take them as kernel
  // arguments, so their graphs are captured again when the arrays change.
  const bool table = use_fused(ctx) && !cnn;
  if (table) {
    if (p.bound_u != u || p.bound_f != f) {
      MG_HIP(launch_bind_caller(ctx->stream, p.caller, u, f));
      p.bound_u = u;
      p.bound_f = f;
    }
  } else if (p.graph[k] && (p.graph_u[k] != u || p.graph_f[k] != f)) {
    MG_HIP(hipGraphExecDestroy(p.graph[k]));
    p.graph[k] = nullptr;
  }
  if (!p.graph[k]) {
    hipGraph_t g = nullptr;
    MG_HIP(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeRelaxed));
    const int32_t st =
        enqueue_step(ctx, p, u, f, ctx->capture, cnn, have_res, table ? p.caller : nullptr);
    hipError_t e = hipStreamEndCapture(ctx->capture, &g);
    ++ctx->graph_captures;
    if (st != MG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(MG_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&p.graph[k], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      p.graph[k] = nullptr;
      return fail(MG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    ++ctx->graph_instantiations;
    p.graph_u[k] = u;
    p.graph_f[k] = f;
  }
  MG_HIP(hipGraphLaunch(p.graph[k], ctx->stream));
  return MG_OK;
}

// Queue ||f - A u||^2 (and ||f||^2) into p.sums[0..1].
int32_t enqueue_resnorm(mg_ctx_s* ctx, Problem& p, const double* u, const double* f) {
  int nb = 0;
  const double m = unknowns_side(p.n, p.bc);
  MG_TRY(timed(ctx, ctx->stream, MG_K_RESNORM, 0, 16 * m * m, [&] {
    return launch_resnorm(ctx->stream, p.bc, p.n, u, p.pitch0, f, p.pitch0, p.partials, true, &nb);
  }));
  MG_HIP(launch_reduce(ctx->stream, p.partials, nb, nb, 2, p.sums));
  return MG_OK;
}

// Mixed path: ||f - A u||^2 into p.sums[0] from the FP64 residual that the
// next refinement step starts from; its FP32 copy stays in the level-0
// right-hand side, so that step skips it (run_step with have_res).
int32_t enqueue_check_mixed(mg_ctx_s* ctx, Problem& p, const double* u, const double* f) {
  int nb = 0;
  const double nn = (double)p.n * p.n;
  MG_TRY(timed(ctx, ctx->stream, MG_K_RESIDUAL_MIXED, 0, 20 * nn, [&] {
    return launch_residual_mixed(ctx->stream, p.bc, p.n, u, p.pitch0, f, p.pitch0, p.h32.f[0],
                                 p.pitch[0], p.partials, &nb);
  }));
  MG_HIP(launch_reduce(ctx->stream, p.partials, nb, nb, 1, p.sums));
  return MG_OK;
}

// ||f||^2 over the unknowns into p.sums[1] (the denominator read_relres
// uses), through p.sums[2..3].
int32_t enqueue_fnorm(mg_ctx_s* ctx, Problem& p, const double* f) {
  int nb = 0;
  MG_HIP(launch_rhs_moments(ctx->stream, p.bc, p.n, f, p.pitch0, p.partials, &nb));
  MG_HIP(launch_reduce(ctx->stream, p.partials, nb, nb, 2, p.sums + 2));
  MG_HIP(hipMemcpyAsync(p.sums + 1, p.sums + 3, sizeof(double), hipMemcpyDeviceToDevice,
                        ctx->stream));
  return MG_OK;
}

// ---------------------------------------------------------------- persistent

template <typename T>
const Hierarchy<T>& hier(const Problem& p);
template <>
const Hierarchy<double>& hier<double>(const Problem& p) {
  return p.h64;
}
template <>
const Hierarchy<float>& hier<float>(const Problem& p) {
  return p.h32;
}

bool cnn_cycles(const mg_ctx_s* ctx) { return ctx->cnn.on && ctx->cnn.levels > 0; }

bool persistent_eligible(const mg_ctx_s* ctx, std::string* why) {
  const auto& o = ctx->opt;
  if (o.prolong == MG_PROLONG_SRCNN) {
    *why = "the persistent schedule uses the spline prolongation only";
    return false;
  }
  if (o.kernel_path != 0 || o.nu_pre != 2 || o.nu_post != 2) {
    *why = "the persistent schedule needs kernel_path 0 and nu_pre = nu_post = 2";
    return false;
  }
  if (o.precision == MG_MIXED && o.inner_cycles != 1) {
    *why = "the persistent schedule needs inner_cycles = 1";
    return false;
  }
  for (const auto& p : ctx->probs)
    if (p.bc != ctx->probs[0].bc) {
      *why = "the persistent schedule needs one boundary condition for the whole batch";
      return false;
    }
  return true;
}

// Flattens one step of every problem into phases aligned from the coarsest
// level and uploads the tables.
template <typename T>
int32_t build_persistent(mg_ctx_s* ctx) {
  Persist& P = ctx->ps;
  const bool mixed = ctx->opt.precision == MG_MIXED;
  const int B = (int)ctx->probs.size();
  P.bc = ctx->probs[0].bc;
  P.h_probs.assign(B, PProblem{});
  P.lds_pre = P.lds_tail = 0;
  int K = 0;
  size_t lds = 0;
  for (int b = 0; b < B; ++b) {
    const Problem& p = ctx->probs[b];
    const Hierarchy<T>& h = hier<T>(p);
    PProblem& q = P.h_probs[b];
    q.levels = p.levels;
    q.tail = p.tail;
    q.bc = p.bc;
    q.active = 1;
    q.pitch64 = p.pitch0;
    q.zero_guess = mixed ? 1 : 0;
    for (int l = 0; l < p.levels; ++l) {
      PLevel& L = q.lv[l];
      L.u = h.u[l];
      L.f = h.f[l];
      L.b = h.r[l];
      L.c = h.c[l];
      L.tmp = h.tmp[l];
      L.n = p.side[l];
      L.pitch = L.pitch_u = L.pitch_f = p.pitch[l];
      if (l == 0 && !mixed) L.pitch_u = L.pitch_f = p.pitch0;
      L.hs_down = stream_segment_rows(L.n, p.bc, stream_down_owned());
      L.hs_up = stream_segment_rows(L.n, p.bc, stream_up_owned());
      const int extent = p.bc == kPeriodic ? L.n - 1 : L.n;
      L.nb_down = (extent + stream_down_owned() - 1) / stream_down_owned();
      L.nb_up = (extent + stream_up_owned() - 1) / stream_up_owned();
      if (l > 0 && l < p.tail) P.lds_pre = std::max(P.lds_pre, dev::PreTile<T>::kLds);
    }
    K = std::max(K, p.tail);
    P.lds_tail = std::max(P.lds_tail, dev::tail_bytes(p.side[p.tail], sizeof(T)));
  }
  // Segment rows of the streaming phases: every problem's level in a phase
  // gets the smallest even height at which the phase's items over the whole
  // batch fit the kernel's resident wavefronts (a problem alone would cut
  // its levels much finer, each segment re-reading its halo rows).
  {
    long slots_down = 0, slots_up = 0;
    MG_HIP(phase_wave_slots<T>(P.bc, kItemDown, &slots_down));
    MG_HIP(phase_wave_slots<T>(P.bc, kItemUp, &slots_up));
    for (int k = 0; k < K; ++k)
      for (int down = 0; down < 2; ++down) {
        const long slots = down ? slots_down : slots_up;
        auto items_at = [&](int hs) {
          long tot = 0;
          for (int b = 0; b < B; ++b) {
            const int l = ctx->probs[b].tail - 1 - k;
            if (l < 0) continue;
            const PLevel& L = P.h_probs[b].lv[l];
            const int extent = P.bc == kPeriodic ? L.n - 1 : L.n;
            tot += (long)(down ? L.nb_down : L.nb_up) * ((extent + hs - 1) / hs);
          }
          return tot;
        };
        int hs = 8;
        while (hs < 4096 && items_at(hs) > slots) hs += 2;
        for (int b = 0; b < B; ++b) {
          const int l = ctx->probs[b].tail - 1 - k;
          if (l < 0) continue;
          PLevel& L = P.h_probs[b].lv[l];
          (down ? L.hs_down : L.hs_up) = hs;
        }
      }
  }
  std::vector<PPhase> phases;
  std::vector<PItem> items;
  auto close_phase = [&](int kind, size_t first) {
    if (items.size() > first) phases.push_back({kind, (int)first, (int)(items.size() - first), 0});
  };
  auto band_items = [&](int b, int l, bool down) {
    const PLevel& L = P.h_probs[b].lv[l];
    const int extent = P.bc == kPeriodic ? L.n - 1 : L.n;
    const int hs = down ? L.hs_down : L.hs_up, nb = down ? L.nb_down : L.nb_up;
    const int ns = (extent + hs - 1) / hs;
    for (int sg = 0; sg < ns; ++sg)
      for (int bd = 0; bd < nb; ++bd) items.push_back({b, l, bd, sg});
  };
  // Mixed path: the FP64 residual of problems whose level 0 is the tail
  // (the level-0 down pass makes it for the others).
  if (mixed) {
    const size_t first = items.size();
    const int ow = stream_res_owned();
    for (int b = 0; b < B; ++b) {
      if (ctx->probs[b].tail > 0) continue;
      const int n = ctx->probs[b].n;
      for (int sg = 0; sg < (n + kResSegRows - 1) / kResSegRows; ++sg)
        for (int bd = 0; bd < (n + ow - 1) / ow; ++bd) items.push_back({b, 0, bd, sg});
    }
    close_phase(kItemRes, first);
  }
  for (int k = K - 1; k >= 0; --k) {
    const size_t first = items.size();
    for (int b = 0; b < B; ++b) {
      const int l = ctx->probs[b].tail - 1 - k;
      if (l >= 0) band_items(b, l, true);
    }
    close_phase(kItemDown, first);
  }
  {
    const size_t first = items.size();
    for (int b = 0; b < B; ++b) items.push_back({b, ctx->probs[b].tail, 0, 0});
    close_phase(kItemTail, first);
  }
  for (int k = 0; k < K; ++k) {
    size_t first = items.size();
    for (int b = 0; b < B; ++b) {
      const int l = ctx->probs[b].tail - 1 - k;
      if (l >= 0 && l + 1 < ctx->probs[b].tail) {
        using C = dev::PreTile<T>;
        const int nc = ctx->probs[b].side[l + 1];
        const int extent = P.bc == kPeriodic ? nc - 1 : nc;
        const int tx = (extent + C::TW - 1) / C::TW, ty = (extent + C::TH - 1) / C::TH;
        for (int tile = 0; tile < tx * ty; ++tile) items.push_back({b, l + 1, tile, tx});
      }
    }
    close_phase(kItemPre, first);
    first = items.size();
    for (int b = 0; b < B; ++b) {
      const int l = ctx->probs[b].tail - 1 - k;
      if (l >= 0) band_items(b, l, false);
    }
    close_phase(kItemUp, first);
  }
  // Mixed path: the level-0 up pass adds into the FP64 iterate; only
  // problems that lie wholly in the tail still need the update rows.
  if (mixed) {
    const size_t first = items.size();
    for (int b = 0; b < B; ++b)
      if (ctx->probs[b].tail == 0)
        for (int r = 0; r < ctx->probs[b].n; r += kRowsPerItem) items.push_back({b, 0, r, 0});
    close_phase(kItemUpd, first);
  }

  // Algorithmic bytes of the step, per pass (m = unknowns per side):
  // residual 20 m^2 (u, f FP64 read, r FP32 written); down pass
  // (2 or 3) m^2 + mc^2 words (f read, pre-smoothed u written, u read
  // unless the guess is zero, fc written), the mixed level-0 pass 20 m^2 +
  // 4 mc^2 (u, f FP64 read, r written, no pre-smoothed u); tail (2 or 3)
  // nt^2 words; prefilter 2 nc^2 words; up pass 3 m^2 + nc^2 words, the
  // mixed level-0 pass 20 m^2 + 4 nc^2 (r read, the FP64 iterate read and
  // written); update 20 m^2.
  {
    const double sz = sizeof(T);
    double by = 0.0;
    for (int b = 0; b < B; ++b) {
      const Problem& p = ctx->probs[b];
      auto unk = [&](int l) {
        const double m = unknowns_side(p.side[l], p.bc);
        return m * m;
      };
      if (mixed && p.tail == 0) by += 20.0 * unk(0);
      for (int l = 0; l < p.tail; ++l) {
        const double nc2 = (double)p.side[l + 1] * p.side[l + 1];
        if (l + 1 < p.tail) by += 2.0 * nc2 * sz;
        if (l == 0 && mixed) {
          by += 20.0 * unk(0) + 4.0 * unk(1) + 20.0 * unk(0) + 4.0 * nc2;
          continue;
        }
        const bool uin = l == 0 && !mixed;
        by += ((uin ? 3.0 : 2.0) * unk(l) + unk(l + 1)) * sz;
        by += (3.0 * unk(l) + nc2) * sz;
      }
      const double nt2 = (double)p.side[p.tail] * p.side[p.tail];
      by += ((p.tail == 0 && !mixed) ? 3.0 : 2.0) * nt2 * sz;
      if (mixed && p.tail == 0) by += 20.0 * unk(0);
    }
    P.bytes = by;
  }
  lds = std::max(P.lds_pre, P.lds_tail);
  P.lds = lds;
  P.h_phases = phases;
  MG_HIP(persistent_init(std::max(lds, (size_t)65536), std::max(lds, (size_t)65536)));
  MG_HIP(persistent_blocks<T>(P.bc, lds, &P.blocks));
  if (P.blocks <= 0) return fail(MG_ERR_UNSUPPORTED, "persistent kernel does not fit on a CU");
  unsigned char* d = nullptr;
  MG_TRY(alloc_level<unsigned char>(ctx, 1, (int)(sizeof(PProblem) * B), &d));
  P.d_probs = reinterpret_cast<PProblem*>(d);
  MG_TRY(alloc_level<unsigned char>(ctx, 1, (int)(sizeof(PPhase) * phases.size()), &d));
  P.d_phases = reinterpret_cast<PPhase*>(d);
  MG_TRY(alloc_level<unsigned char>(ctx, 1, (int)(sizeof(PItem) * items.size()), &d));
  P.d_items = reinterpret_cast<PItem*>(d);
  MG_TRY(alloc_level<unsigned char>(ctx, 1, (int)sizeof(PBarrier), &d));
  P.d_bar = reinterpret_cast<PBarrier*>(d);
  MG_TRY(alloc_level<double>(ctx, 2 * B, P.slots, &P.d_partials));
  MG_TRY(alloc_level<double>(ctx, 2, B, &P.d_sums));
  MG_HIP(hipMemcpyAsync(P.d_phases, phases.data(), sizeof(PPhase) * phases.size(),
                        hipMemcpyHostToDevice, ctx->stream));
  MG_HIP(hipMemcpyAsync(P.d_items, items.data(), sizeof(PItem) * items.size(),
                        hipMemcpyHostToDevice, ctx->stream));
  MG_HIP(hipStreamSynchronize(ctx->stream));
  P.nphases = (int)phases.size();
  P.on = true;
  P.dirty = true;
  return MG_OK;
}

// Points the problem table at the caller's arrays and activity flags, and
// uploads it if anything changed.
int32_t persistent_bind(mg_ctx_s* ctx, double* const* u, const double* const* f,
                        const std::vector<int>& active) {
  Persist& P = ctx->ps;
  const bool mixed = ctx->opt.precision == MG_MIXED;
  for (size_t b = 0; b < P.h_probs.size(); ++b) {
    PProblem& q = P.h_probs[b];
    const int act = active.empty() ? 1 : active[b];
    if (q.u64 != u[b] || q.f64 != f[b] || q.active != act) P.dirty = true;
    q.u64 = u[b];
    q.f64 = f[b];
    q.active = act;
    if (!mixed) {
      q.lv[0].u = u[b];
      q.lv[0].f = const_cast<double*>(f[b]);
    }
  }
  if (P.dirty) {
    MG_HIP(hipMemcpyAsync(P.d_probs, P.h_probs.data(), sizeof(PProblem) * P.h_probs.size(),
                          hipMemcpyHostToDevice, ctx->stream));
    P.dirty = false;
  }
  return MG_OK;
}

int32_t persistent_launch(mg_ctx_s* ctx) {
  Persist& P = ctx->ps;
  const bool mixed = ctx->opt.precision == MG_MIXED;
  auto launch = [&](hipStream_t s) {
    if (!P.phased)
      return mixed ? launch_persistent<float>(s, P.bc, P.d_probs, P.d_phases, P.nphases,
                                              P.d_items, P.d_bar, ctx->inv[P.bc], P.blocks, P.lds)
                   : launch_persistent<double>(s, P.bc, P.d_probs, P.d_phases, P.nphases,
                                               P.d_items, P.d_bar, ctx->inv[P.bc], P.blocks,
                                               P.lds);
    // One launch per phase: workgroup items one workgroup each, wavefront
    // items kPersistThreads / 64 per workgroup.
    for (int ph = 0; ph < P.nphases; ++ph) {
      const PPhase& q = P.h_phases[ph];
      const bool wg = q.kind == kItemTail || q.kind == kItemPre;
      const int per = kPersistThreads / 64;
      const int blocks = wg ? q.count : (q.count + per - 1) / per;
      const size_t lds = q.kind == kItemTail ? P.lds_tail : (q.kind == kItemPre ? P.lds_pre : 0);
      const hipError_t e =
          mixed ? launch_phase<float>(s, P.bc, q.kind, P.d_probs, P.d_phases, ph, P.d_items,
                                      ctx->inv[P.bc], blocks, lds)
                : launch_phase<double>(s, P.bc, q.kind, P.d_probs, P.d_phases, ph, P.d_items,
                                       ctx->inv[P.bc], blocks, lds);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  if (!ctx->opt.use_graph || ctx->timing) {
    MG_TRY(timed(ctx, ctx->stream, P.phased ? MG_K_PHASED : MG_K_PERSISTENT, 0, P.bytes,
                 [&] { return launch(ctx->stream); }));
    return MG_OK;
  }
  if (!P.graph) {
    hipGraph_t g = nullptr;
    MG_HIP(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeRelaxed));
    const hipError_t le = launch(ctx->capture);
    hipError_t e = hipStreamEndCapture(ctx->capture, &g);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(MG_ERR_HIP, std::string("persistent launch: ") + hipGetErrorString(le));
    }
    if (e != hipSuccess) return fail(MG_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&P.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      P.graph = nullptr;
      return fail(MG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
  }
  MG_HIP(hipGraphLaunch(P.graph, ctx->stream));
  return MG_OK;
}

// Reads the device-wide barrier's error word (synchronises).  A barrier that
// timed out in an earlier launch leaves the word set, and every later launch
// exits at entry while it is; so the word is cleared here and the call that
// queued the failed launches reports MG_ERR_HIP.
int32_t persistent_check(mg_ctx_s* ctx) {
  Persist& P = ctx->ps;
  PBarrier bar{};
  MG_HIP(hipMemcpyAsync(&bar, P.d_bar, sizeof bar, hipMemcpyDeviceToHost, ctx->stream));
  MG_HIP(hipStreamSynchronize(ctx->stream));
  if (bar.error) {
    MG_HIP(hipMemsetAsync(P.d_bar, 0, sizeof(PBarrier), ctx->stream));
    MG_HIP(hipStreamSynchronize(ctx->stream));
    return fail(MG_ERR_HIP, "persistent kernel: device-wide barrier timed out");
  }
  return MG_OK;
}

// Relative residuals of all problems from the batched kernels (synchronises);
// also reports a timed-out device barrier.
int32_t persistent_relres(mg_ctx_s* ctx, double* rel) {
  Persist& P = ctx->ps;
  const int B = (int)ctx->probs.size();
  MG_HIP(launch_resnorm_batched(ctx->stream, P.bc, P.d_probs, B, P.d_partials, P.slots,
                                P.d_sums));
  std::vector<double> sums(2 * B);
  MG_HIP(hipMemcpyAsync(sums.data(), P.d_sums, sizeof(double) * 2 * B, hipMemcpyDeviceToHost,
                        ctx->stream));
  MG_TRY(persistent_check(ctx));
  for (int b = 0; b < B; ++b) {
    const double rr = sums[2 * b], ff = sums[2 * b + 1];
    rel[b] = ff > 0.0 ? std::sqrt(rr) / std::sqrt(ff) : std::sqrt(rr);
  }
  return MG_OK;
}

// ----------------------------------------------------------------- SR-CNN setup

// bfloat16 nearest-even rounding of a finite float (bit pattern).
unsigned short bf16_bits(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (unsigned short)(b >> 16);
}
float bf16_float(float x) {
  const uint32_t b = (uint32_t)bf16_bits(x) << 16;
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}

// Validates the network levels against every problem, converts the weight
// blob (PyTorch order, see MG_SRCNN_WEIGHT_COUNT) to the kernels' layouts and
// allocates the activation buffers for the largest coarse level.
int32_t cnn_setup(mg_ctx_s* ctx, const float* blob) {
  Cnn& c = ctx->cnn;
  c.levels = ctx->opt.cnn_levels;
  for (size_t b = 0; b < ctx->probs.size(); ++b) {
    const Problem& p = ctx->probs[b];
    if (c.levels > p.levels - 1)
      return fail(MG_ERR_UNSUPPORTED, "problem " + std::to_string(b) + ": cnn_levels exceeds the hierarchy");
    for (int l = 0; l < c.levels; ++l)
      if (p.side[l + 1] < 129)
        return fail(MG_ERR_UNSUPPORTED, "problem " + std::to_string(b) +
                                             ": SR-CNN levels need a coarse side of at least 129");
    if (p.levels > 1 && p.side[1] - 1 >= 32) c.max_n = std::max(c.max_n, p.side[1] - 1);
  }
  for (size_t k = 0; k < (size_t)MG_SRCNN_WEIGHT_COUNT; ++k)
    if (!std::isfinite(blob[k])) return fail(MG_ERR_INVALID_ARG, "non-finite SR-CNN weight");
  constexpr int W = kCnnWidth;
  const size_t set = kCnnConvSet;
  std::vector<unsigned short> w((2 * kCnnBlocks + 4) * set);
  std::vector<float> stem(W * 9), fin(9 * W);
  const float* src_stem = blob;
  const float* src_body = blob + W * 9;
  const float* src_up = src_body + 2 * kCnnBlocks * set;
  const float* src_fin = src_up + 4 * set;
  for (int o = 0; o < W; ++o)
    for (int t = 0; t < 9; ++t) stem[o * 9 + t] = bf16_float(src_stem[o * 9 + t]);
  for (int k = 0; k < 2 * kCnnBlocks; ++k)
    for (int o = 0; o < W; ++o)
      for (int i = 0; i < W; ++i)
        for (int t = 0; t < 9; ++t)
          w[k * set + ((size_t)t * W + o) * W + i] = bf16_bits(src_body[k * set + ((size_t)o * W + i) * 9 + t]);
  for (int ab = 0; ab < 4; ++ab)
    for (int ch = 0; ch < W; ++ch)
      for (int i = 0; i < W; ++i)
        for (int t = 0; t < 9; ++t)
          w[(2 * kCnnBlocks + ab) * set + ((size_t)t * W + ch) * W + i] =
              bf16_bits(src_up[((size_t)(4 * ch + ab) * W + i) * 9 + t]);
  for (int i = 0; i < W; ++i)
    for (int t = 0; t < 9; ++t) fin[t * W + i] = bf16_float(src_fin[i * 9 + t]);

  MG_TRY(alloc_level<unsigned short>(ctx, 2 * kCnnBlocks + 4, (int)set, &c.w));
  MG_TRY(alloc_level<float>(ctx, 1, W * 9, &c.stem));
  MG_TRY(alloc_level<float>(ctx, 1, 9 * W, &c.fin));
  MG_TRY(alloc_level<float>(ctx, 1, cnn_partials() + 1, &c.partials));
  c.scale = c.partials + cnn_partials();
  if (c.max_n > 0) {
    const int N = c.max_n;
    MG_TRY(alloc_level<unsigned short>(ctx, N * N, W, &c.h));
    MG_TRY(alloc_level<unsigned short>(ctx, N * N, W, &c.t));
    MG_TRY(alloc_level<unsigned short>(ctx, 4 * N * N, W, &c.z));
  }
  MG_HIP(hipMemcpyAsync(c.w, w.data(), w.size() * sizeof(unsigned short), hipMemcpyHostToDevice,
                        ctx->stream));
  MG_HIP(hipMemcpyAsync(c.stem, stem.data(), stem.size() * sizeof(float), hipMemcpyHostToDevice,
                        ctx->stream));
  MG_HIP(hipMemcpyAsync(c.fin, fin.data(), fin.size() * sizeof(float), hipMemcpyHostToDevice,
                        ctx->stream));
  MG_HIP(hipStreamSynchronize(ctx->stream));  // the host staging vectors go out of scope
  MG_HIP(cnn_init());
  c.on = true;
  return MG_OK;
}

// ----------------------------------------------------------------- autotuner
//
// Choices are keyed by (GPU architecture, cycle precision, boundary
// condition, level side) for the per-level kernels, and by the batch's
// signature for the schedule.  They live in a process-wide table and, when
// tune_cache_path is set, in a text file of lines
//   L <arch> <fp32|fp64> <bc> <n> <down_var> <down_hs> <up_var> <up_hs> <us>
//   S <arch> <fp32|fp64> <bc> <batch signature> <schedule>
// read at setup and appended when new choices are measured.

struct LevelChoice {
  int down_var = 0, down_hs = 0, up_var = 0, up_hs = 0;
};

std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}
std::map<std::string, LevelChoice>& level_table() {
  static std::map<std::string, LevelChoice> t;
  return t;
}
std::map<std::string, int>& schedule_table() {
  static std::map<std::string, int> t;
  return t;
}

std::string device_arch(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

void load_tune_file(const char* path) {
  if (!path) return;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return;
  char line[512];
  while (std::fgets(line, sizeof line, fp)) {
    char kind[4], arch[64], prec[8], sig[256];
    int bc = 0, n = 0, dv = 0, dh = 0, uv = 0, uh = 0, sched = 0;
    double us = 0.0;
    if (std::sscanf(line, "%3s", kind) != 1) continue;
    if (kind[0] == 'L' &&
        std::sscanf(line, "L %63s %7s %d %d %d %d %d %d %lf", arch, prec, &bc, &n, &dv, &dh, &uv,
                    &uh, &us) == 9) {
      LevelChoice c;
      c.down_var = dv;
      c.down_hs = dh;
      c.up_var = uv;
      c.up_hs = uh;
      level_table()[std::string(arch) + " " + prec + " " + std::to_string(bc) + " " +
                    std::to_string(n)] = c;
    } else if (kind[0] == 'S' &&
               std::sscanf(line, "S %63s %7s %d %255s %d", arch, prec, &bc, sig, &sched) == 5) {
      schedule_table()[std::string(arch) + " " + prec + " " + std::to_string(bc) + " " + sig] =
          sched;
    }
  }
  std::fclose(fp);
}

void append_tune_file(const char* path, const std::string& line) {
  if (!path) return;
  FILE* fp = std::fopen(path, "a");
  if (!fp) return;
  std::fputs(line.c_str(), fp);
  std::fclose(fp);
}

// Mean time of `reps` launches of `launch` on the context's stream (ms).
template <class Launch>
int32_t time_launches(mg_ctx_s* ctx, int reps, Launch&& launch, float* ms) {
  hipEvent_t a = take_event(ctx), b = take_event(ctx);
  if (!a || !b) return fail(MG_ERR_HIP, "hipEventCreate failed");
  MG_HIP(launch());  // warm-up
  MG_HIP(hipEventRecord(a, ctx->stream));
  for (int r = 0; r < reps; ++r) MG_HIP(launch());
  MG_HIP(hipEventRecord(b, ctx->stream));
  MG_HIP(hipEventSynchronize(b));
  MG_HIP(hipEventElapsedTime(ms, a, b));
  *ms /= reps;
  ctx->pool_used -= 2;
  return MG_OK;
}

// Per-level kernel choice: the streaming passes with several segment heights
// against the LDS-tiled passes, each timed on the level's own arrays (the
// level-0 caller arrays are stood in for by library arrays of the same
// shape).  Values do not matter to the timing.  The mixed path's level-0 up
// pass adds into the FP64 iterate and makes the pre-smoothed iterate again
// (a different kernel, keyed "fp32a"), so it is timed that way, against a
// scratch FP64 array, and only among the streaming candidates; its
// streaming down pass makes the FP64 residual itself and stores no
// pre-smoothed iterate, so it is timed in that form, and the tiled down pass
// is charged the separate residual pass it then needs.
template <typename T>
int32_t tune_levels(mg_ctx_s* ctx, Problem& p, const std::string& arch, T* scratch_u, T* scratch_f,
                    int pitch0) {
  const Hierarchy<T>& h = hier<T>(p);
  const bool mixed = ctx->opt.precision == MG_MIXED;
  double* u64 = nullptr;
  struct Free {
    double*& q;
    ~Free() {
      if (q) (void)hipFree(q);
    }
  } free_u64{u64};
  for (int l = 0; l < p.tail; ++l) {
    const int n = p.side[l];
    const bool add = mixed && l == 0;
    const char* prec = sizeof(T) == 8 ? "fp64" : (add ? "fp32a" : "fp32");
    const std::string key = arch + " " + prec + " " + std::to_string(p.bc) + " " + std::to_string(n);
    {
      std::lock_guard<std::mutex> lk(tune_mutex());
      auto it = level_table().find(key);
      if (it != level_table().end()) {
        p.down_var[l] = it->second.down_var;
        p.down_hs[l] = it->second.down_hs;
        p.up_var[l] = it->second.up_var;
        p.up_hs[l] = it->second.up_hs;
        continue;
      }
    }
    T* u = l == 0 ? scratch_u : h.u[l];
    const T* f = l == 0 ? scratch_f : h.f[l];
    const int pu = l == 0 ? pitch0 : p.pitch[l];
    const T* uin = (l == 0 && !mixed) ? u : nullptr;
    const int reps = n >= 2049 ? 3 : 6;
    // Fixed heights, plus for each pass the height at which all its items
    // are resident at once (at 4097^2 the mixed up pass runs 85 us at 64
    // rows, 70 us at 38, and 97 us at 32, where the items no longer fit).
    std::vector<int> hs_cands = {0, 4, 8, 16, 32, 64, 96, 128};
    {
      const int fd = stream_fit_rows<T>(add ? kFitDownRes : (uin ? kFitDownIn : kFitDown), p.bc, n);
      const int fu = stream_fit_rows<T>(add ? kFitUpPre : kFitUp, p.bc, n);
      for (int hs : {fd, fu})
        if (hs > 0 && std::find(hs_cands.begin(), hs_cands.end(), hs) == hs_cands.end())
          hs_cands.push_back(hs);
    }
    if (add && !u64) {
      if (hipMalloc(&u64, sizeof(double) * (size_t)n * p.pitch[0]) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MG_ERR_OOM, "scratch FP64 array for tuning");
      }
    }
    float best_d = 1e30f, best_u = 1e30f, us_total = 0.f;
    LevelChoice c;
    // The separate prefilter of level l + 1, charged to the up-pass variants
    // that need it (variant 2 prefilters inside its tiles).
    float mp = 0.f, mr = 0.f;
    if (add) {
      int nb = 0;
      MG_TRY(time_launches(ctx, reps, [&] {
        return launch_residual_mixed(ctx->stream, p.bc, n, u64, p.pitch[0], u64, p.pitch[0],
                                     reinterpret_cast<float*>(scratch_f), pu, p.partials, &nb);
      }, &mr));
    }
    const bool can_pre = !add && l + 1 < p.tail;
    if (can_pre) {
      const int nc = p.side[l + 1], pc = p.pitch[l + 1];
      MG_TRY(time_launches(ctx, reps, [&] {
        return launch_prefilter_iir<T>(ctx->stream, p.bc, nc, h.u[l + 1], pc, h.tmp[l + 1], pc,
                                       h.c[l + 1], pc);
      }, &mp));
    }
    // Short segments re-read more halo rows.  Timed alone, a pass finds those
    // rows in the 256 MB last-level cache; inside a cycle over a level larger
    // than that cache they come from HBM (4097^2 mixed down pass: 16-row
    // segments time faster here but run 9 % slower in the cycle), so such
    // levels do not try them.
    const double level_bytes = (double)n * n * (add ? 24.0 : 3.0 * sizeof(T));
    const bool big = level_bytes > 256e6;
    for (int var = 0; var < 3; ++var)
      for (int hs : hs_cands) {
        if (var >= 1 && hs != 0) continue;
        if (var == 2 && !can_pre) continue;
        if (big && hs > 0 && hs < 32) continue;
        float md = 1e30f, mu = 0.f;
        if (var < 2)  // variant 2 concerns the up pass only
          MG_TRY(time_launches(ctx, reps, [&] {
            if constexpr (sizeof(T) == sizeof(float)) {
              // As it runs in the cycle: the pre-smoothed iterate is not
              // stored (the up pass makes it again).
              if (add && var == 0)
                return launch_down_res_stream(ctx->stream, p.bc, n, u64, p.pitch[0], u64,
                                              p.pitch[0], scratch_f, pu, nullptr, p.pitch[l],
                                              h.f[l + 1], p.pitch[l + 1], hs);
            }
            return var == 1 ? launch_down<T>(ctx->stream, p.bc, n, uin, pu, h.r[l], p.pitch[l], f,
                                             pu, h.f[l + 1], p.pitch[l + 1])
                            : launch_down_stream<T>(ctx->stream, p.bc, n, uin, pu, h.r[l],
                                                    p.pitch[l], f, pu, h.f[l + 1], p.pitch[l + 1],
                                                    hs);
          }, &md));
        if (add && var == 1) md += mr;
        if (add && var >= 1) {
          mu = 1e30f;  // the tiled up pass does not add into the FP64 iterate
        } else {
          MG_TRY(time_launches(ctx, reps, [&] {
            if constexpr (sizeof(T) == sizeof(float)) {
              if (add)
                return launch_up_pre_stream(ctx->stream, p.bc, n, f, pu, h.c[l + 1],
                                            p.pitch[l + 1], hs, u64, p.pitch[0]);
            }
            if (var >= 1)
              return launch_up<T>(ctx->stream, p.bc, n, h.r[l], p.pitch[l], u, pu, f, pu,
                                  var == 2 ? h.u[l + 1] : h.c[l + 1], p.pitch[l + 1], var == 2);
            return launch_up_stream<T>(ctx->stream, p.bc, n, h.r[l], p.pitch[l], u, pu, f, pu,
                                       h.c[l + 1], p.pitch[l + 1], hs, add ? u64 : nullptr,
                                       p.pitch[0]);
          }, &mu));
          if (var < 2) mu += mp;
        }
        // A candidate replaces the current best only when it is more than 3%
        // faster, so that near-ties keep the default and choices stay stable.
        if (md < 0.97f * best_d) {
          best_d = md;
          c.down_var = var;
          c.down_hs = hs;
        }
        if (mu < 0.97f * best_u) {
          best_u = mu;
          c.up_var = var;
          c.up_hs = hs;
        }
      }
    us_total = 1e3f * (best_d + best_u);
    p.down_var[l] = c.down_var;
    p.down_hs[l] = c.down_hs;
    p.up_var[l] = c.up_var;
    p.up_hs[l] = c.up_hs;
    std::lock_guard<std::mutex> lk(tune_mutex());
    level_table()[key] = c;
    char line[256];
    std::snprintf(line, sizeof line, "L %s %s %d %d %d %d %d %d %.2f\n", arch.c_str(), prec, p.bc,
                  n, c.down_var, c.down_hs, c.up_var, c.up_hs, us_total);
    append_tune_file(ctx->opt.tune_cache_path, line);
  }
  // The level arrays used as stand-ins were overwritten: clear them again.
  for (int l = 0; l < p.levels; ++l) {
    if (h.u[l]) MG_HIP(launch_zero<T>(ctx->stream, p.side[l], h.u[l], p.pitch[l]));
    if (h.r[l]) MG_HIP(launch_zero<T>(ctx->stream, p.side[l], h.r[l], p.pitch[l]));
  }
  return MG_OK;
}

// Runs the autotuner for every problem (per-level kernels), then, for
// batches that may use it, picks the schedule by timing a few steps of each.
int32_t autotune(mg_ctx_s* ctx) {
  const bool mixed = ctx->opt.precision == MG_MIXED;
  const std::string arch = device_arch(ctx->device);
  {
    std::lock_guard<std::mutex> lk(tune_mutex());
    static std::string loaded;
    if (ctx->opt.tune_cache_path && loaded != ctx->opt.tune_cache_path) {
      load_tune_file(ctx->opt.tune_cache_path);
      loaded = ctx->opt.tune_cache_path;
    }
  }
  // Level-0 stand-ins: the largest level-0 shape of the batch.
  size_t elems = 0;
  int pitch0 = 0;
  for (const auto& p : ctx->probs) {
    elems = std::max(elems, (size_t)p.n * p.pitch[0]);
    pitch0 = std::max(pitch0, p.pitch[0]);
  }
  void* su = nullptr;
  void* sf = nullptr;
  const size_t bytes = elems * (mixed ? sizeof(float) : sizeof(double));
  if (hipMalloc(&su, bytes) != hipSuccess || hipMalloc(&sf, bytes) != hipSuccess) {
    if (su) (void)hipFree(su);
    (void)hipGetLastError();
    return fail(MG_ERR_OOM, "autotuner scratch allocation failed");
  }
  int32_t st = MG_OK;
  if (hipMemsetAsync(su, 0, bytes, ctx->stream) != hipSuccess ||
      hipMemsetAsync(sf, 0, bytes, ctx->stream) != hipSuccess)
    st = fail(MG_ERR_HIP, "autotuner scratch clear failed");
  for (auto& p : ctx->probs) {
    if (st != MG_OK) break;
    st = mixed ? tune_levels<float>(ctx, p, arch, (float*)su, (float*)sf, p.pitch[0])
               : tune_levels<double>(ctx, p, arch, (double*)su, (double*)sf, p.pitch[0]);
  }
  if (st == MG_OK && hipStreamSynchronize(ctx->stream) != hipSuccess)
    st = fail(MG_ERR_HIP, "autotuner synchronisation failed");
  (void)hipFree(su);
  (void)hipFree(sf);
  return st;
}

// Batch schedule: per-problem graphs against the persistent launch and
// against one launch per phase, each timed over a few steps on
// library-owned arrays of the callers' shapes.
int32_t tune_schedule(mg_ctx_s* ctx) {
  const int B = (int)ctx->probs.size();
  std::string why;
  if (B < 2 || !persistent_eligible(ctx, &why)) return MG_OK;
  const bool mixed = ctx->opt.precision == MG_MIXED;
  unsigned long long hsh = 1469598103934665603ULL;  // FNV-1a over the sizes
  for (const auto& p : ctx->probs) {
    hsh ^= (unsigned long long)p.n;
    hsh *= 1099511628211ULL;
  }
  char sig[64];
  std::snprintf(sig, sizeof sig, "B%d:%016llx", B, hsh);
  const std::string arch = device_arch(ctx->device);
  const char* prec = mixed ? "fp32" : "fp64";
  const int bc = ctx->probs[0].bc;
  const std::string key = arch + " " + prec + " " + std::to_string(bc) + " " + sig;
  int choice = -1;
  {
    std::lock_guard<std::mutex> lk(tune_mutex());
    auto it = schedule_table().find(key);
    if (it != schedule_table().end()) choice = it->second;
  }
  if (choice == 1) return MG_OK;
  MG_TRY(mixed ? build_persistent<float>(ctx) : build_persistent<double>(ctx));
  if (choice == 2 || choice == 3) {
    ctx->ps.phased = choice == 3;
    return MG_OK;
  }

  // Stand-in arrays (zeros: the work per step does not depend on values).
  std::vector<size_t> off(B + 1, 0);
  for (int b = 0; b < B; ++b)
    off[b + 1] = off[b] + ((size_t)ctx->probs[b].n * ctx->probs[b].pitch0 + 63) / 64 * 64;
  double* buf = nullptr;
  if (hipMalloc(&buf, 2 * off[B] * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return MG_OK;  // not enough memory to measure: keep the persistent schedule
  }
  std::vector<double*> us(B);
  std::vector<const double*> fs(B);
  for (int b = 0; b < B; ++b) {
    us[b] = buf + off[b];
    fs[b] = buf + off[B] + off[b];
  }
  int32_t st = MG_OK;
  float t_graph = 0.f, t_pers = 0.f, t_phased = 0.f;
  auto per_problem = [&]() -> hipError_t {
    for (int b = 0; b < B; ++b)
      if (run_step(ctx, ctx->probs[b], us[b], fs[b]) != MG_OK) return hipErrorUnknown;
    return hipSuccess;
  };
  auto persistent = [&]() -> hipError_t {
    if (persistent_bind(ctx, us.data(), fs.data(), {}) != MG_OK ||
        persistent_launch(ctx) != MG_OK)
      return hipErrorUnknown;
    return hipSuccess;
  };
  if (hipMemsetAsync(buf, 0, 2 * off[B] * sizeof(double), ctx->stream) != hipSuccess)
    st = fail(MG_ERR_HIP, "clear of the schedule stand-ins failed");
  if (st == MG_OK) st = time_launches(ctx, 2, per_problem, &t_graph);
  if (st == MG_OK) st = time_launches(ctx, 2, persistent, &t_pers);
  if (st == MG_OK) {
    std::vector<double> rel(B);
    st = persistent_relres(ctx, rel.data());  // also reports a timed-out barrier
  }
  if (st == MG_OK) {
    if (ctx->ps.graph) (void)hipGraphExecDestroy(ctx->ps.graph);
    ctx->ps.graph = nullptr;
    ctx->ps.phased = true;
    st = time_launches(ctx, 2, persistent, &t_phased);
    if (ctx->ps.graph) (void)hipGraphExecDestroy(ctx->ps.graph);
    ctx->ps.graph = nullptr;
    ctx->ps.phased = false;
  }
  for (auto& p : ctx->probs)
    for (auto& g : p.graph)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (st != MG_OK) return st;
  choice = t_pers < t_graph ? 2 : 1;
  if (t_phased < (choice == 2 ? t_pers : t_graph)) choice = 3;
  ctx->ps.phased = choice == 3;
  if (choice == 1) {
    if (ctx->ps.graph) (void)hipGraphExecDestroy(ctx->ps.graph);
    ctx->ps.graph = nullptr;
    ctx->ps.on = false;
  }
  std::lock_guard<std::mutex> lk(tune_mutex());
  schedule_table()[key] = choice;
  char line[256];
  std::snprintf(line, sizeof line, "S %s %s %d %s %d\n", arch.c_str(), prec, bc, sig, choice);
  append_tune_file(ctx->opt.tune_cache_path, line);
  return MG_OK;
}

int32_t destroy_ctx(mg_ctx_s* ctx) {
  if (!ctx) return MG_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& p : ctx->probs)
    for (auto g : p.graph)
      if (g) (void)hipGraphExecDestroy(g);
  if (ctx->ps.graph) (void)hipGraphExecDestroy(ctx->ps.graph);
  for (void* q : ctx->owned) (void)hipFree(q);
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->host) (void)hipHostFree(ctx->host);
  if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
  delete ctx;
  return MG_OK;
}

int32_t setup_impl(const mg_grid* grids, int32_t batch, const mg_options* opt, void* stream,
                   mg_ctx* out) {
  if (!out) return fail(MG_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!grids || !opt) return fail(MG_ERR_INVALID_ARG, "grids or opt is NULL");
  if (batch <= 0) return fail(MG_ERR_INVALID_ARG, "batch must be positive");
  if (opt->precision != MG_FP64 && opt->precision != MG_MIXED)
    return fail(MG_ERR_INVALID_ARG, "precision must be MG_FP64 or MG_MIXED");
  if (opt->nu_pre < 0 || opt->nu_pre > 8 || opt->nu_post < 0 || opt->nu_post > 8)
    return fail(MG_ERR_INVALID_ARG, "nu_pre/nu_post must be in 0..8");
  if (opt->inner_cycles < 1 || opt->inner_cycles > 8)
    return fail(MG_ERR_INVALID_ARG, "inner_cycles must be in 1..8");
  if (opt->prolong != MG_PROLONG_SPLINE && opt->prolong != MG_PROLONG_SRCNN)
    return fail(MG_ERR_INVALID_ARG, "unknown prolongation kind");
  if (opt->check_every < 0) return fail(MG_ERR_INVALID_ARG, "check_every must be >= 0");
  if (opt->kernel_path < 0 || opt->kernel_path > 2)
    return fail(MG_ERR_INVALID_ARG, "kernel_path must be 0, 1 or 2");
  if (opt->schedule < 0 || opt->schedule > 3)
    return fail(MG_ERR_INVALID_ARG, "schedule must be 0, 1 or 2");
  for (int b = 0; b < batch; ++b) {
    const mg_grid& g = grids[b];
    if (!valid_side(g.n))
      return fail(MG_ERR_INVALID_ARG, "problem " + std::to_string(b) + ": n=" +
                                          std::to_string(g.n) + " is not 4*2^k+1 in 5..16385");
    if (g.bc != MG_BC_DIRICHLET0 && g.bc != MG_BC_PERIODIC)
      return fail(MG_ERR_INVALID_ARG, "problem " + std::to_string(b) + ": bad boundary condition");
    if (g.pitch != 0 && (g.pitch < g.n || g.pitch > (1 << 24)))
      return fail(MG_ERR_INVALID_ARG, "problem " + std::to_string(b) + ": pitch < n");
    if (opt->prolong == MG_PROLONG_SRCNN && g.bc != MG_BC_PERIODIC)
      return fail(MG_ERR_UNSUPPORTED, "SR-CNN prolongation needs periodic grids");
  }
  if (opt->prolong == MG_PROLONG_SRCNN && (!opt->cnn_weights || opt->cnn_weights_bytes == 0))
    return fail(MG_ERR_UNSUPPORTED, "SR-CNN prolongation needs weights");
  if (opt->prolong == MG_PROLONG_SRCNN) {
    if (opt->cnn_weights_bytes != sizeof(float) * (size_t)MG_SRCNN_WEIGHT_COUNT)
      return fail(MG_ERR_INVALID_ARG, "SR-CNN weights must be " +
                                          std::to_string(MG_SRCNN_WEIGHT_COUNT) + " float32 values");
    if (opt->cnn_levels < 0 || opt->cnn_levels > kMaxLevels)
      return fail(MG_ERR_INVALID_ARG, "cnn_levels out of range");
    if (!(opt->cnn_max_ratio >= 0.0) || !(opt->cnn_min_relres >= 0.0))
      return fail(MG_ERR_INVALID_ARG, "cnn_max_ratio and cnn_min_relres must be >= 0");
  }
  if (!(opt->n_gan >= 0.0) || opt->n_gan > 1e9 || (opt->n_gan > 0.0 && opt->n_gan < 1e-9) ||
      !(opt->s_thres >= 0.0))
    return fail(MG_ERR_INVALID_ARG, "n_gan must be 0 or in [1e-9, 1e9], s_thres >= 0");
  if (opt->n_gan > 0.0 && opt->prolong != MG_PROLONG_SRCNN)
    return fail(MG_ERR_INVALID_ARG, "n_gan needs the SR-CNN prolongation");

  int ndev = 0;
  MG_HIP(hipGetDeviceCount(&ndev));
  if (ndev <= 0) return fail(MG_ERR_HIP, "no HIP device");

  mg_ctx_s* ctx = new (std::nothrow) mg_ctx_s();
  if (!ctx) return fail(MG_ERR_OOM, "host allocation failed");
  ctx->opt = *opt;
  ctx->stream = static_cast<hipStream_t>(stream);
  auto bail = [&](int32_t st) {
    std::string keep = g_last_error;
    destroy_ctx(ctx);
    g_last_error = keep;
    return st;
  };
  if (hipGetDevice(&ctx->device) != hipSuccess) return bail(fail(MG_ERR_HIP, "hipGetDevice"));
  if (hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(MG_ERR_HIP, "hipStreamCreateWithFlags"));
  if (hipHostMalloc((void**)&ctx->host, sizeof(double) * 8 * (size_t)batch) != hipSuccess)
    return bail(fail(MG_ERR_OOM, "hipHostMalloc"));
  {
    hipError_t e = fused_init();
    if (e != hipSuccess) return bail(fail(MG_ERR_HIP, std::string("fused_init: ") + hipGetErrorString(e)));
  }

  for (int bc = 0; bc < 2; ++bc) {
    double tbl[kTailMatOffset + kTailMatElems];
    coarsest_inverse(bc, tbl);
    for (int nc : {5, 9, 17, 33}) prefilter_matrix(nc, bc, tbl + kTailMatOffset + tail_mat_offset(nc));
    int32_t st = alloc_level<double>(ctx, 1, kTailMatOffset + kTailMatElems, &ctx->inv[bc]);
    if (st != MG_OK) return bail(st);
    if (hipMemcpyAsync(ctx->inv[bc], tbl, sizeof tbl, hipMemcpyHostToDevice, ctx->stream) !=
        hipSuccess)
      return bail(fail(MG_ERR_HIP, "copy of the coarsest inverse"));
    if (hipStreamSynchronize(ctx->stream) != hipSuccess)
      return bail(fail(MG_ERR_HIP, "hipStreamSynchronize"));
  }

  ctx->probs.resize(batch);
  CallerArgs* slots = nullptr;
  {
    int32_t st = alloc_level<CallerArgs>(ctx, 1, batch, &slots);
    if (st != MG_OK) return bail(st);
  }
  for (int b = 0; b < batch; ++b) {
    Problem& p = ctx->probs[b];
    p.caller = slots + b;
    p.n = grids[b].n;
    p.bc = grids[b].bc;
    p.pitch0 = grids[b].pitch ? grids[b].pitch : grids[b].n;
    for (int n = p.n;; n = (n - 1) / 2 + 1) {
      p.side.push_back(n);
      p.pitch.push_back(pitch_for(n));
      if (n == 5) break;
    }
    p.levels = (int)p.side.size();
    const int L = p.levels;
    p.taps64.resize(L);
    p.taps32.resize(L);
    for (int l = 0; l < L; ++l) {
      spline_taps(p.side[l], p.bc, kPrefilterHalfTapsF64, &p.taps64[l]);
      spline_taps(p.side[l], p.bc, kPrefilterHalfTapsF32, &p.taps32[l]);
    }
    p.tail = 0;
    while (p.side[p.tail] > kTailMaxSide) ++p.tail;
    p.down_var.assign(L, 0);
    p.up_var.assign(L, 0);
    p.down_hs.assign(L, 0);
    p.up_hs.assign(L, 0);
    {
      const size_t tb = sizeof(PrefilterTaps) * (size_t)L;
      unsigned char* d = nullptr;
      int32_t st = alloc_level<unsigned char>(ctx, 2, (int)tb, &d);
      if (st != MG_OK) return bail(st);
      p.taps64_dev = reinterpret_cast<PrefilterTaps*>(d);
      p.taps32_dev = reinterpret_cast<PrefilterTaps*>(d + tb);
      if (hipMemcpyAsync(p.taps64_dev, p.taps64.data(), tb, hipMemcpyHostToDevice, ctx->stream) !=
              hipSuccess ||
          hipMemcpyAsync(p.taps32_dev, p.taps32.data(), tb, hipMemcpyHostToDevice, ctx->stream) !=
              hipSuccess)
        return bail(fail(MG_ERR_HIP, "copy of the prefilter tables"));
    }
    auto& h = p.h64;
    h.u.assign(L, nullptr);
    h.f.assign(L, nullptr);
    h.r.assign(L, nullptr);
    h.c.assign(L, nullptr);
    h.tmp.assign(L, nullptr);
    for (int l = 0; l < L; ++l) {
      const int n = p.side[l], pt = p.pitch[l];
      int32_t st = alloc_level<double>(ctx, n, pt, &h.r[l]);
      if (st == MG_OK && l > 0) st = alloc_level<double>(ctx, n, pt, &h.u[l]);
      if (st == MG_OK && l > 0) st = alloc_level<double>(ctx, n, pt, &h.f[l]);
      if (st == MG_OK && l > 0) st = alloc_level<double>(ctx, n, pt, &h.c[l]);
      if (st == MG_OK && l > 0) st = alloc_level<double>(ctx, n, pt, &h.tmp[l]);
      if (st != MG_OK) return bail(st);
    }
    if (opt->precision == MG_MIXED) {
      auto& g = p.h32;
      g.u.assign(L, nullptr);
      g.f.assign(L, nullptr);
      g.r.assign(L, nullptr);
      g.c.assign(L, nullptr);
      g.tmp.assign(L, nullptr);
      for (int l = 0; l < L; ++l) {
        const int n = p.side[l], pt = p.pitch[l];
        int32_t st = alloc_level<float>(ctx, n, pt, &g.u[l]);
        if (st == MG_OK) st = alloc_level<float>(ctx, n, pt, &g.f[l]);
        if (st == MG_OK) st = alloc_level<float>(ctx, n, pt, &g.r[l]);
        if (st == MG_OK && l > 0) st = alloc_level<float>(ctx, n, pt, &g.c[l]);
        if (st == MG_OK && l > 0) st = alloc_level<float>(ctx, n, pt, &g.tmp[l]);
        if (st != MG_OK) return bail(st);
      }
    }
    p.nblocks = std::max(blocks_for(p.n, p.bc), (int)((p.n + 63) / 64) * ((p.n + 3) / 4));
    int32_t st = alloc_level<double>(ctx, 2, p.nblocks, &p.partials);
    if (st == MG_OK) st = alloc_level<double>(ctx, 1, 4, &p.sums);
    if (st == MG_OK && opt->n_gan > 0.0 && opt->s_thres > 0.0)
      st = alloc_level<double>(ctx, p.n, p.n, &p.uprev);
    if (st != MG_OK) return bail(st);
  }
  if (opt->prolong == MG_PROLONG_SRCNN) {
    const int32_t st = cnn_setup(ctx, static_cast<const float*>(opt->cnn_weights));
    if (st != MG_OK) return bail(st);
  }
  ctx->opt.cnn_weights = nullptr;  // copied; the caller's blob is not retained
  if (hipStreamSynchronize(ctx->stream) != hipSuccess)
    return bail(fail(MG_ERR_HIP, "hipStreamSynchronize after setup"));
  if (opt->schedule == 0 && opt->kernel_path == 0) {
    int32_t st = autotune(ctx);
    if (st == MG_OK) st = tune_schedule(ctx);
    if (st != MG_OK) return bail(st);
  }
  if (opt->schedule == 2 || opt->schedule == 3) {
    std::string why;
    if (!persistent_eligible(ctx, &why)) return bail(fail(MG_ERR_UNSUPPORTED, why));
    const int32_t st = opt->precision == MG_MIXED ? build_persistent<float>(ctx)
                                                  : build_persistent<double>(ctx);
    if (st != MG_OK) return bail(st);
    ctx->ps.phased = opt->schedule == 3;
  }
  *out = ctx;
  return MG_OK;
}

int32_t check_ctx_arrays(mg_ctx ctx, double* const* u, const double* const* f) {
  if (!ctx) return fail(MG_ERR_INVALID_ARG, "ctx is NULL");
  if (!u || !f) return fail(MG_ERR_INVALID_ARG, "u or f is NULL");
  for (size_t b = 0; b < ctx->probs.size(); ++b)
    if (!u[b] || !f[b]) return fail(MG_ERR_INVALID_ARG, "u[" + std::to_string(b) + "] or f is NULL");
  return MG_OK;
}

// Reads p.sums[0..1] of every listed problem into relres[b] (host sync),
// and with `diff` also sqrt(p.sums[2]) into diff[b].
int32_t read_relres(mg_ctx ctx, const std::vector<int>& which, double* relres,
                    double* diff = nullptr) {
  const int w = diff ? 3 : 2;
  for (size_t k = 0; k < which.size(); ++k)
    MG_HIP(hipMemcpyAsync(ctx->host + w * k, ctx->probs[which[k]].sums, w * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->stream));
  MG_HIP(hipStreamSynchronize(ctx->stream));
  for (size_t k = 0; k < which.size(); ++k) {
    const double rr = ctx->host[w * k], ff = ctx->host[w * k + 1];
    relres[k] = ff > 0.0 ? std::sqrt(rr) / std::sqrt(ff) : std::sqrt(rr);
    if (diff) diff[k] = std::sqrt(ctx->host[w * k + 2]);
  }
  return MG_OK;
}

// ||u - uprev||^2 over the unknowns into p.sums[2], and uprev = u.
int32_t enqueue_diffnorm(mg_ctx_s* ctx, Problem& p, const double* u) {
  int nb = 0;
  MG_HIP(launch_diffnorm(ctx->stream, p.bc, p.n, u, p.pitch0, p.uprev, p.n, p.partials, &nb));
  MG_HIP(launch_reduce(ctx->stream, p.partials, nb, nb, 1, p.sums + 2));
  return MG_OK;
}

int32_t vcycle_impl(mg_ctx ctx, double* const* u, const double* const* f, int32_t ncycles,
                    double* relres_out) {
  MG_TRY(check_ctx_arrays(ctx, u, f));
  if (ncycles < 0) return fail(MG_ERR_INVALID_ARG, "ncycles < 0");
  MG_HIP(hipSetDevice(ctx->device));
  const int B = (int)ctx->probs.size();
  if (ctx->ps.on) {
    MG_TRY(persistent_bind(ctx, u, f, {}));
    for (int c = 0; c < ncycles; ++c) MG_TRY(persistent_launch(ctx));
    if (ctx->ps.bc == kPeriodic && ncycles > 0)
      MG_HIP(launch_seam_batched(ctx->stream, ctx->ps.d_probs, B));
    // The persistent launch's barrier may have timed out: read its error
    // word (synchronises).  The phased schedule has no barrier and returns
    // after queueing.
    if (!relres_out) return (ncycles > 0 && !ctx->ps.phased) ? persistent_check(ctx) : MG_OK;
    MG_TRY(persistent_relres(ctx, relres_out));
    for (int b = 0; b < B; ++b)
      if (!std::isfinite(relres_out[b])) return fail(MG_ERR_NONFINITE, "non-finite residual");
    return MG_OK;
  }
  for (int c = 0; c < ncycles; ++c)
    for (int b = 0; b < B; ++b) MG_TRY(run_step(ctx, ctx->probs[b], u[b], f[b], cnn_cycles(ctx)));
  if (!relres_out) return MG_OK;
  std::vector<int> all(B);
  for (int b = 0; b < B; ++b) {
    all[b] = b;
    MG_TRY(enqueue_resnorm(ctx, ctx->probs[b], u[b], f[b]));
  }
  MG_TRY(read_relres(ctx, all, relres_out));
  for (int b = 0; b < B; ++b)
    if (!std::isfinite(relres_out[b])) return fail(MG_ERR_NONFINITE, "non-finite residual");
  return MG_OK;
}

int32_t solve_impl(mg_ctx ctx, double* const* u, const double* const* f, double rtol,
                   int32_t max_cycles, int32_t* cycles_out, double* relres_out) {
  MG_TRY(check_ctx_arrays(ctx, u, f));
  if (!(rtol >= 0.0)) return fail(MG_ERR_INVALID_ARG, "rtol must be >= 0");
  if (max_cycles < 0) return fail(MG_ERR_INVALID_ARG, "max_cycles < 0");
  MG_HIP(hipSetDevice(ctx->device));
  const int B = (int)ctx->probs.size();

  // Periodic right-hand sides must have zero mean (the constants are the
  // null space of A).
  {
    std::vector<int> per;
    for (int b = 0; b < B; ++b) {
      Problem& p = ctx->probs[b];
      if (p.bc != kPeriodic) continue;
      int nb = 0;
      MG_HIP(launch_rhs_moments(ctx->stream, p.bc, p.n, f[b], p.pitch0, p.partials, &nb));
      MG_HIP(launch_reduce(ctx->stream, p.partials, nb, nb, 2, p.sums));
      per.push_back(b);
    }
    for (size_t k = 0; k < per.size(); ++k)
      MG_HIP(hipMemcpyAsync(ctx->host + 2 * k, ctx->probs[per[k]].sums, 2 * sizeof(double),
                            hipMemcpyDeviceToHost, ctx->stream));
    MG_HIP(hipStreamSynchronize(ctx->stream));
    for (size_t k = 0; k < per.size(); ++k) {
      const Problem& p = ctx->probs[per[k]];
      const double M = (double)(p.n - 1) * (double)(p.n - 1);
      const double sum = ctx->host[2 * k], sq = ctx->host[2 * k + 1];
      if (!std::isfinite(sum) || !std::isfinite(sq))
        return fail(MG_ERR_NONFINITE, "non-finite right-hand side");
      if (std::fabs(sum) > 1e-10 * std::sqrt(M) * std::sqrt(sq))
        return fail(MG_ERR_INCOMPATIBLE_RHS,
                    "periodic f of problem " + std::to_string(per[k]) + " has nonzero mean");
    }
  }

  std::vector<int> cycles(B, 0), state(B, 1);  // state: 1 active, 0 converged, <0 failure
  std::vector<double> rel(B, 0.0), prev(B, -1.0);
  std::vector<int> prev_cycles(B, 0), slow(B, 0), next_check(B, 1), all(B);
  const bool pers = ctx->ps.on;
  // Mixed path: every norm check is the FP64 residual the next step needs
  // anyway (have_res: the next step of b skips it).
  const bool mixed_chk = !pers && ctx->opt.precision == MG_MIXED;
  std::vector<char> have_res(B, 0);
  for (int b = 0; b < B; ++b) all[b] = b;
  if (pers) {
    MG_TRY(persistent_bind(ctx, u, f, {}));
    MG_TRY(persistent_relres(ctx, rel.data()));
  } else if (mixed_chk) {
    for (int b = 0; b < B; ++b) {
      // Periodic problems: the right-hand-side check above left ||f||^2 in
      // p.sums[1] already (the same kernel and reduction).
      if (ctx->probs[b].bc != kPeriodic) MG_TRY(enqueue_fnorm(ctx, ctx->probs[b], f[b]));
      MG_TRY(enqueue_check_mixed(ctx, ctx->probs[b], u[b], f[b]));
      have_res[b] = 1;
    }
    MG_TRY(read_relres(ctx, all, rel.data()));
  } else {
    for (int b = 0; b < B; ++b) MG_TRY(enqueue_resnorm(ctx, ctx->probs[b], u[b], f[b]));
    MG_TRY(read_relres(ctx, all, rel.data()));
  }
  for (int b = 0; b < B; ++b) {
    if (!std::isfinite(rel[b])) state[b] = MG_ERR_NONFINITE;
    else if (rel[b] <= rtol) state[b] = 0;
    else if (max_cycles == 0) state[b] = MG_ERR_NOT_CONVERGED;
    prev[b] = rel[b];
  }
  const int every = ctx->opt.check_every;
  // Network-prolongated cycles until a cycle's residual ratio exceeds
  // cnn_max_ratio or the residual reaches cnn_min_relres; checked after every
  // such cycle.
  std::vector<char> cnn_on(B, cnn_cycles(ctx) ? 1 : 0);
  // Hybrid schedule (n_gan > 0) in place of that rule: cycle i of this call
  // takes the second operator when i is a multiple of N + 1 or when the
  // previous cycle changed u by at most s_thres, else the first; with
  // s_thres > 0 that change is measured and every cycle is checked.
  const bool sched = ctx->opt.n_gan > 0.0 && cnn_cycles(ctx);
  const bool track = sched && ctx->opt.s_thres > 0.0;
  const bool net_first = ctx->opt.n_gan >= 1.0;
  const long long nper =
      sched ? std::llround(net_first ? ctx->opt.n_gan : 1.0 / ctx->opt.n_gan) + 1 : 1;
  std::vector<char> sw(B, 0);
  if (sched) std::fill(cnn_on.begin(), cnn_on.end(), 0);
  auto use_net = [&](int b) -> bool {
    if (!sched) return cnn_on[b] != 0;
    const long long i = (long long)cycles[b] + 1;
    return (i % nper != 0 && !sw[b]) ? net_first : !net_first;
  };
  for (int b = 0; b < B; ++b) {
    ctx->probs[b].hist_op.clear();
    ctx->probs[b].hist_diff.clear();
    if (track && state[b] == 1) MG_TRY(enqueue_diffnorm(ctx, ctx->probs[b], u[b]));
  }
  std::vector<double> dif(B, 0.0);
  for (;;) {
    std::vector<int> act;
    for (int b = 0; b < B; ++b)
      if (state[b] == 1) act.push_back(b);
    if (act.empty()) break;
    // Cycle every active problem up to the earliest next check.
    int steps = 1 << 30;
    for (int b : act) steps = std::min(steps, next_check[b] - cycles[b]);
    steps = std::max(steps, 1);
    for (int k = 0; k < steps; ++k) {
      if (pers) {
        std::vector<int> on(B, 0);
        bool any = false;
        for (int b : act)
          if (cycles[b] < max_cycles && cycles[b] < next_check[b]) {
            on[b] = 1;
            any = true;
            ++cycles[b];
            ctx->probs[b].hist_op.push_back(MG_PROLONG_SPLINE);
            ctx->probs[b].hist_diff.push_back(NAN);
          }
        if (any) {
          MG_TRY(persistent_bind(ctx, u, f, on));
          MG_TRY(persistent_launch(ctx));
        }
        continue;
      }
      for (int b : act)
        if (cycles[b] < max_cycles && cycles[b] < next_check[b]) {
          const bool net = use_net(b);
          Problem& p = ctx->probs[b];
          MG_TRY(run_step(ctx, p, u[b], f[b], net, have_res[b] != 0));
          if (track) MG_TRY(enqueue_diffnorm(ctx, p, u[b]));
          p.hist_op.push_back(net ? MG_PROLONG_SRCNN : MG_PROLONG_SPLINE);
          p.hist_diff.push_back(NAN);
          have_res[b] = 0;
          ++cycles[b];
        }
    }
    std::vector<int> chk;
    for (int b : act)
      if (cycles[b] >= next_check[b] || cycles[b] >= max_cycles) chk.push_back(b);
    std::vector<double> r(chk.size());
    if (pers) {
      std::vector<double> rall(B);
      MG_TRY(persistent_relres(ctx, rall.data()));
      for (size_t k = 0; k < chk.size(); ++k) r[k] = rall[chk[k]];
    } else if (mixed_chk) {
      for (int b : chk) {
        MG_TRY(enqueue_check_mixed(ctx, ctx->probs[b], u[b], f[b]));
        have_res[b] = 1;
      }
      MG_TRY(read_relres(ctx, chk, r.data(), track ? dif.data() : nullptr));
    } else {
      for (int b : chk) MG_TRY(enqueue_resnorm(ctx, ctx->probs[b], u[b], f[b]));
      MG_TRY(read_relres(ctx, chk, r.data(), track ? dif.data() : nullptr));
    }
    for (size_t k = 0; k < chk.size(); ++k) {
      const int b = chk[k];
      const double rr = r[k], last = prev[b];
      const int span = cycles[b] - prev_cycles[b];
      rel[b] = rr;
      if (track && !ctx->probs[b].hist_diff.empty()) {  // one cycle per check
        ctx->probs[b].hist_diff.back() = dif[k];
        sw[b] = dif[k] <= ctx->opt.s_thres ? 1 : 0;
      }
      if (!std::isfinite(rr)) {
        state[b] = MG_ERR_NONFINITE;
        continue;
      }
      if (rr <= rtol) {
        state[b] = 0;
        continue;
      }
      // Stagnation: three checks in a row each with less than 10% reduction
      // per cycle.
      const double rate = span > 0 && last > 0.0 ? std::pow(rr / last, 1.0 / span) : 1.0;
      slow[b] = rate > 0.9 ? slow[b] + 1 : 0;
      bool switched = false;
      if (cnn_on[b] && (rate > ctx->opt.cnn_max_ratio || rr <= ctx->opt.cnn_min_relres)) {
        cnn_on[b] = 0;
        switched = true;  // the rate seen so far is not the spline cycle's
      }
      prev[b] = rr;
      prev_cycles[b] = cycles[b];
      if (slow[b] >= 3) {
        state[b] = MG_ERR_STAGNATED;
        continue;
      }
      if (cycles[b] >= max_cycles) {
        state[b] = MG_ERR_NOT_CONVERGED;
        continue;
      }
      // Next check: every `every` cycles, or (auto) at the cycle where the
      // observed rate predicts the tolerance is crossed, at most 8 ahead.
      int gap = 1;
      if (track || cnn_on[b] || switched) {
        gap = 1;
      } else if (every > 0) {
        gap = every;
      } else if (rate > 0.0 && rate < 0.9) {
        const double need = std::log(rtol / rr) / std::log(rate);
        gap = std::max(1, std::min(8, (int)std::ceil(need - 0.25)));
      }
      next_check[b] = cycles[b] + gap;
    }
  }
  // Periodic results: zero mean and rewritten seam.
  for (int b = 0; b < B; ++b) {
    Problem& p = ctx->probs[b];
    if (p.bc != kPeriodic || cycles[b] == 0) continue;
    int nb = 0;
    MG_HIP(launch_sum(ctx->stream, p.bc, p.n, u[b], p.pitch0, p.partials, &nb));
    MG_HIP(launch_reduce(ctx->stream, p.partials, nb, nb, 1, p.sums + 2));
    MG_HIP(launch_remove_mean(ctx->stream, p.n, u[b], p.pitch0, p.sums + 2));
  }
  MG_HIP(hipStreamSynchronize(ctx->stream));
  int32_t status = MG_OK;
  for (int b = 0; b < B; ++b) {
    if (cycles_out) cycles_out[b] = cycles[b];
    if (relres_out) relres_out[b] = rel[b];
    if (state[b] < 0 && status == MG_OK) status = state[b];
  }
  if (status != MG_OK) fail(status, mg_status_string(status));
  return status;
}

template <typename T>
int32_t step_common(mg_ctx ctx, int32_t problem, int32_t level, Problem** pp) {
  if (!ctx) return fail(MG_ERR_INVALID_ARG, "ctx is NULL");
  if (problem < 0 || problem >= (int)ctx->probs.size())
    return fail(MG_ERR_INVALID_ARG, "problem index out of range");
  Problem& p = ctx->probs[problem];
  if (level < 0 || level >= p.levels) return fail(MG_ERR_INVALID_ARG, "level out of range");
  *pp = &p;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(MG_ERR_HIP, "hipSetDevice");
  return MG_OK;
}

template <typename T>
int32_t relax_t(mg_ctx ctx, int32_t problem, int32_t level, void* u, const void* f, int32_t colour,
                int32_t count) {
  Problem* p;
  MG_TRY(step_common<T>(ctx, problem, level, &p));
  if (!u || !f) return fail(MG_ERR_INVALID_ARG, "NULL array");
  if ((colour != 0 && colour != 1) || count < 0) return fail(MG_ERR_INVALID_ARG, "bad colour/count");
  const int n = p->side[level];
  MG_HIP(launch_relax<T>(ctx->stream, p->bc, n, (T*)u, n, (const T*)f, n, colour, count));
  if (p->bc == kPeriodic) MG_HIP(launch_seam<T>(ctx->stream, n, (T*)u, n));
  return MG_OK;
}

template <typename T>
int32_t residual_t(mg_ctx ctx, int32_t problem, int32_t level, const void* u, const void* f,
                   void* r) {
  Problem* p;
  MG_TRY(step_common<T>(ctx, problem, level, &p));
  if (!u || !f || !r) return fail(MG_ERR_INVALID_ARG, "NULL array");
  const int n = p->side[level];
  MG_HIP(launch_residual<T>(ctx->stream, p->bc, n, (const T*)u, n, (const T*)f, n, (T*)r, n));
  return MG_OK;
}

template <typename T>
int32_t restrict_t(mg_ctx ctx, int32_t problem, int32_t level, const void* r, void* fc) {
  Problem* p;
  MG_TRY(step_common<T>(ctx, problem, level, &p));
  if (!r || !fc) return fail(MG_ERR_INVALID_ARG, "NULL array");
  if (level + 1 >= p->levels) return fail(MG_ERR_INVALID_ARG, "no coarser level");
  const int n = p->side[level], nc = p->side[level + 1];
  MG_HIP(launch_restrict<T>(ctx->stream, p->bc, n, (const T*)r, n, (T*)fc, nc));
  return MG_OK;
}

template <typename T>
int32_t coarse_t(mg_ctx ctx, int32_t problem, const void* f, void* u) {
  Problem* p;
  MG_TRY(step_common<T>(ctx, problem, 0, &p));
  if (!u || !f) return fail(MG_ERR_INVALID_ARG, "NULL array");
  MG_HIP(launch_coarse<T>(ctx->stream, p->bc, (const T*)f, 5, (T*)u, 5, ctx->inv[p->bc]));
  return MG_OK;
}

template <typename T>
int32_t prolong_t(mg_ctx ctx, int32_t problem, int32_t coarse_level, int32_t kind,
                  const void* coarse, void* fine) {
  Problem* p;
  MG_TRY(step_common<T>(ctx, problem, coarse_level, &p));
  if (coarse_level < 1) return fail(MG_ERR_INVALID_ARG, "coarse_level must be >= 1");
  if (!coarse || !fine) return fail(MG_ERR_INVALID_ARG, "NULL array");
  const int nc = p->side[coarse_level], n = p->side[coarse_level - 1];
  const int pc = p->pitch[coarse_level];
  if (kind == MG_PROLONG_SRCNN) {
    if (!ctx->cnn.on) return fail(MG_ERR_UNSUPPORTED, "no SR-CNN weights were given at setup");
    const int N = nc - 1;
    if (N < 32 || N % 32 != 0 || N > ctx->cnn.max_n)
      return fail(MG_ERR_UNSUPPORTED, "SR-CNN needs a coarse unique side that is a multiple of 32");
    return enqueue_cnn<T>(ctx, ctx->stream, coarse_level - 1, N, (const T*)coarse, nc, nullptr, 0,
                          (T*)fine, n);
  }
  // Workspace: the FP64 hierarchy's coefficient arrays of that level (their
  // byte size also covers FP32 data with the same element pitch).
  T* tmp = reinterpret_cast<T*>(p->h64.tmp[coarse_level]);
  T* c = reinterpret_cast<T*>(p->h64.c[coarse_level]);
  const PrefilterTaps& taps =
      sizeof(T) == 8 ? p->taps64[coarse_level] : p->taps32[coarse_level];
  MG_HIP(launch_prefilter<T>(ctx->stream, p->bc, nc, taps, (const T*)coarse, nc, tmp, pc, c, pc));
  MG_HIP(launch_prolong<T>(ctx->stream, p->bc, n, (T*)fine, n, c, pc, false));
  return MG_OK;
}

#define MG_GUARD(body)                                              \
  try {                                                             \
    body                                                            \
  } catch (const std::bad_alloc&) {                                 \
    return fail(MG_ERR_OOM, "host allocation failed");              \
  } catch (...) {                                                   \
    return fail(MG_ERR_HIP, "unexpected exception");                \
  }

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

void mg_options_default(mg_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof *opt);
  opt->precision = MG_FP64;
  opt->nu_pre = 2;
  opt->nu_post = 2;
  opt->inner_cycles = 1;
  opt->prolong = MG_PROLONG_SPLINE;
  opt->cnn_levels = 2;
  opt->check_every = 0;
  opt->use_graph = 1;
  opt->tune_cache_path = nullptr;
  opt->kernel_path = 0;
  opt->schedule = 0;
  opt->cnn_max_ratio = 0.5;
  opt->cnn_min_relres = 1e-7;
  opt->n_gan = 0.0;
  opt->s_thres = 0.0;
}

int32_t mg_setup(const mg_grid* grids, int32_t batch, const mg_options* opt, void* hip_stream,
                 mg_ctx* out) {
  g_last_error.clear();
  MG_GUARD(return setup_impl(grids, batch, opt, hip_stream, out);)
}

int32_t mg_vcycle(mg_ctx ctx, double* const* u, const double* const* f, int32_t ncycles,
                  double* relres_out) {
  g_last_error.clear();
  MG_GUARD(return vcycle_impl(ctx, u, f, ncycles, relres_out);)
}

int32_t mg_solve(mg_ctx ctx, double* const* u, const double* const* f, double rtol,
                 int32_t max_cycles, int32_t* cycles_out, double* relres_out) {
  g_last_error.clear();
  MG_GUARD(return solve_impl(ctx, u, f, rtol, max_cycles, cycles_out, relres_out);)
}

int32_t mg_prolong(mg_ctx ctx, int32_t problem, int32_t coarse_level, int32_t kind,
                   const void* coarse, void* fine, int32_t dtype) {
  g_last_error.clear();
  if (kind != MG_PROLONG_SPLINE && kind != MG_PROLONG_SRCNN)
    return fail(MG_ERR_INVALID_ARG, "unknown prolongation kind");
  MG_GUARD(if (dtype == MG_DT_F64)
               return prolong_t<double>(ctx, problem, coarse_level, kind, coarse, fine);
           if (dtype == MG_DT_F32)
               return prolong_t<float>(ctx, problem, coarse_level, kind, coarse, fine);
           return fail(MG_ERR_INVALID_ARG, "bad dtype");)
}

int32_t mg_relax(mg_ctx ctx, int32_t problem, int32_t level, void* u, const void* f,
                 int32_t colour, int32_t count, int32_t dtype) {
  g_last_error.clear();
  MG_GUARD(if (dtype == MG_DT_F64) return relax_t<double>(ctx, problem, level, u, f, colour, count);
           if (dtype == MG_DT_F32) return relax_t<float>(ctx, problem, level, u, f, colour, count);
           return fail(MG_ERR_INVALID_ARG, "bad dtype");)
}

int32_t mg_residual(mg_ctx ctx, int32_t problem, int32_t level, const void* u, const void* f,
                    void* r, int32_t dtype) {
  g_last_error.clear();
  MG_GUARD(if (dtype == MG_DT_F64) return residual_t<double>(ctx, problem, level, u, f, r);
           if (dtype == MG_DT_F32) return residual_t<float>(ctx, problem, level, u, f, r);
           return fail(MG_ERR_INVALID_ARG, "bad dtype");)
}

int32_t mg_restrict(mg_ctx ctx, int32_t problem, int32_t level, const void* r, void* fc,
                    int32_t dtype) {
  g_last_error.clear();
  MG_GUARD(if (dtype == MG_DT_F64) return restrict_t<double>(ctx, problem, level, r, fc);
           if (dtype == MG_DT_F32) return restrict_t<float>(ctx, problem, level, r, fc);
           return fail(MG_ERR_INVALID_ARG, "bad dtype");)
}

int32_t mg_coarse_solve(mg_ctx ctx, int32_t problem, const void* f, void* u, int32_t dtype) {
  g_last_error.clear();
  MG_GUARD(if (dtype == MG_DT_F64) return coarse_t<double>(ctx, problem, f, u);
           if (dtype == MG_DT_F32) return coarse_t<float>(ctx, problem, f, u);
           return fail(MG_ERR_INVALID_ARG, "bad dtype");)
}

namespace mg {
namespace {
int32_t ns_check(int32_t n, int32_t pitch, int32_t dtype, std::initializer_list<const void*> in,
                 std::initializer_list<const void*> out) {
  if (!valid_side(n)) return fail(MG_ERR_INVALID_ARG, "n is not 4*2^k+1 in 5..16385");
  if (pitch < n) return fail(MG_ERR_INVALID_ARG, "pitch < n");
  if (dtype != MG_DT_F64 && dtype != MG_DT_F32) return fail(MG_ERR_INVALID_ARG, "bad dtype");
  for (const void* a : in)
    if (!a) return fail(MG_ERR_INVALID_ARG, "NULL array");
  for (const void* a : out) {
    if (!a) return fail(MG_ERR_INVALID_ARG, "NULL array");
    for (const void* b : in)
      if (a == b) return fail(MG_ERR_INVALID_ARG, "an output aliases an input");
  }
  return MG_OK;
}
}  // namespace
}  // namespace mg

int32_t mg_ns_rhs(int32_t n, const void* ux, const void* uy, void* f, int32_t pitch,
                  int32_t dtype, void* hip_stream) {
  g_last_error.clear();
  MG_GUARD(MG_TRY(ns_check(n, pitch, dtype, {ux, uy}, {f}));
           const hipStream_t s = static_cast<hipStream_t>(hip_stream);
           if (dtype == MG_DT_F64) MG_HIP(launch_ns_rhs<double>(
               s, n, static_cast<const double*>(ux), static_cast<const double*>(uy),
               static_cast<double*>(f), pitch));
           else MG_HIP(launch_ns_rhs<float>(s, n, static_cast<const float*>(ux),
                                            static_cast<const float*>(uy),
                                            static_cast<float*>(f), pitch));
           return MG_OK;)
}

int32_t mg_ns_update(int32_t n, const void* ux, const void* uy, const void* q, double dt,
                     void* ux_out, void* uy_out, int32_t pitch, int32_t dtype, void* hip_stream) {
  g_last_error.clear();
  MG_GUARD(MG_TRY(ns_check(n, pitch, dtype, {ux, uy, q}, {ux_out, uy_out}));
           if (ux_out == uy_out) return fail(MG_ERR_INVALID_ARG, "ux_out == uy_out");
           if (!std::isfinite(dt)) return fail(MG_ERR_INVALID_ARG, "dt is not finite");
           const hipStream_t s = static_cast<hipStream_t>(hip_stream);
           if (dtype == MG_DT_F64) MG_HIP(launch_ns_update<double>(
               s, n, static_cast<const double*>(ux), static_cast<const double*>(uy),
               static_cast<const double*>(q), dt, static_cast<double*>(ux_out),
               static_cast<double*>(uy_out), pitch));
           else MG_HIP(launch_ns_update<float>(
               s, n, static_cast<const float*>(ux), static_cast<const float*>(uy),
               static_cast<const float*>(q), dt, static_cast<float*>(ux_out),
               static_cast<float*>(uy_out), pitch));
           return MG_OK;)
}

int32_t mg_timing_enable(mg_ctx ctx, int32_t enable) {
  g_last_error.clear();
  if (!ctx) return fail(MG_ERR_INVALID_ARG, "ctx is NULL");
  MG_HIP(hipStreamSynchronize(ctx->stream));
  ctx->recs.clear();
  ctx->pool_used = 0;
  ctx->timing = enable != 0;
  return MG_OK;
}

int32_t mg_graph_stats(mg_ctx ctx, int64_t* captures, int64_t* instantiations) {
  g_last_error.clear();
  if (!ctx) return fail(MG_ERR_INVALID_ARG, "ctx is NULL");
  if (captures) *captures = ctx->graph_captures;
  if (instantiations) *instantiations = ctx->graph_instantiations;
  return MG_OK;
}

int32_t mg_timing_read(mg_ctx ctx, int32_t kind, int32_t level, int64_t* launches,
                       double* total_ms, double* bytes) {
  g_last_error.clear();
  if (!ctx) return fail(MG_ERR_INVALID_ARG, "ctx is NULL");
  if (kind < 0 || kind >= MG_K_COUNT) return fail(MG_ERR_INVALID_ARG, "bad kernel class");
  MG_HIP(hipStreamSynchronize(ctx->stream));
  int64_t cnt = 0;
  double ms = 0.0, by = 0.0;
  for (const auto& r : ctx->recs) {
    if (r.kind != kind || (level >= 0 && r.level != level)) continue;
    float t = 0.f;
    MG_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ++cnt;
    ms += t;
    by += r.bytes;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  if (bytes) *bytes = by;
  return MG_OK;
}

const char* mg_kernel_name(int32_t kind) {
  switch (kind) {
    case MG_K_RELAX: return "relax";
    case MG_K_RESIDUAL: return "residual";
    case MG_K_RESTRICT: return "restrict";
    case MG_K_PREFILTER: return "prefilter";
    case MG_K_PROLONG: return "prolong";
    case MG_K_COARSE: return "coarse";
    case MG_K_RESIDUAL_MIXED: return "residual_mixed";
    case MG_K_UPDATE_MIXED: return "update_mixed";
    case MG_K_RESNORM: return "resnorm";
    case MG_K_ZERO: return "zero";
    case MG_K_DOWN: return "down";
    case MG_K_UP: return "up";
    case MG_K_TAIL: return "tail";
    case MG_K_PERSISTENT: return "persistent";
    case MG_K_CNN: return "cnn_conv";
    case MG_K_CNN_AUX: return "cnn_aux";
    case MG_K_PHASED: return "phased";
    default: return "?";
  }
}

int32_t mg_persistent_mark_timeout(mg_ctx ctx) {
  g_last_error.clear();
  if (!ctx) return fail(MG_ERR_INVALID_ARG, "ctx is NULL");
  if (!ctx->ps.on || ctx->ps.phased)
    return fail(MG_ERR_UNSUPPORTED, "the context does not use the persistent schedule");
  MG_GUARD(MG_HIP(hipSetDevice(ctx->device));
           const unsigned one = 1u;
           MG_HIP(hipMemcpyAsync(&ctx->ps.d_bar->error, &one, sizeof one, hipMemcpyHostToDevice,
                                 ctx->stream));
           MG_HIP(hipStreamSynchronize(ctx->stream));
           return MG_OK;)
}

int32_t mg_num_levels(mg_ctx ctx, int32_t problem) {
  if (!ctx) return fail(MG_ERR_INVALID_ARG, "ctx is NULL");
  if (problem < 0 || problem >= (int)ctx->probs.size())
    return fail(MG_ERR_INVALID_ARG, "problem index out of range");
  return ctx->probs[problem].levels;
}

int32_t mg_solve_history(mg_ctx ctx, int32_t problem, int32_t cap, int32_t* prolong_out,
                         double* diff_out, int32_t* count_out) {
  if (!ctx || !count_out) return fail(MG_ERR_INVALID_ARG, "ctx or count_out is NULL");
  if (problem < 0 || problem >= (int)ctx->probs.size())
    return fail(MG_ERR_INVALID_ARG, "problem index out of range");
  if (cap < 0) return fail(MG_ERR_INVALID_ARG, "cap < 0");
  const mg::Problem& p = ctx->probs[problem];
  const int n = (int)p.hist_op.size();
  for (int k = 0; k < std::min(n, (int)cap); ++k) {
    if (prolong_out) prolong_out[k] = p.hist_op[k];
    if (diff_out) diff_out[k] = p.hist_diff[k];
  }
  *count_out = n;
  return MG_OK;
}

int32_t mg_destroy(mg_ctx ctx) {
  MG_GUARD(return destroy_ctx(ctx);)
}

const char* mg_status_string(int32_t status) {
  switch (status) {
    case MG_OK: return "ok";
    case MG_ERR_INVALID_ARG: return "invalid argument";
    case MG_ERR_UNSUPPORTED: return "unsupported";
    case MG_ERR_OOM: return "out of memory";
    case MG_ERR_HIP: return "HIP runtime error";
    case MG_ERR_INCOMPATIBLE_RHS: return "incompatible right-hand side";
    case MG_ERR_NOT_CONVERGED: return "not converged";
    case MG_ERR_STAGNATED: return "stagnated";
    case MG_ERR_NONFINITE: return "non-finite residual";
    default: return "unknown status";
  }
}

const char* mg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
