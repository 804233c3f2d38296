// Cycles, solves and norm checks of the per-problem schedule (and the solve
// loop of every schedule): the enqueue functions queue one cycle or step of
// one problem on a stream, run_step replays it as a captured graph, and
// vcycle_impl / solve_impl implement mg_vcycle and mg_solve.

#include <hip/hip_runtime.h>

#include "mg_host.h"

namespace mg {


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


template int32_t enqueue_cnn<double>(mg_ctx_s*, hipStream_t, int, int, const double*, int,
                                     const double*, int, double*, int);
template int32_t enqueue_cnn<float>(mg_ctx_s*, hipStream_t, int, int, const float*, int,
                                    const float*, int, float*, int);

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

// StepPart (mg_host.h) for one problem's step: kHead is the level-0 down
// pass in the form that also sums r^2 of the iterate it starts from (the
// mixed pass that makes the FP64 residual; the FP64 pass that reads u), kRest
// all but that pass (its outputs are already in place).  The iterate
// changes only in the level-0 up pass, so the head alone leaves it as it
// was.

// The fused schedule: down passes to the first level of at most 65 x 65,
// the tail kernel, then prefilter + up passes back to level 0.  Level l's
// pre-smoothed u goes to h.r[l] (ping-pong against h.u[l] / u0).
// part (mixed level 0 with the residual made in the down pass and the
// iterate made again in the up pass, or an FP64 cycle from the caller's
// iterate with a streaming level-0 down pass): kHead queues that down pass
// with per-wavefront partials into norm_partials (mixed: ||r||^2 and ||f||^2;
// FP64: ||r||^2; count per sum to *norm_items); kRest the rest of the cycle.
template <typename T>
int32_t enqueue_cycle_fused(mg_ctx_s* ctx, const Problem& p, const Hierarchy<T>& h,
                            const PrefilterTaps* taps_dev, T* u0, int pu0, const T* f0, int pf0,
                            bool zero_guess, hipStream_t s, bool cnn, double* u64 = nullptr,
                            int p64 = 0, bool* added = nullptr, const double* res_u = nullptr,
                            const double* res_f = nullptr, int res_p = 0, T* r_out = nullptr,
                            const CallerArgs* ca = nullptr, StepPart part = kWhole,
                            double* norm_partials = nullptr, int* norm_items = nullptr) {
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
  // FP64 cycle from the caller's iterate whose level-0 down pass streams:
  // its head is that pass with the residual norm of the iterate it reads.
  const bool head64 = f64 && !zero_guess && t > 0 && ctx->opt.kernel_path != 2 &&
                      p.down_var[0] == 0 && !(cnn && ctx->cnn.levels > 0);
  if (part != kWhole && !remake0 && !head64)
    return fail(MG_ERR_INVALID_ARG, "split step without a streaming level-0 down pass");
  for (int l = 0; l < t; ++l) {
    const int n = p.side[l];
    const double m = unknowns_side(n, bc), mc = unknowns_side(p.side[l + 1], bc);
    const T* uin = (l == 0 && !zero_guess) ? u0 : nullptr;
    const double bytes = ((uin ? 3 : 2) * m * m + mc * mc) * sz;
    if constexpr (sizeof(T) == sizeof(float)) {
      if (l == 0 && res_u) {
        // Mixed level 0: the right-hand side is made from the FP64 iterate
        // inside the down pass (and stored for the up pass).
        if (part == kRest) continue;
        MG_TRY(timed(ctx, s, MG_K_DOWN, 0, (16 + 4 + (remake0 ? 0 : 4)) * m * m + 4 * mc * mc, [&] {
          return launch_down_res_stream(s, bc, n, res_u, res_p, res_f, res_p, r_out, pf0,
                                        remake0 ? nullptr : h.r[0], p.pitch[0], h.f[1],
                                        p.pitch[1], p.down_hs[0], ca,
                                        part == kHead ? norm_partials : nullptr,
                                        2 * p.nblocks, norm_items);
        }));
        if (part == kHead) return MG_OK;
        continue;
      }
    }
    if (l == 0 && head64 && part == kRest) continue;
    MG_TRY(timed(ctx, s, MG_K_DOWN, l, bytes, [&] {
      if (ctx->opt.kernel_path == 2 || p.down_var[l] == 1)
        return launch_down<T>(s, bc, n, uin, pu0, h.r[l], p.pitch[l], F(l), PF(l), h.f[l + 1],
                              p.pitch[l + 1], ca_at(l));
      const bool norm = l == 0 && head64 && part == kHead;
      return launch_down_stream<T>(s, bc, n, uin, pu0, h.r[l], p.pitch[l], F(l), PF(l),
                                   h.f[l + 1], p.pitch[l + 1], p.down_hs[l], ca_at(l),
                                   norm ? norm_partials : nullptr, 2 * p.nblocks,
                                   norm ? norm_items : nullptr);
    }));
    if (l == 0 && head64 && part == kHead) return MG_OK;
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

// A step of p whose convergence check is the step's own first pass (the
// level-0 down pass, which reads the iterate and leaves it unchanged, with
// the residual norm of that iterate), so that a step after a check queues
// only the rest: a mixed step whose level-0 passes make the residual and
// the iterate themselves (one inner cycle, both level-0 passes streaming),
// or an FP64 cycle whose level-0 down pass streams; no network.
bool split_step(const mg_ctx_s* ctx, const Problem& p) {
  if (!use_fused(ctx) || cnn_cycles(ctx) || p.tail == 0 || ctx->opt.kernel_path == 2 ||
      p.down_var[0] != 0)
    return false;
  if (ctx->opt.precision == MG_FP64) return true;
  return ctx->opt.inner_cycles == 1 && p.up_var[0] == 0;
}

// One step for problem p: an FP64 V-cycle, or one mixed refinement step
// (FP64 residual, FP32 inner cycles, FP64 update).  have_res: the mixed
// step's residual of this u is already in the level-0 right-hand side (left
// there by enqueue_check_mixed), so the step starts with the inner cycles;
// for a split step (mixed or FP64), the whole level-0 down pass has run as
// the check (enqueue_check_mixed, enqueue_check_head64).
int32_t enqueue_step(mg_ctx_s* ctx, const Problem& p, double* u, const double* f,
                     hipStream_t s, bool cnn, bool have_res = false,
                     const CallerArgs* ca = nullptr) {
  const double m = unknowns_side(p.n, p.bc), nn = (double)p.n * p.n;
  const bool fused = use_fused(ctx);
  if (ctx->opt.precision == MG_FP64) {
    if (fused)
      MG_TRY(enqueue_cycle_fused<double>(ctx, p, p.h64, p.taps64_dev, u, p.pitch0, f, p.pitch0,
                                         false, s, cnn, nullptr, 0, nullptr, nullptr, nullptr, 0,
                                         nullptr, ca,
                                         have_res && split_step(ctx, p) ? kRest : kWhole));
    else
      MG_TRY(enqueue_cycle<double>(ctx, p, p.h64, p.taps64, u, p.pitch0, f, p.pitch0, s, cnn));
  } else {
    int nb = 0;
    float* e0 = p.h32.u[0];
    float* r0 = p.h32.f[0];
    // The first inner cycle's streaming down pass can make the residual
    // itself when level 0 lies above the tail and both level-0 passes stream
    // (the up pass reads only rows and columns that down pass stores).
    const bool split = split_step(ctx, p);
    const bool res_in_down = fused && (!have_res || split) && p.tail > 0 &&
                             ctx->opt.kernel_path != 2 && p.down_var[0] == 0 && p.up_var[0] == 0;
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
                                          p.pitch0, r0, ca, split && have_res ? kRest : kWhole));
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

int32_t run_step(mg_ctx_s* ctx, Problem& p, double* u, const double* f, bool cnn,
                 bool have_res) {
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
// right-hand side, so that step skips it (run_step with have_res).  A split
// step's check is that step's level-0 down pass itself, with its norms
// (||f||^2 into p.sums[1] as well).
int32_t enqueue_check_mixed(mg_ctx_s* ctx, Problem& p, const double* u, const double* f) {
  int nb = 0;
  if (split_step(ctx, p)) {
    MG_TRY(enqueue_cycle_fused<float>(ctx, p, p.h32, p.taps32_dev, p.h32.u[0], p.pitch[0],
                                      p.h32.f[0], p.pitch[0], true, ctx->stream, false,
                                      const_cast<double*>(u),  // not written by the head
                                      p.pitch0, nullptr, u, f, p.pitch0, p.h32.f[0], nullptr,
                                      kHead, p.partials, &nb));
    MG_HIP(launch_reduce(ctx->stream, p.partials, nb, nb, 2, p.sums));
    return MG_OK;
  }
  const double nn = (double)p.n * p.n;
  MG_TRY(timed(ctx, ctx->stream, MG_K_RESIDUAL_MIXED, 0, 20 * nn, [&] {
    return launch_residual_mixed(ctx->stream, p.bc, p.n, u, p.pitch0, f, p.pitch0, p.h32.f[0],
                                 p.pitch[0], p.partials, &nb);
  }));
  MG_HIP(launch_reduce(ctx->stream, p.partials, nb, nb, 1, p.sums));
  return MG_OK;
}

// FP64 path, split steps: ||f - A u||^2 into p.sums[0] from the next
// cycle's level-0 down pass (the head of that cycle, which leaves u as it
// was); ||f||^2 is in p.sums[1] already.
int32_t enqueue_check_head64(mg_ctx_s* ctx, Problem& p, double* u, const double* f) {
  int nb = 0;
  MG_TRY(enqueue_cycle_fused<double>(ctx, p, p.h64, p.taps64_dev, u, p.pitch0, f, p.pitch0, false,
                                     ctx->stream, false, nullptr, 0, nullptr, nullptr, nullptr, 0,
                                     nullptr, nullptr, kHead, p.partials, &nb));
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

  // Split batches: every check is the head of the next step (hsums: each
  // problem's sum of r^2; fsq: its sum of f^2, from the moments below).
  const bool split = ctx->ps.on && ctx->ps.split;
  std::vector<double> hsums(split ? B : 0), fsq(split ? B : 0);
  bool have_head = false;
  // Periodic right-hand sides must have zero mean (the constants are the
  // null space of A).
  {
    std::vector<int> per;
    std::vector<double> mom;
    if (ctx->ps.on) {
      // The batch schedules: one launch for every problem's sums.
      MG_TRY(persistent_bind(ctx, u, f, {}));
      if (ctx->ps.bc == kPeriodic || split) {
        if (ctx->ps.bc == kPeriodic)
          for (int b = 0; b < B; ++b) per.push_back(b);
        mom.resize(2 * B);
        MG_HIP(launch_moments_batched(ctx->stream, ctx->ps.d_probs, B, ctx->ps.d_partials,
                                      ctx->ps.slots, ctx->ps.d_sums, false));
        MG_HIP(hipMemcpyAsync(mom.data(), ctx->ps.d_sums, sizeof(double) * 2 * B,
                              hipMemcpyDeviceToHost, ctx->stream));
      }
    } else {
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
    }
    MG_HIP(hipStreamSynchronize(ctx->stream));
    for (int b = 0; b < (split ? B : 0); ++b) fsq[b] = mom[2 * b + 1];
    for (size_t k = 0; k < per.size(); ++k) {
      const Problem& p = ctx->probs[per[k]];
      const double M = (double)(p.n - 1) * (double)(p.n - 1);
      const double* m2 = mom.empty() ? ctx->host + 2 * k : mom.data() + 2 * k;
      const double sum = m2[0], sq = m2[1];
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
  if (split) {
    MG_TRY(persistent_bind(ctx, u, f, {}));
    MG_TRY(persistent_head(ctx, hsums.data()));
    have_head = true;
    for (int b = 0; b < B; ++b) {
      const double rr = hsums[b], ff = fsq[b];
      rel[b] = ff > 0.0 ? std::sqrt(rr) / std::sqrt(ff) : std::sqrt(rr);
    }
  } else if (pers) {
    MG_TRY(persistent_bind(ctx, u, f, {}));
    MG_TRY(persistent_relres(ctx, rel.data()));
  } else if (mixed_chk) {
    for (int b = 0; b < B; ++b) {
      // Periodic problems: the right-hand-side check above left ||f||^2 in
      // p.sums[1] already (the same kernel and reduction); a split step's
      // check makes it in its own pass.
      if (ctx->probs[b].bc != kPeriodic && !split_step(ctx, ctx->probs[b]))
        MG_TRY(enqueue_fnorm(ctx, ctx->probs[b], f[b]));
      MG_TRY(enqueue_check_mixed(ctx, ctx->probs[b], u[b], f[b]));
      have_res[b] = 1;
    }
    MG_TRY(read_relres(ctx, all, rel.data()));
  } else {
    for (int b = 0; b < B; ++b) {
      Problem& p = ctx->probs[b];
      if (split_step(ctx, p)) {
        // ||f||^2 once (periodic: the mean check above left it), then the
        // head of the first cycle.
        if (p.bc != kPeriodic) MG_TRY(enqueue_fnorm(ctx, p, f[b]));
        MG_TRY(enqueue_check_head64(ctx, p, u[b], f[b]));
        have_res[b] = 1;
      } else {
        MG_TRY(enqueue_resnorm(ctx, p, u[b], f[b]));
      }
    }
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
          MG_TRY(persistent_launch(ctx, have_head ? kRest : kWhole));
        }
        have_head = false;
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
    if (split) {
      // The head of the next step for every problem still running.
      std::vector<int> run(B, 0);
      for (int b = 0; b < B; ++b) run[b] = state[b] == 1 ? 1 : 0;
      MG_TRY(persistent_bind(ctx, u, f, run));
      MG_TRY(persistent_head(ctx, hsums.data()));
      have_head = true;
      for (size_t k = 0; k < chk.size(); ++k) {
        const int b = chk[k];
        const double rr = hsums[b], ff = fsq[b];
        r[k] = ff > 0.0 ? std::sqrt(rr) / std::sqrt(ff) : std::sqrt(rr);
      }
    } else if (pers) {
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
      for (int b : chk) {
        Problem& p = ctx->probs[b];
        if (split_step(ctx, p)) {
          MG_TRY(enqueue_check_head64(ctx, p, u[b], f[b]));
          have_res[b] = 1;
        } else {
          MG_TRY(enqueue_resnorm(ctx, p, u[b], f[b]));
        }
      }
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
  // Periodic results: zero mean and rewritten seam (the batch schedules: in
  // three launches for every problem that stepped).
  if (pers && ctx->ps.bc == kPeriodic) {
    std::vector<int> stepped(B);
    for (int b = 0; b < B; ++b) stepped[b] = cycles[b] > 0 ? 1 : 0;
    MG_TRY(persistent_bind(ctx, u, f, stepped));
    MG_HIP(launch_moments_batched(ctx->stream, ctx->ps.d_probs, B, ctx->ps.d_partials,
                                  ctx->ps.slots, ctx->ps.d_sums, true));
    MG_HIP(launch_remove_mean_batched(ctx->stream, ctx->ps.d_probs, B, ctx->ps.d_sums));
  }
  for (int b = 0; b < B && !(pers && ctx->ps.bc == kPeriodic); ++b) {
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

}  // namespace mg
