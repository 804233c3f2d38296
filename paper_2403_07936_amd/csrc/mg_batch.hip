// Batch schedules: the phase table of one step of every problem (built at
// set-up), the problem table that points at the caller's arrays, and the
// launches of the persistent kernel or of one kernel per phase.

#include <hip/hip_runtime.h>

#include "mg_host.h"
#include "mg_tail_dev.h"

namespace mg {

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
  // Level-0 down items of each problem (mixed path): global index range.
  std::vector<int> nfirst(B, 0), ncount(B, 0);
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
      if (l < 0) continue;
      const int at = (int)items.size();
      band_items(b, l, true);
      if (l == 0) {
        nfirst[b] = at;
        ncount[b] = (int)items.size() - at;
      }
    }
    close_phase(kItemDown, first);
  }
  P.head_end = (int)phases.size();  // the tail phase follows the down phases
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
  // Mixed path: the norm partials of the level-0 down items, 1 per item
  // (every such item writes one, whether or not the steps are split).
  // Split steps need every problem's level 0 above the tail.
  P.split = mixed;
  long nitems0 = 0;
  for (int b = 0; b < B; ++b) {
    if (ctx->probs[b].tail == 0) P.split = false;
    nitems0 += ncount[b];
  }
  for (int b = 0; b < B; ++b) P.h_probs[b].npart = nullptr, P.h_probs[b].ncount = 0;
  if (mixed && nitems0 > 0) {
    if (nitems0 > (1L << 28)) return fail(MG_ERR_UNSUPPORTED, "batch too large for its norm table");
    MG_TRY(alloc_level<double>(ctx, 1, (int)nitems0, &P.d_npart));
    MG_TRY(alloc_level<double>(ctx, 1, B, &P.d_nsums));
    long off = 0;
    for (int b = 0; b < B; ++b) {
      PProblem& q = P.h_probs[b];
      q.npart = P.d_npart + off;
      q.nfirst = nfirst[b];
      q.ncount = ncount[b];
      off += ncount[b];
    }
  }
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

void persistent_drop_graphs(Persist& P) {
  for (auto& g : P.graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

int32_t persistent_launch(mg_ctx_s* ctx, StepPart part) {
  Persist& P = ctx->ps;
  const bool mixed = ctx->opt.precision == MG_MIXED;
  if (part != kWhole && !P.split) return fail(MG_ERR_INVALID_ARG, "batch steps are not split");
  const int ph0 = part == kRest ? P.head_end : 0;
  const int ph1 = part == kHead ? P.head_end : P.nphases;
  auto launch = [&](hipStream_t s) {
    if (!P.phased)
      return mixed ? launch_persistent<float>(s, P.bc, P.d_probs, P.d_phases, ph0, ph1,
                                              P.d_items, P.d_bar, ctx->inv[P.bc], P.blocks, P.lds)
                   : launch_persistent<double>(s, P.bc, P.d_probs, P.d_phases, ph0, ph1,
                                               P.d_items, P.d_bar, ctx->inv[P.bc], P.blocks,
                                               P.lds);
    // One launch per phase: workgroup items one workgroup each, wavefront
    // items kPersistThreads / 64 per workgroup.
    for (int ph = ph0; ph < ph1; ++ph) {
      const PPhase& q = P.h_phases[ph];
      const bool wg = q.kind == kItemTail || q.kind == kItemPre;
      const int per = kPersistThreads / 64;
      const int blocks = wg ? q.count : (q.count + per - 1) / per;
      const size_t lds = q.kind == kItemTail ? P.lds_tail : (q.kind == kItemPre ? P.lds_pre : 0);
      const hipError_t e =
          mixed ? launch_phase<float>(s, P.bc, q, P.d_probs, P.d_items, ctx->inv[P.bc], blocks, lds)
                : launch_phase<double>(s, P.bc, q, P.d_probs, P.d_items, ctx->inv[P.bc], blocks,
                                       lds);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  if (!ctx->opt.use_graph || ctx->timing) {
    if (part != kWhole) {
      MG_HIP(launch(ctx->stream));
      return MG_OK;
    }
    MG_TRY(timed(ctx, ctx->stream, P.phased ? MG_K_PHASED : MG_K_PERSISTENT, 0, P.bytes,
                 [&] { return launch(ctx->stream); }));
    return MG_OK;
  }
  hipGraphExec_t& ge = P.graph[part];
  if (!ge) {
    hipGraph_t g = nullptr;
    MG_HIP(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeRelaxed));
    const hipError_t le = launch(ctx->capture);
    hipError_t e = hipStreamEndCapture(ctx->capture, &g);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(MG_ERR_HIP, std::string("persistent launch: ") + hipGetErrorString(le));
    }
    if (e != hipSuccess) return fail(MG_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      ge = nullptr;
      return fail(MG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
  }
  MG_HIP(hipGraphLaunch(ge, ctx->stream));
  return MG_OK;
}

int32_t persistent_head(mg_ctx_s* ctx, double* sums) {
  Persist& P = ctx->ps;
  const int B = (int)ctx->probs.size();
  MG_TRY(persistent_launch(ctx, kHead));
  MG_HIP(launch_reduce_norms(ctx->stream, P.d_probs, B, P.d_nsums));
  MG_HIP(hipMemcpyAsync(sums, P.d_nsums, sizeof(double) * B, hipMemcpyDeviceToHost,
                        ctx->stream));
  if (!P.phased) return persistent_check(ctx);  // synchronises
  MG_HIP(hipStreamSynchronize(ctx->stream));
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

template int32_t build_persistent<double>(mg_ctx_s* ctx);
template int32_t build_persistent<float>(mg_ctx_s* ctx);

}  // namespace mg
