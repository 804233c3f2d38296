// The autotuner: per-level kernel choices and the batch schedule, measured
// at set-up with HIP events and cached in process and in a text file.

#include <hip/hip_runtime.h>

#include "mg_host.h"
#include <cstdio>
#include <map>
#include <mutex>

namespace mg {

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
    // Short segments re-read more halo rows.  Timed alone, a pass finds those
    // rows in the 256 MB last-level cache; inside a cycle over a level larger
    // than that cache they come from HBM (4097^2 mixed down pass: 16-row
    // segments time faster here but run 9 % slower in the cycle), so such
    // levels do not try them, and there the resident heights are timed
    // first, so that a fixed height must beat them by the margin below
    // (periodic 4097^2 mixed up pass: 64 rows timed within it alone, but ran
    // 86.7 us in the cycle against 70.3 us at 38).
    const double level_bytes = (double)n * n * (add ? 24.0 : 3.0 * sizeof(T));
    const bool big = level_bytes > 256e6;
    std::vector<int> hs_cands = {0, 4, 8, 16, 32, 64, 96, 128};
    {
      const int fd = stream_fit_rows<T>(add ? kFitDownRes : (uin ? kFitDownIn : kFitDown), p.bc, n);
      const int fu = stream_fit_rows<T>(add ? kFitUpPre : kFitUp, p.bc, n);
      for (int hs : {fu, fd}) {
        if (hs <= 0) continue;
        auto at = std::find(hs_cands.begin(), hs_cands.end(), hs);
        if (big) {
          if (at != hs_cands.end()) hs_cands.erase(at);
          hs_cands.insert(hs_cands.begin(), hs);
        } else if (at == hs_cands.end()) {
          hs_cands.push_back(hs);
        }
      }
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
    persistent_drop_graphs(ctx->ps);
    ctx->ps.phased = true;
    st = time_launches(ctx, 2, persistent, &t_phased);
    persistent_drop_graphs(ctx->ps);
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
    persistent_drop_graphs(ctx->ps);
    ctx->ps.on = false;
  }
  std::lock_guard<std::mutex> lk(tune_mutex());
  schedule_table()[key] = choice;
  char line[256];
  std::snprintf(line, sizeof line, "S %s %s %d %s %d\n", arch.c_str(), prec, bc, sig, choice);
  append_tune_file(ctx->opt.tune_cache_path, line);
  return MG_OK;
}

}  // namespace mg
