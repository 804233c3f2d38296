// Host runtime and C ABI of the multigrid library (declared in include/mg.h).
//
// A context owns, per problem, the grid hierarchy down to 5 x 5, the
// per-level work arrays, the prefilter tables and, optionally, hipGraphs of
// one cycle.  The caller owns the finest-level u and f.
//
// The context's state and the helpers shared with mg_cycle.hip, mg_batch.hip
// and mg_tune.hip are in mg_host.h.

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
#include "mg_host.h"

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

namespace {
thread_local std::string g_last_error;
}  // namespace

int32_t fail(int32_t status, const std::string& why) {
  g_last_error = why;
  return status;
}

int32_t set_last_error(int32_t status, const char* why) {
  g_last_error = why ? why : "";
  return status;
}

bool valid_side(int n) {
  if (n < 5 || n > 16385) return false;
  const int m = (n - 1) / 4;
  return (n - 1) % 4 == 0 && (m & (m - 1)) == 0;
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

int32_t destroy_ctx(mg_ctx_s* ctx) {
  if (!ctx) return MG_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& p : ctx->probs)
    for (auto g : p.graph)
      if (g) (void)hipGraphExecDestroy(g);
  persistent_drop_graphs(ctx->ps);
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
    {
      // The level-0 down pass's norm partials: one per wavefront at the
      // shortest segments (2 rows).
      const int ext = p.bc == kPeriodic ? p.n - 1 : p.n;
      const int nb = (ext + stream_down_owned() - 1) / stream_down_owned();
      p.nblocks = std::max(p.nblocks, nb * ((ext + 1) / 2));
    }
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

namespace {

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
