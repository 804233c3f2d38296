// Fused, LDS-tiled kernels of the V(2,2) cycle for gfx950.
//
//   k_down  : 2 red-black sweeps + residual + full-weighting restriction of
//             one level in one pass (temporal blocking: the tile is loaded
//             with a 6-node halo, each half-sweep invalidates one more ring).
//   k_up    : cubic-spline evaluation of the coarse correction, u += P e_c,
//             then 2 red-black sweeps, in one pass (4-node halo).
//   k_pre_x / k_pre_y : B-spline prefilter of a coarse level (the non-local
//             part of the spline), as causal + anti-causal first-order
//             recursions over 64-node segments with a warm-up run long enough
//             that the truncated state is below the working precision.
//   k_tail  : the whole V-cycle below a 65 x 65 level in one workgroup, with
//             every level resident in LDS, including the 5 x 5 direct solve
//             (FP64) and the prefilter of the top tail level.
//
// The arithmetic of every step is the same as in mg_kernels.hip (Section 2.2
// and the appendix's V-cycle); only the schedule differs.  In-place updates
// across workgroups would race on halos, so a pass reads one buffer and
// writes another.

#include <algorithm>

#include "mg_device.h"

namespace mg {
namespace {

constexpr int kThreads = 256;
constexpr int kTailThreads = 1024;

template <typename T, int BC, int W, int HH>
__device__ __forceinline__ void load_tile(T* s, const T* __restrict__ g, int pg, int n, int gy0,
                                          int gx0, bool zero) {
  const int N = n - 1;
#pragma unroll
  for (int k = threadIdx.x; k < W * HH; k += kThreads) {
    const int ly = k / W, lx = k - ly * W;
    int gy = gy0 + ly, gx = gx0 + lx;
    T v = T(0);
    if (!zero) {
      if constexpr (BC == kPeriodic) {
        gy = gy < 0 ? gy + N : (gy >= N ? gy - N : gy);
        gx = gx < 0 ? gx + N : (gx >= N ? gx - N : gx);
        v = g[(size_t)gy * pg + gx];
      } else {
        if (gy >= 0 && gy < n && gx >= 0 && gx < n) v = g[(size_t)gy * pg + gx];
      }
    }
    s[k] = v;
  }
}

// One red-black half-sweep over the inner nodes of an LDS tile whose node
// (0, 0) is global node (gy0, gx0), gx0 even.
template <typename T, int BC, int W, int HH>
__device__ __forceinline__ void tile_half_sweep(T* su, const T* sf, int n, int gy0, int gx0,
                                                int colour, T h2) {
  constexpr int NL = (W - 2) / 2;
  for (int k = threadIdx.x; k < (HH - 2) * NL; k += blockDim.x) {
    const int ly = 1 + k / NL;
    const int q = k - (ly - 1) * NL;
    const int gy = gy0 + ly;
    const int lx = 1 + ((colour + gy + 1) & 1) + 2 * q;
    if constexpr (BC == kDirichlet) {
      const int gx = gx0 + lx;
      if (gy < 1 || gy > n - 2 || gx < 1 || gx > n - 2) continue;
    }
    const int c = ly * W + lx;
    const T s = ((su[c - W] + su[c + W]) + su[c - 1]) + su[c + 1];
    su[c] = (h2 * sf[c] + s) * T(0.25);
  }
}

template <int BC>
__device__ __forceinline__ bool is_unknown(int gy, int gx, int n) {
  if constexpr (BC == kPeriodic) return true;
  return gy >= 1 && gy <= n - 2 && gx >= 1 && gx <= n - 2;
}

template <typename T, int BC, int TX, int TY>
__global__ void __launch_bounds__(kThreads)
    k_down(int n, const T* __restrict__ uin, T* __restrict__ uout, int pui, int puo,
           const T* __restrict__ f, int pf, T* __restrict__ fc, int pfc, int tiles_x, int ntiles,
           T h2, T inv_h2) {
  constexpr int H = 6, W = TX + 2 * H, HH = TY + 2 * H;
  __shared__ T su[W * HH];
  __shared__ T sf[W * HH];
  const int t = xcd_tile(blockIdx.x, ntiles);
  const int x0 = (t % tiles_x) * TX, y0 = (t / tiles_x) * TY;
  const int gx0 = x0 - H, gy0 = y0 - H;
  load_tile<T, BC, W, HH>(su, uin, pui, n, gy0, gx0, uin == nullptr);
  load_tile<T, BC, W, HH>(sf, f, pf, n, gy0, gx0, false);
  __syncthreads();
  for (int s = 0; s < 4; ++s) {
    tile_half_sweep<T, BC, W, HH>(su, sf, n, gy0, gx0, s & 1, h2);
    __syncthreads();
  }
  // Residual, in place of f, on the nodes the restriction reads.
  constexpr int RW = TX + 1;
  for (int k = threadIdx.x; k < (TY + 1) * RW; k += blockDim.x) {
    const int ly = H - 1 + k / RW, lx = H - 1 + k % RW;
    const int c = ly * W + lx;
    T r = T(0);
    if (is_unknown<BC>(gy0 + ly, gx0 + lx, n)) {
      const T s = ((su[c - W] + su[c + W]) + su[c - 1]) + su[c + 1];
      r = sf[c] - (T(4) * su[c] - s) * inv_h2;
    }
    sf[c] = r;
  }
  __syncthreads();
  const int nc = (n - 1) / 2 + 1;
  constexpr int CX = TX / 2;
  for (int k = threadIdx.x; k < (TY / 2) * CX; k += blockDim.x) {
    const int a = k / CX, b = k - a * CX;
    const int I = y0 / 2 + a, J = x0 / 2 + b;
    const bool ok = BC == kPeriodic ? (I < nc - 1 && J < nc - 1)
                                    : (I >= 1 && I <= nc - 2 && J >= 1 && J <= nc - 2);
    if (!ok) continue;
    const int c = (H + 2 * a) * W + H + 2 * b;
    const T edges = ((sf[c - W] + sf[c + W]) + sf[c - 1]) + sf[c + 1];
    const T corners = ((sf[c - W - 1] + sf[c - W + 1]) + sf[c + W - 1]) + sf[c + W + 1];
    fc[(size_t)I * pfc + J] = ((T(4) * sf[c] + T(2) * edges) + corners) * T(0.0625);
  }
  for (int k = threadIdx.x; k < TY * TX; k += blockDim.x) {
    const int a = k / TX, b = k - a * TX;
    const int gy = y0 + a, gx = x0 + b;
    const bool ok = BC == kPeriodic ? (gy < n - 1 && gx < n - 1)
                                    : (gy >= 1 && gy <= n - 2 && gx >= 1 && gx <= n - 2);
    if (ok) uout[(size_t)gy * puo + gx] = su[(H + a) * W + H + b];
  }
}

template <typename T, int BC, int TX, int TY>
__global__ void __launch_bounds__(kThreads)
    k_up(int n, const T* __restrict__ uin, T* __restrict__ uout, int pui, int puo,
         const T* __restrict__ f, int pf, const T* __restrict__ c, int pc, int tiles_x, int ntiles,
         T h2) {
  constexpr int H = 4, W = TX + 2 * H, HH = TY + 2 * H;
  constexpr int CW = TX / 2 + H + 3, CH = TY / 2 + H + 3;
  __shared__ T su[W * HH];
  __shared__ T sf[W * HH];
  __shared__ T sc[CW * CH];
  __shared__ T sx[CH * W];
  const int t = xcd_tile(blockIdx.x, ntiles);
  const int x0 = (t % tiles_x) * TX, y0 = (t / tiles_x) * TY;
  const int gx0 = x0 - H, gy0 = y0 - H;
  const int nc = (n - 1) / 2 + 1;
  const int cx0 = (gx0 >> 1) - 1, cy0 = (gy0 >> 1) - 1;
  load_tile<T, BC, W, HH>(su, uin, pui, n, gy0, gx0, false);
  load_tile<T, BC, W, HH>(sf, f, pf, n, gy0, gx0, false);
#pragma unroll
  for (int k = threadIdx.x; k < CW * CH; k += kThreads) {
    const int cy = k / CW, cx = k - cy * CW;
    bool ny, nx;
    const int I = ext_node<BC>(cy0 + cy, nc, &ny);
    const int J = ext_node<BC>(cx0 + cx, nc, &nx);
    const T v = c[(size_t)I * pc + J];
    sc[k] = (ny != nx) ? -v : v;
  }
  __syncthreads();
  // Spline along x for every coarse row of the tile.
  for (int k = threadIdx.x; k < CH * W; k += blockDim.x) {
    const int cy = k / W, lx = k - cy * W;
    int base;
    T w[4];
    const int nt = bspline_taps<T>(gx0 + lx, &base, w);
    const T* row = sc + cy * CW + (base - cx0);
    T v = (w[0] * row[0] + w[1] * row[1]) + w[2] * row[2];
    if (nt == 4) v += w[3] * row[3];
    sx[k] = v;
  }
  __syncthreads();
  // Then along y, and add the correction to u.
  for (int k = threadIdx.x; k < HH * W; k += blockDim.x) {
    const int ly = k / W, lx = k - ly * W;
    if (!is_unknown<BC>(gy0 + ly, gx0 + lx, n)) continue;
    int base;
    T w[4];
    const int nt = bspline_taps<T>(gy0 + ly, &base, w);
    const T* col = sx + (base - cy0) * W + lx;
    T v = (w[0] * col[0] + w[1] * col[W]) + w[2] * col[2 * W];
    if (nt == 4) v += w[3] * col[3 * W];
    su[k] += v;
  }
  __syncthreads();
  for (int s = 0; s < 4; ++s) {
    tile_half_sweep<T, BC, W, HH>(su, sf, n, gy0, gx0, s & 1, h2);
    __syncthreads();
  }
  for (int k = threadIdx.x; k < TY * TX; k += blockDim.x) {
    const int a = k / TX, b = k - a * TX;
    const int gy = y0 + a, gx = x0 + b;
    const bool ok = BC == kPeriodic ? (gy < n - 1 && gx < n - 1)
                                    : (gy >= 1 && gy <= n - 2 && gx >= 1 && gx <= n - 2);
    if (ok) uout[(size_t)gy * puo + gx] = su[(H + a) * W + H + b];
  }
}

// B-spline prefilter along one axis: c = S^-1 e with S = (1, 4, 1)/6 on the
// extended sequence.  S^-1 = g / ((1 - z q^-1)(1 - z q)), z = sqrt(3) - 2,
// g = 12 - 6 sqrt(3): a causal recursion p_k = e_k + z p_{k-1} followed by an
// anti-causal one m_k = p_k + z m_{k+1}, c_k = g m_k.  A thread filters one
// segment of S nodes of one line held in registers; both recursions start K
// nodes outside the segment from a zero state, and the neglected state is
// below |z|^K of the data.
constexpr double kZ = kPrefZ;
constexpr double kG = kPrefG;

template <typename T, int L, int K>
__device__ __forceinline__ void iir_regs(T (&v)[L]) {
  const T z = T(kZ), g = T(kG);
  T p = T(0);
#pragma unroll
  for (int k = 0; k < L; ++k) {
    p = v[k] + z * p;
    v[k] = p;
  }
  T m = T(0);
#pragma unroll
  for (int k = L - 1; k >= K; --k) {
    m = v[k] + z * m;
    v[k] = g * m;
  }
}

template <typename T>
struct PreCfg {
  static constexpr int K = sizeof(T) == 8 ? kPrefilterHalfTapsF64 : kPrefilterHalfTapsF32;
  static constexpr int S = sizeof(T) == 8 ? 16 : 32;  // segment length
  static constexpr int L = S + 2 * K;
  // LDS row pitch for the x pass: lanes read rows with this stride, chosen
  // so that 32 consecutive rows fall on distinct banks.
  static constexpr int P = sizeof(T) == 8 ? (L + 15) / 16 * 16 + 1 : L + 1 - (L % 2);
};

// Along y: one thread per (column, segment); lanes are consecutive columns,
// so every load and store is coalesced.
template <typename T, int BC>
__global__ void __launch_bounds__(256)
    k_pre_y(int nc, const T* __restrict__ in, int pi, T* __restrict__ out, int po, int nseg) {
  using C = PreCfg<T>;
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int seg = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (seg >= nseg) return;
  const int r0 = seg * C::S;
  const bool cok = col < nc;
  const int cc = cok ? col : 0;
  T v[C::L];
#pragma unroll
  for (int k = 0; k < C::L; ++k) {
    bool neg;
    const int r = ext_node_any<BC>(r0 - C::K + k, nc, &neg);
    const T x = cok ? in[(size_t)r * pi + cc] : T(0);
    v[k] = neg ? -x : x;
  }
  iir_regs<T, C::L, C::K>(v);
  if (!cok) return;
#pragma unroll
  for (int j = 0; j < C::S; ++j) {
    const int r = r0 + j;
    if (r >= nc) break;
    T y = v[C::K + j];
    if (BC == kDirichlet && (r == 0 || r == nc - 1)) y = T(0);
    out[(size_t)r * po + col] = y;
  }
}

// Along x: one wavefront per row, the recursion carried across the row in
// chunks of 64 columns (wave_line_prefilter); each element is read and
// written once, coalesced.  The causal values wait in LDS.
template <typename T, int BC>
__global__ void __launch_bounds__(256)
    k_pre_x(int nc, const T* __restrict__ in, int pi, T* __restrict__ out, int po) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int M = BC == kPeriodic ? nc - 1 : nc;
  T* buf = reinterpret_cast<T*>(smem_raw) + wave * (M + 128);
  const int r = blockIdx.x * (blockDim.x >> 6) + wave;
  if (r >= nc) return;
  const ScanWeights<T> w(lane);
  wave_line_prefilter<T, BC>(in + (size_t)r * pi, 1, buf, out + (size_t)r * po, 1, nc, w, lane);
}

// ------------------------------------------------------------------ tail --
// All levels from side nt down to 5 in one workgroup.  LDS holds u and f of
// every level (pitch = side) and one scratch grid of the top side.

template <int BC>
__device__ __forceinline__ int wrap_prev(int i, int n) {
  return BC == kPeriodic ? (i == 0 ? n - 2 : i - 1) : i - 1;
}
template <int BC>
__device__ __forceinline__ int wrap_next(int i, int n) {
  return BC == kPeriodic ? (i == n - 2 ? 0 : i + 1) : i + 1;
}

// The tail's 1024 threads form a 32 x 32 layout; a grid of side n <= 65 is
// covered by visiting nodes (ty + 32a, tx + 32b), a, b < 3.
#define MG_TAIL_FOR(n, i, j, ...)                         \
  do {                                                    \
    _Pragma("unroll") for (int a_ = 0; a_ < 3; ++a_) {    \
      const int i = (int)threadIdx.y + 32 * a_;           \
      if (i < (n)) {                                      \
        _Pragma("unroll") for (int b_ = 0; b_ < 3; ++b_) { \
          const int j = (int)threadIdx.x + 32 * b_;       \
          if (j < (n)) {                                  \
            __VA_ARGS__                                   \
          }                                               \
        }                                                 \
      }                                                   \
    }                                                     \
  } while (0)

template <int BC>
__device__ __forceinline__ bool tail_unknown(int i, int j, int n) {
  return BC == kPeriodic ? (i < n - 1 && j < n - 1) : (i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2);
}

template <typename T, int BC>
__device__ __forceinline__ void tail_sweeps(T* u, const T* f, int n, int count) {
  const double hd = 1.0 / (double)(n - 1);
  const T h2 = T(hd * hd);
  for (int s = 0; s < count; ++s) {
    const int colour = s & 1;
    MG_TAIL_FOR(n, i, j, {
      if (tail_unknown<BC>(i, j, n) && ((i + j) & 1) == colour) {
        const T sum = ((u[wrap_prev<BC>(i, n) * n + j] + u[wrap_next<BC>(i, n) * n + j]) +
                       u[i * n + wrap_prev<BC>(j, n)]) +
                      u[i * n + wrap_next<BC>(j, n)];
        u[i * n + j] = (h2 * f[i * n + j] + sum) * T(0.25);
      }
    });
    __syncthreads();
  }
}

// r = f - A u into r (pitch n, unknown nodes only), then f_c = FW(r).
template <typename T, int BC>
__device__ __forceinline__ void tail_restrict(const T* u, const T* f, T* r, T* fc, int n) {
  const T inv_h2 = T((double)(n - 1) * (double)(n - 1));
  MG_TAIL_FOR(n, i, j, {
    T v = T(0);
    if (tail_unknown<BC>(i, j, n)) {
      const T s = ((u[wrap_prev<BC>(i, n) * n + j] + u[wrap_next<BC>(i, n) * n + j]) +
                   u[i * n + wrap_prev<BC>(j, n)]) +
                  u[i * n + wrap_next<BC>(j, n)];
      v = f[i * n + j] - (T(4) * u[i * n + j] - s) * inv_h2;
    }
    r[i * n + j] = v;
  });
  __syncthreads();
  const int nc = (n - 1) / 2 + 1;
  MG_TAIL_FOR(nc, I, J, {
    T v = T(0);
    if (tail_unknown<BC>(I, J, nc)) {
      const int i = 2 * I, j = 2 * J;
      const int im = wrap_prev<BC>(i, n), ip = wrap_next<BC>(i, n);
      const int jm = wrap_prev<BC>(j, n), jp = wrap_next<BC>(j, n);
      const T edges = ((r[im * n + j] + r[ip * n + j]) + r[i * n + jm]) + r[i * n + jp];
      const T corners = ((r[im * n + jm] + r[im * n + jp]) + r[ip * n + jm]) + r[ip * n + jp];
      v = ((T(4) * r[i * n + j] + T(2) * edges) + corners) * T(0.0625);
    }
    fc[I * nc + J] = v;
  });
  __syncthreads();
}

// Prefilter a tail grid: rows of src (in place), then columns into dst
// (pitch pd); each wavefront takes every 16th line, with its own slice of
// the scratch grid for the causal values.
template <typename T, int BC>
__device__ __forceinline__ void tail_prefilter(T* src, T* tmp, T* dst, int pd, int nc) {
  const int t = threadIdx.y * 32 + threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const ScanWeights<T> w(lane);
  T* buf = tmp + wave * (nc + 128);
  for (int line = wave; line < nc; line += 16)
    wave_line_prefilter<T, BC>(src + line * nc, 1, buf, src + line * nc, 1, nc, w, lane);
  __syncthreads();
  for (int line = wave; line < nc; line += 16)
    wave_line_prefilter<T, BC>(src + line, nc, buf, dst + line, pd, nc, w, lane);
  __syncthreads();
}

// u += P c on a tail grid of side n from coefficients c of side nc.
template <typename T, int BC>
__device__ __forceinline__ void tail_prolong_add(T* u, const T* c, int n) {
  const int nc = (n - 1) / 2 + 1;
  MG_TAIL_FOR(n, i, j, {
    if (tail_unknown<BC>(i, j, n)) {
      int bi, bj;
      T wi[4], wj[4];
      const int ni = bspline_taps<T>(i, &bi, wi);
      const int nj = bspline_taps<T>(j, &bj, wj);
      T v = T(0);
      for (int a = 0; a < ni; ++a) {
        bool na;
        const int I = ext_node<BC>(bi + a, nc, &na);
        T row = T(0);
        for (int b = 0; b < nj; ++b) {
          bool nb;
          const int J = ext_node<BC>(bj + b, nc, &nb);
          const T x = c[I * nc + J];
          row += wj[b] * (nb ? -x : x);
        }
        v += wi[a] * (na ? -row : row);
      }
      u[i * n + j] += v;
    }
  });
  __syncthreads();
}

// Level l of the tail has side ((nt - 1) >> l) + 1; its u and f follow the
// arrays of the levels above it, and the scratch grid follows the last level.
__device__ __forceinline__ int tail_side(int nt, int l) { return ((nt - 1) >> l) + 1; }
__device__ __forceinline__ int tail_levels(int nt) {
  int l = 0;
  while (tail_side(nt, l) > 5) ++l;
  return l + 1;
}
__device__ __forceinline__ int tail_offu(int nt, int l) {
  int off = 0;
  for (int k = 0; k < l; ++k) {
    const int n = tail_side(nt, k);
    off += 2 * n * n;
  }
  return off;
}
__device__ __forceinline__ int tail_offf(int nt, int l) {
  const int n = tail_side(nt, l);
  return tail_offu(nt, l) + n * n;
}

template <typename T, int BC>
__global__ void __launch_bounds__(kTailThreads)
    k_tail(int nt, const T* __restrict__ uin, int pui, T* __restrict__ uout, int puo,
           const T* __restrict__ f, int pf, T* __restrict__ cout, int pco,
           const double* __restrict__ inv) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int L = tail_levels(nt);
  T* tmp = sm + tail_offu(nt, L);
  MG_TAIL_FOR(nt, i, j, {
    sm[i * nt + j] = uin ? uin[(size_t)i * pui + j] : T(0);
    sm[nt * nt + i * nt + j] = f[(size_t)i * pf + j];
  });
  __syncthreads();
  for (int l = 0; l + 1 < L; ++l) {
    const int n = tail_side(nt, l);
    T* u = sm + tail_offu(nt, l);
    T* ff = sm + tail_offf(nt, l);
    if (l > 0) {
      MG_TAIL_FOR(n, i, j, { u[i * n + j] = T(0); });
      __syncthreads();
    }
    tail_sweeps<T, BC>(u, ff, n, 4);
    tail_restrict<T, BC>(u, ff, tmp, sm + tail_offf(nt, l + 1), n);
  }
  {
    // 5 x 5 direct solve in FP64.
    T* u = sm + tail_offu(nt, L - 1);
    const T* ff = sm + tail_offf(nt, L - 1);
    constexpr int m = BC == kDirichlet ? 9 : 16;
    const int t = threadIdx.y * 32 + threadIdx.x;
    if (t < 25) {
      const int i = t / 5, j = t % 5;
      int k = -1;
      if (BC == kDirichlet) {
        if (i >= 1 && i <= 3 && j >= 1 && j <= 3) k = (i - 1) * 3 + (j - 1);
      } else {
        k = (i % 4) * 4 + (j % 4);
      }
      double v = 0.0;
      if (k >= 0)
        for (int q = 0; q < m; ++q) {
          const int qi = BC == kDirichlet ? q / 3 + 1 : q / 4;
          const int qj = BC == kDirichlet ? q % 3 + 1 : q % 4;
          v += inv[k * m + q] * (double)ff[qi * 5 + qj];
        }
      u[t] = T(v);
    }
    __syncthreads();
  }
  for (int l = L - 2; l >= 0; --l) {
    const int n = tail_side(nt, l), nc = tail_side(nt, l + 1);
    T* uc = sm + tail_offu(nt, l + 1);
    tail_prefilter<T, BC>(uc, tmp, uc, nc, nc);
    tail_prolong_add<T, BC>(sm + tail_offu(nt, l), uc, n);
    tail_sweeps<T, BC>(sm + tail_offu(nt, l), sm + tail_offf(nt, l), n, 4);
  }
  if (uout)
    MG_TAIL_FOR(nt, i, j, {
      if (tail_unknown<BC>(i, j, nt)) uout[(size_t)i * puo + j] = sm[i * nt + j];
    });
  if (cout) {
    __syncthreads();
    tail_prefilter<T, BC>(sm, tmp, cout, pco, nt);
  }
}

// u and f of every tail level, then the scratch grid: the residual of the
// top level, or 16 per-wavefront line buffers of the prefilter.
size_t tail_bytes(int nt, size_t elem) {
  size_t tot = 0;
  for (int n = nt;; n = (n - 1) / 2 + 1) {
    tot += 2 * (size_t)n * n;
    if (n == 5) break;
  }
  const size_t scratch = std::max((size_t)nt * nt, (size_t)16 * (nt + 128));
  return (tot + scratch) * elem;
}

template <typename T, int BC>
struct Fused {
  static constexpr int TX = 64, TY = 32;
};

}  // namespace

int fused_tile_x() { return 64; }
int fused_tile_y() { return 32; }

hipError_t fused_init() {
  // x-pass line buffers: one wavefront per workgroup suffices up to the
  // largest coarse level (nc = 8193 for n = 16385): (8193 + 128) doubles.
  const int xmax = (8193 + 128) * 8;
  hipError_t e0;
  e0 = hipFuncSetAttribute((const void*)k_pre_x<double, kDirichlet>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, xmax);
  if (e0 != hipSuccess) return e0;
  e0 = hipFuncSetAttribute((const void*)k_pre_x<double, kPeriodic>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, xmax);
  if (e0 != hipSuccess) return e0;
  const size_t max64 = tail_bytes(kTailMaxSide, sizeof(double));
  const size_t max32 = tail_bytes(kTailMaxSide, sizeof(float));
  hipError_t e;
  e = hipFuncSetAttribute((const void*)k_tail<double, kDirichlet>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)max64);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_tail<double, kPeriodic>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)max64);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_tail<float, kDirichlet>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)max32);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_tail<float, kPeriodic>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)max32);
}

static inline int tiles_along(int n, int bc, int T) {
  const int extent = bc == kPeriodic ? n - 1 : n;
  return (extent + T - 1) / T;
}

template <typename T>
hipError_t launch_down(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout, int puo,
                       const T* f, int pf, T* fc, int pfc) {
  constexpr int TX = 64, TY = 32;
  const int tx = tiles_along(n, bc, TX), ty = tiles_along(n, bc, TY);
  const int nt = tx * ty;
  const double hd = 1.0 / (double)(n - 1);
  const T h2 = T(hd * hd), inv_h2 = T((double)(n - 1) * (double)(n - 1));
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_down<T, kDirichlet, TX, TY>), dim3(nt), dim3(kThreads), 0, s, n, uin,
                       uout, pui, puo, f, pf, fc, pfc, tx, nt, h2, inv_h2);
  else
    hipLaunchKernelGGL((k_down<T, kPeriodic, TX, TY>), dim3(nt), dim3(kThreads), 0, s, n, uin, uout,
                       pui, puo, f, pf, fc, pfc, tx, nt, h2, inv_h2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_up(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout, int puo,
                     const T* f, int pf, const T* c, int pc) {
  constexpr int TX = 64, TY = 32;
  const int tx = tiles_along(n, bc, TX), ty = tiles_along(n, bc, TY);
  const int nt = tx * ty;
  const double hd = 1.0 / (double)(n - 1);
  const T h2 = T(hd * hd);
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_up<T, kDirichlet, TX, TY>), dim3(nt), dim3(kThreads), 0, s, n, uin, uout,
                       pui, puo, f, pf, c, pc, tx, nt, h2);
  else
    hipLaunchKernelGGL((k_up<T, kPeriodic, TX, TY>), dim3(nt), dim3(kThreads), 0, s, n, uin, uout,
                       pui, puo, f, pf, c, pc, tx, nt, h2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prefilter_iir(hipStream_t s, int bc, int nc, const T* e, int pe, T* tmp, int pt,
                                T* c, int pc) {
  using C = PreCfg<T>;
  const int nseg = (nc + C::S - 1) / C::S;
  int waves = 4;
  while (waves > 1 && (size_t)waves * (nc + 128) * sizeof(T) > 65536) waves /= 2;
  const dim3 gx((nc + waves - 1) / waves);
  const size_t lds = (size_t)waves * (nc + 128) * sizeof(T);
  const dim3 gy((nc + 63) / 64, (nseg + 3) / 4);
  if (bc == kDirichlet) {
    hipLaunchKernelGGL((k_pre_x<T, kDirichlet>), gx, dim3(64 * waves), lds, s, nc, e, pe, tmp, pt);
    hipLaunchKernelGGL((k_pre_y<T, kDirichlet>), gy, dim3(256), 0, s, nc, tmp, pt, c, pc, nseg);
  } else {
    hipLaunchKernelGGL((k_pre_x<T, kPeriodic>), gx, dim3(64 * waves), lds, s, nc, e, pe, tmp, pt);
    hipLaunchKernelGGL((k_pre_y<T, kPeriodic>), gy, dim3(256), 0, s, nc, tmp, pt, c, pc, nseg);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail(hipStream_t s, int bc, int nt, const T* uin, int pui, T* uout, int puo,
                       const T* f, int pf, T* cout, int pco, const double* inv,
                       const PrefilterTaps* taps) {
  const size_t bytes = tail_bytes(nt, sizeof(T));
  (void)taps;
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_tail<T, kDirichlet>), dim3(1), dim3(32, 32), bytes, s, nt, uin, pui, uout,
                       puo, f, pf, cout, pco, inv);
  else
    hipLaunchKernelGGL((k_tail<T, kPeriodic>), dim3(1), dim3(32, 32), bytes, s, nt, uin, pui, uout,
                       puo, f, pf, cout, pco, inv);
  return hipGetLastError();
}

#define MG_FUSED_INSTANTIATE(T)                                                                  \
  template hipError_t launch_down<T>(hipStream_t, int, int, const T*, int, T*, int, const T*,    \
                                     int, T*, int);                                              \
  template hipError_t launch_up<T>(hipStream_t, int, int, const T*, int, T*, int, const T*, int, \
                                   const T*, int);                                               \
  template hipError_t launch_prefilter_iir<T>(hipStream_t, int, int, const T*, int, T*, int, T*, \
                                              int);                                              \
  template hipError_t launch_tail<T>(hipStream_t, int, int, const T*, int, T*, int, const T*,    \
                                     int, T*, int, const double*, const PrefilterTaps*);

MG_FUSED_INSTANTIATE(double)
MG_FUSED_INSTANTIATE(float)

}  // namespace mg
