// Fused, LDS-tiled kernels of the V(2,2) cycle for gfx950.
//
//   k_down  : 2 red-black sweeps + residual + full-weighting restriction of
//             one level in one pass (temporal blocking: the tile is loaded
//             with a 6-node halo, each half-sweep invalidates one more ring).
//   k_up    : cubic-spline evaluation of the coarse correction, u += P e_c,
//             then 2 red-black sweeps, in one pass (4-node halo).
//   k_pre_tile : B-spline prefilter of a coarse level (the non-local part of
//             the spline) in one pass over LDS tiles, as causal + anti-causal
//             first-order recursions over short chunks with a warm-up run
//             long enough that the truncated state is below the working
//             precision.
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
#include "mg_tail_dev.h"

namespace mg {
namespace {

// Threads of the LDS-tiled passes: sixteen wavefronts per tile hide its load
// and LDS latencies (with 256 the tuner rarely picks these passes, and the
// 4097^2 cycle is 2.5 % (mixed) to 4 % (FP64) slower).
constexpr int kThreads = 1024;
constexpr int kTailThreads = 1024;
// Tile of the LDS up pass and the coarse support its spline reads.
constexpr int kUpTX = 64, kUpTY = 32, kUpH = 4;
constexpr int kUpCW = kUpTX / 2 + kUpH + 3, kUpCH = kUpTY / 2 + kUpH + 3;

// Loads a W x HH tile whose node (0, 0) is global node (gy0, gx0) into s:
// periodic wrap, zero outside a Dirichlet grid, all zero if `zero`.  Every
// load of the thread is issued (from clamped, in-bounds indices) before the
// first store to LDS, so the tile costs one memory round trip.
template <typename T, int BC, int W, int HH>
__device__ __forceinline__ void load_tile(T* s, const T* __restrict__ g, int pg, int n, int gy0,
                                          int gx0, bool zero) {
  constexpr int kIt = (W * HH + kThreads - 1) / kThreads;
  if (zero) {
#pragma unroll
    for (int i = 0; i < kIt; ++i) {
      const int k = threadIdx.x + i * kThreads;
      if (k < W * HH) s[k] = T(0);
    }
    return;
  }
  const int N = n - 1;
  T v[kIt];
#pragma unroll
  for (int i = 0; i < kIt; ++i) {
    const int k0 = threadIdx.x + i * kThreads;
    const int k = k0 < W * HH ? k0 : W * HH - 1;
    const int ly = k / W, lx = k - ly * W;
    int gy = gy0 + ly, gx = gx0 + lx;
    if constexpr (BC == kPeriodic) {
      gy = gy < 0 ? gy + N : (gy >= N ? gy - N : gy);
      gx = gx < 0 ? gx + N : (gx >= N ? gx - N : gx);
    } else {
      gy = gy < 0 ? 0 : (gy > N ? N : gy);
      gx = gx < 0 ? 0 : (gx > N ? N : gx);
    }
    v[i] = g[(size_t)gy * pg + gx];
  }
#pragma unroll
  for (int i = 0; i < kIt; ++i) {
    const int k = threadIdx.x + i * kThreads;
    if (k < W * HH) {
      T x = v[i];
      if constexpr (BC == kDirichlet) {
        const int ly = k / W, lx = k - ly * W;
        const int gy = gy0 + ly, gx = gx0 + lx;
        if (gy < 0 || gy > N || gx < 0 || gx > N) x = T(0);
      }
      s[k] = x;
    }
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
           T h2, T inv_h2, const CallerArgs* ca) {
  if constexpr (sizeof(T) == sizeof(double))
    if (ca) {
      if (uin) uin = ca->u;
      f = ca->f;
    }
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

// PRE: c holds the coarse correction itself, and the tile computes the
// B-spline coefficients of its own support (prefilter_region) in place of a
// separate prefilter pass over the level.
template <typename T, int BC, int TX, int TY, bool PRE>
__global__ void __launch_bounds__(kThreads)
    k_up(int n, const T* __restrict__ uin, T* __restrict__ uout, int pui, int puo,
         const T* __restrict__ f, int pf, const T* __restrict__ c, int pc, int tiles_x, int ntiles,
         T h2, const CallerArgs* ca) {
  if constexpr (sizeof(T) == sizeof(double))
    if (ca) uout = ca->u, f = ca->f;
  constexpr int H = kUpH, W = TX + 2 * H, HH = TY + 2 * H;
  constexpr int CW = TX / 2 + H + 3, CH = TY / 2 + H + 3;
  static_assert(!PRE || (CW == kUpCW && CH == kUpCH), "launch_up sizes the prefilter LDS");
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
  if constexpr (PRE) {
    extern __shared__ __align__(16) unsigned char pre_lds[];
    dev::prefilter_region<T, BC, kThreads, CH, CW>(nc, c, pc, cy0, cx0, sc, CW,
                                                   reinterpret_cast<T*>(pre_lds));
  } else {
    // Coarse coefficients of the tile's spline support (all loads first).
    constexpr int kIt = (CW * CH + kThreads - 1) / kThreads;
    T v[kIt];
    bool neg[kIt];
#pragma unroll
    for (int i = 0; i < kIt; ++i) {
      const int k0 = threadIdx.x + i * kThreads;
      const int k = k0 < CW * CH ? k0 : CW * CH - 1;
      const int cy = k / CW, cx = k - cy * CW;
      bool ny, nx;
      const int I = ext_node<BC>(cy0 + cy, nc, &ny);
      const int J = ext_node<BC>(cx0 + cx, nc, &nx);
      v[i] = c[(size_t)I * pc + J];
      neg[i] = ny != nx;
    }
#pragma unroll
    for (int i = 0; i < kIt; ++i) {
      const int k = threadIdx.x + i * kThreads;
      if (k < CW * CH) sc[k] = neg[i] ? -v[i] : v[i];
    }
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

using namespace dev;

// 1024 threads per tile: one LDS tile per compute unit fits (FP64) or two
// (FP32), and the sixteen wavefronts hide the latency of the tile's loads
// and of the recursion chains (256 threads: 2049^2 FP32 22.5 us, FP64
// 66.7 us; 1024: 18.4 and 54.6 us).
constexpr int kPreThreads = 1024;

template <typename T, int BC>
__global__ void __launch_bounds__(kPreThreads)
    k_pre_tile(int nc, const T* __restrict__ in, int pi, T* __restrict__ out, int po, int tiles_x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // Consecutive tiles on one XCD, so that the halos neighbouring tiles share
  // are read from that XCD's L2 rather than again from HBM.
  pre_tile_block<T, BC, kPreThreads>(nc, in, pi, out, po, xcd_tile(blockIdx.x, gridDim.x), tiles_x,
                             reinterpret_cast<T*>(smem_raw));
}

template <typename T, int BC>
__global__ void __launch_bounds__(kTailThreads)
    k_tail(int nt, const T* __restrict__ uin, int pui, T* __restrict__ uout, int puo,
           const T* __restrict__ f, int pf, T* __restrict__ cout, int pco,
           const double* __restrict__ inv, const CallerArgs* ca) {
  if constexpr (sizeof(T) == sizeof(double))
    if (ca) {
      if (uin) uin = ca->u;
      if (uout) uout = ca->u;
      f = ca->f;
    }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  tail_block<T, BC, kTailThreads / 32>(nt, uin, pui, uout, puo, f, pf, cout, pco, inv,
                                       reinterpret_cast<T*>(smem_raw));
}

template <typename T, int BC>
struct Fused {
  static constexpr int TX = 64, TY = 32;
};

}  // namespace

int fused_tile_x() { return 64; }
int fused_tile_y() { return 32; }

hipError_t fused_init() {
  hipError_t e0;
  e0 = hipFuncSetAttribute((const void*)k_pre_tile<double, kDirichlet>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)PreTile<double>::kLds);
  if (e0 != hipSuccess) return e0;
  e0 = hipFuncSetAttribute((const void*)k_pre_tile<double, kPeriodic>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)PreTile<double>::kLds);
  if (e0 != hipSuccess) return e0;
  e0 = hipFuncSetAttribute((const void*)k_pre_tile<float, kDirichlet>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)PreTile<float>::kLds);
  if (e0 != hipSuccess) return e0;
  e0 = hipFuncSetAttribute((const void*)k_pre_tile<float, kPeriodic>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)PreTile<float>::kLds);
  if (e0 != hipSuccess) return e0;
  {
    const int l64 = (int)PreRegion<double, kUpCH, kUpCW>::kLds;
    const int l32 = (int)PreRegion<float, kUpCH, kUpCW>::kLds;
    hipError_t e1 = hipFuncSetAttribute((const void*)k_up<double, kDirichlet, kUpTX, kUpTY, true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, l64);
    if (e1 == hipSuccess)
      e1 = hipFuncSetAttribute((const void*)k_up<double, kPeriodic, kUpTX, kUpTY, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, l64);
    if (e1 == hipSuccess)
      e1 = hipFuncSetAttribute((const void*)k_up<float, kDirichlet, kUpTX, kUpTY, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, l32);
    if (e1 == hipSuccess)
      e1 = hipFuncSetAttribute((const void*)k_up<float, kPeriodic, kUpTX, kUpTY, true>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, l32);
    if (e1 != hipSuccess) return e1;
  }
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
                       const T* f, int pf, T* fc, int pfc, const CallerArgs* ca) {
  constexpr int TX = 64, TY = 32;
  const int tx = tiles_along(n, bc, TX), ty = tiles_along(n, bc, TY);
  const int nt = tx * ty;
  const double hd = 1.0 / (double)(n - 1);
  const T h2 = T(hd * hd), inv_h2 = T((double)(n - 1) * (double)(n - 1));
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_down<T, kDirichlet, TX, TY>), dim3(nt), dim3(kThreads), 0, s, n, uin,
                       uout, pui, puo, f, pf, fc, pfc, tx, nt, h2, inv_h2, ca);
  else
    hipLaunchKernelGGL((k_down<T, kPeriodic, TX, TY>), dim3(nt), dim3(kThreads), 0, s, n, uin, uout,
                       pui, puo, f, pf, fc, pfc, tx, nt, h2, inv_h2, ca);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_up(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout, int puo,
                     const T* f, int pf, const T* c, int pc, bool pre, const CallerArgs* ca) {
  constexpr int TX = kUpTX, TY = kUpTY;
  const int tx = tiles_along(n, bc, TX), ty = tiles_along(n, bc, TY);
  const int nt = tx * ty;
  const double hd = 1.0 / (double)(n - 1);
  const T h2 = T(hd * hd);
  const size_t lds = pre ? dev::PreRegion<T, kUpCH, kUpCW>::kLds : 0;
#define MG_TILE_UP(BCV, PREV)                                                                    \
  hipLaunchKernelGGL((k_up<T, BCV, TX, TY, PREV>), dim3(nt), dim3(kThreads), lds, s, n, uin, uout, \
                     pui, puo, f, pf, c, pc, tx, nt, h2, ca)
  if (bc == kDirichlet && pre)
    MG_TILE_UP(kDirichlet, true);
  else if (bc == kDirichlet)
    MG_TILE_UP(kDirichlet, false);
  else if (pre)
    MG_TILE_UP(kPeriodic, true);
  else
    MG_TILE_UP(kPeriodic, false);
#undef MG_TILE_UP
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prefilter_iir(hipStream_t s, int bc, int nc, const T* e, int pe, T* tmp, int pt,
                                T* c, int pc) {
  using C = PreTile<T>;
  (void)tmp;
  (void)pt;
  const int extent = bc == kPeriodic ? nc - 1 : nc;
  const int tx = (extent + C::TW - 1) / C::TW, ty = (extent + C::TH - 1) / C::TH;
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_pre_tile<T, kDirichlet>), dim3(tx * ty), dim3(kPreThreads), C::kLds, s, nc, e, pe,
                       c, pc, tx);
  else
    hipLaunchKernelGGL((k_pre_tile<T, kPeriodic>), dim3(tx * ty), dim3(kPreThreads), C::kLds, s, nc, e, pe,
                       c, pc, tx);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail(hipStream_t s, int bc, int nt, const T* uin, int pui, T* uout, int puo,
                       const T* f, int pf, T* cout, int pco, const double* inv,
                       const PrefilterTaps* taps, const CallerArgs* ca) {
  const size_t bytes = tail_bytes(nt, sizeof(T));
  (void)taps;
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_tail<T, kDirichlet>), dim3(1), dim3(32, 32), bytes, s, nt, uin, pui, uout,
                       puo, f, pf, cout, pco, inv, ca);
  else
    hipLaunchKernelGGL((k_tail<T, kPeriodic>), dim3(1), dim3(32, 32), bytes, s, nt, uin, pui, uout,
                       puo, f, pf, cout, pco, inv, ca);
  return hipGetLastError();
}

#define MG_FUSED_INSTANTIATE(T)                                                                  \
  template hipError_t launch_down<T>(hipStream_t, int, int, const T*, int, T*, int, const T*,    \
                                     int, T*, int, const CallerArgs*);                           \
  template hipError_t launch_up<T>(hipStream_t, int, int, const T*, int, T*, int, const T*, int, \
                                   const T*, int, bool, const CallerArgs*);                      \
  template hipError_t launch_prefilter_iir<T>(hipStream_t, int, int, const T*, int, T*, int, T*, \
                                              int);                                              \
  template hipError_t launch_tail<T>(hipStream_t, int, int, const T*, int, T*, int, const T*,    \
                                     int, T*, int, const double*, const PrefilterTaps*,          \
                                     const CallerArgs*);

MG_FUSED_INSTANTIATE(double)
MG_FUSED_INSTANTIATE(float)

}  // namespace mg
