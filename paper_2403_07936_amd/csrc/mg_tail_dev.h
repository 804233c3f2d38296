// Device functions of the prefilter and of the single-workgroup tail,
// shared by the standalone kernels (mg_fused.hip) and the persistent cycle
// kernel (mg_persist.hip).
#pragma once

#include "mg_device.h"

namespace mg {
namespace dev {

// B-spline prefilter along one axis: c = S^-1 e with S = (1, 4, 1)/6 on the
// extended sequence.  S^-1 = g / ((1 - z q^-1)(1 - z q)), z = sqrt(3) - 2,
// g = 12 - 6 sqrt(3): a causal recursion p_k = e_k + z p_{k-1} followed by an
// anti-causal one m_k = p_k + z m_{k+1}, c_k = g m_k.  A thread filters one
// chunk of S nodes of one line; both recursions start K nodes outside the
// chunk from a zero state, and the neglected state is below |z|^K of the
// data.
constexpr double kZ = kPrefZ;
constexpr double kG = kPrefG;

template <typename T>
struct PreCfg {
  static constexpr int K = sizeof(T) == 8 ? kPrefilterHalfTapsF64 : kPrefilterHalfTapsF32;
};

// B-spline prefilter of a whole level in one pass.  A workgroup owns a
// TH x TW tile of coefficients: it loads the tile with a K-node halo of the
// extended grid (ext_node_any: odd reflection or periodic wrap) into LDS,
// filters every row of the halo'd tile along x into a second LDS array and
// then the tile's columns along y.  Each thread of a pass takes S
// consecutive coefficients of one line; both recursions start K nodes
// outside its chunk from a zero state (chunk_iir), so the
// neglected state is below |z|^K of the data.
template <typename T>
struct PreTile {
  static constexpr int K = PreCfg<T>::K;
  // FP64: 48 columns so that the 28-node halo still fits two columns per
  // lane and the LDS (148 KB); 64 x 32 tiles with 8-node chunks loaded
  // 5.2x their coefficients against 4.1x here and ran 1.3x longer.
  static constexpr int S = 16;
  static constexpr int TW = sizeof(T) == 8 ? 48 : 64;
  static constexpr int TH = 4 * S;       // four column chunks per column
  static constexpr int HI = TH + 2 * K;  // rows of the halo'd tile
  static constexpr int WI = TW + 2 * K;  // columns of the halo'd tile
  static constexpr int PI = WI | 1;      // LDS pitches: odd, so that lanes on
  static constexpr int PM = TW + 1;      // consecutive rows hit distinct banks
  static constexpr size_t kLds = (size_t)(HI * PI + HI * PM) * sizeof(T);
  static_assert(WI <= 128, "a lane loads at most two columns of the halo'd tile");
  static_assert(TW % S == 0 && TH % S == 0, "whole chunks along both axes");
};

// S coefficients y from S + 2K consecutive nodes x[0], x[sx], ... of an
// extended line (chunk at offset K).
template <typename T, int S, int K>
__device__ __forceinline__ void chunk_iir(const T* x, int sx, T (&y)[S]) {
  const T z = T(kZ), g = T(kG);
  T p = T(0);
#pragma unroll
  for (int k = 0; k < K; ++k) p = x[k * sx] + z * p;
  T v[S + K];
#pragma unroll
  for (int k = 0; k < S + K; ++k) {
    p = x[(K + k) * sx] + z * p;
    v[k] = p;
  }
  T m = T(0);
#pragma unroll
  for (int k = S + K - 1; k >= 0; --k) {
    m = v[k] + z * m;
    if (k < S) y[k] = g * m;
  }
}

// One tile of the level prefilter by a workgroup of NT threads (a multiple
// of 64, at least 256); smem = PreTile<T>::kLds bytes of LDS.
template <typename T, int BC, int NT>
__device__ __forceinline__ void pre_tile_block(int nc, const T* __restrict__ in, int pi,
                                               T* __restrict__ out, int po, int tile, int tiles_x,
                                               T* smem) {
  using C = PreTile<T>;
  static_assert(NT % 64 == 0 && NT >= 256, "pre_tile_block needs whole wavefronts, at least four");
  constexpr int kWaves = NT / 64;
  __shared__ int rtab[C::HI], ctab[C::WI];
  T* si = smem;
  T* sm = si + C::HI * C::PI;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int y0 = ty * C::TH, x0 = tx * C::TW;
  // Stored node of every row and column of the halo'd tile, complemented
  // (~index) where the extension negates the value.
  for (int k = t; k < C::HI + C::WI; k += NT) {
    bool neg;
    if (k < C::HI) {
      const int r = ext_node_any<BC>(y0 - C::K + k, nc, &neg);
      rtab[k] = neg ? ~r : r;
    } else {
      const int c = ext_node_any<BC>(x0 - C::K + (k - C::HI), nc, &neg);
      ctab[k - C::HI] = neg ? ~c : c;
    }
  }
  __syncthreads();
  // Load: a wavefront per row, a lane per column (two for the last lanes).
  // Every load of the wavefront is issued before the first store to LDS
  // (rows past the tile repeat its last row and are not stored), so the
  // tile costs one memory round trip.
  constexpr int kRows = (C::HI + kWaves - 1) / kWaves;
  const int lx1 = lane + 64 < C::WI ? lane + 64 : C::WI - 1;
  const int ce0 = ctab[lane < C::WI ? lane : C::WI - 1], ce1 = ctab[lx1];
  const int c0 = ce0 < 0 ? ~ce0 : ce0, c1 = ce1 < 0 ? ~ce1 : ce1;
  T v0[kRows], v1[kRows];
  int re[kRows];
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int ly = wave + i * kWaves;
    re[i] = rtab[ly < C::HI ? ly : C::HI - 1];
  }
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const T* row = in + (size_t)(re[i] < 0 ? ~re[i] : re[i]) * pi;
    v0[i] = row[c0];
    v1[i] = row[c1];
  }
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int ly = wave + i * kWaves;
    if (ly < C::HI) {
      if (lane < C::WI) si[ly * C::PI + lane] = ((re[i] ^ ce0) < 0) ? -v0[i] : v0[i];
      if (lane + 64 < C::WI) si[ly * C::PI + lane + 64] = ((re[i] ^ ce1) < 0) ? -v1[i] : v1[i];
    }
  }
  __syncthreads();
  // Rows of the halo'd tile along x (lanes on consecutive rows).
  for (int w = t; w < C::HI * (C::TW / C::S); w += NT) {
    const int ly = w % C::HI, q = (w / C::HI) * C::S;
    T y[C::S];
    chunk_iir<T, C::S, C::K>(si + ly * C::PI + q, 1, y);
#pragma unroll
    for (int k = 0; k < C::S; ++k) {
      const int gx = x0 + q + k;
      sm[ly * C::PM + q + k] = (BC == kDirichlet && (gx == 0 || gx == nc - 1)) ? T(0) : y[k];
    }
  }
  __syncthreads();
  // Columns along y (lanes on consecutive columns) and the store.
  const int M = BC == kPeriodic ? nc - 1 : nc;
  if (t < C::TW * (C::TH / C::S)) {
    const int x = t % C::TW, q = (t / C::TW) * C::S, gx = x0 + x;
    T y[C::S];
    chunk_iir<T, C::S, C::K>(sm + q * C::PM + x, C::PM, y);
    if (gx < M) {
#pragma unroll
      for (int k = 0; k < C::S; ++k) {
        const int gy = y0 + q + k;
        if (gy < M) {
          const T v = (BC == kDirichlet && (gy == 0 || gy == nc - 1)) ? T(0) : y[k];
          out[(size_t)gy * po + gx] = v;
          if (BC == kPeriodic) {
            if (gy == 0) out[(size_t)(nc - 1) * po + gx] = v;
            if (gx == 0) out[(size_t)gy * po + nc - 1] = v;
            if (gy == 0 && gx == 0) out[(size_t)(nc - 1) * po + nc - 1] = v;
          }
        }
      }
    }
  }
}

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

// The tail's threads (TR rows of 32, linear id tid) cover a grid of side
// n <= 65 by visiting nodes (ty + TR a, tx + 32 b), tx = tid % 32,
// ty = tid / 32.
__device__ __forceinline__ int tail_tid() {
  return (int)(threadIdx.x + blockDim.x * threadIdx.y);
}
#define MG_TAIL_FOR(n, i, j, ...)                                          \
  do {                                                                     \
    const int ty_ = tail_tid() >> 5, tx_ = tail_tid() & 31;               \
    _Pragma("unroll") for (int a_ = 0; a_ < (65 + TR - 1) / TR; ++a_) {    \
      const int i = ty_ + TR * a_;                                          \
      if (i < (n)) {                                      \
        _Pragma("unroll") for (int b_ = 0; b_ < 3; ++b_) { \
          const int j = tx_ + 32 * b_;                    \
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

template <typename T, int BC, int TR>
__device__ __forceinline__ void tail_sweeps(T* u, const T* f, int n, int count) {
  const double hd = 1.0 / (double)(n - 1);
  const T h2 = T(hd * hd);
  // The unknowns of a side n <= 65 lie in rows and columns 0 .. 63, so the
  // 32 lanes of a row take the 32 nodes of the half-sweep's colour (every
  // lane busy, where a lane per column would leave half of them idle).
  static_assert(kTailMaxSide <= 65, "one node of a colour per lane and row");
  const int ty = tail_tid() >> 5, tx = tail_tid() & 31;
  for (int s = 0; s < count; ++s) {
    const int colour = s & 1;
#pragma unroll
    for (int a = 0; a < (64 + TR - 1) / TR; ++a) {
      const int i = ty + TR * a;
      const int j = 2 * tx + ((i + colour) & 1);
      if (i < n && j < n && tail_unknown<BC>(i, j, n)) {
        const T sum = ((u[wrap_prev<BC>(i, n) * n + j] + u[wrap_next<BC>(i, n) * n + j]) +
                       u[i * n + wrap_prev<BC>(j, n)]) +
                      u[i * n + wrap_next<BC>(j, n)];
        u[i * n + j] = (h2 * f[i * n + j] + sum) * T(0.25);
      }
    }
    __syncthreads();
  }
}

// r = f - A u into r (pitch n, unknown nodes only), then f_c = FW(r).
// Only rows and columns 0 .. 63 of r are read (a coarse unknown I <= 31
// reaches fine row 2I + 1 <= 63; periodic wraps reach n - 2 <= 63), so
// each thread makes both columns 2tx, 2tx + 1 of a row; and only the coarse
// unknowns I, J <= 31 are written (the rest of f_c is never read).
template <typename T, int BC, int TR>
__device__ __forceinline__ void tail_restrict(const T* u, const T* f, T* r, T* fc, int n) {
  const T inv_h2 = T((double)(n - 1) * (double)(n - 1));
  const int ty = tail_tid() >> 5, tx = tail_tid() & 31;
  static_assert(kTailMaxSide <= 65, "rows and columns 0 .. 63");
#pragma unroll
  for (int a = 0; a < (64 + TR - 1) / TR; ++a) {
    const int i = ty + TR * a;
    if (i < n - 1) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int j = 2 * tx + c;
        if (j < n - 1) {
          T v = T(0);
          if (tail_unknown<BC>(i, j, n)) {
            const T s = ((u[wrap_prev<BC>(i, n) * n + j] + u[wrap_next<BC>(i, n) * n + j]) +
                         u[i * n + wrap_prev<BC>(j, n)]) +
                        u[i * n + wrap_next<BC>(j, n)];
            v = f[i * n + j] - (T(4) * u[i * n + j] - s) * inv_h2;
          }
          r[i * n + j] = v;
        }
      }
    }
  }
  __syncthreads();
  const int nc = (n - 1) / 2 + 1;
#pragma unroll
  for (int a = 0; a < (32 + TR - 1) / TR; ++a) {
    const int I = ty + TR * a, J = tx;
    if (I < nc && J < nc && tail_unknown<BC>(I, J, nc)) {
      const int i = 2 * I, j = 2 * J;
      const int im = wrap_prev<BC>(i, n), ip = wrap_next<BC>(i, n);
      const int jm = wrap_prev<BC>(j, n), jp = wrap_next<BC>(j, n);
      const T edges = ((r[im * n + j] + r[ip * n + j]) + r[i * n + jm]) + r[i * n + jp];
      const T corners = ((r[im * n + jm] + r[im * n + jp]) + r[ip * n + jm]) + r[ip * n + jp];
      fc[I * nc + J] = ((T(4) * r[i * n + j] + T(2) * edges) + corners) * T(0.0625);
    }
  }
  __syncthreads();
}

// Node q of the extended sequence of a tail line for q in [-Q - 1, 2Q)
// (Q the period of the extension; the prolongation reaches one node
// outside the line).
template <int BC>
__device__ __forceinline__ int tail_ext(int q, int nc, bool* neg) {
  return ext_node<BC>(q, nc, neg);
}

// Coefficients of a coarse region, for an up pass that prefilters its own
// spline support: c on the extended-grid rows [ry0, ry0 + RH) and columns
// [rx0, rx0 + RW) (indices may lie outside [0, nc): the extension of c) into
// out (pitch po), from the coarse values `in` (pitch pi), by the chunked
// recursions of pre_tile_block; smem = PreRegion<...>::kLds bytes of LDS.
// On a Dirichlet grid the coefficients of boundary nodes are 0, as there.
template <typename T, int RH, int RW>
struct PreRegion {
  static constexpr int K = PreCfg<T>::K;
  static constexpr int S = sizeof(T) == 8 ? 8 : 16;
  static constexpr int CX = (RW + S - 1) / S, CY = (RH + S - 1) / S;  // chunks per line
  static constexpr int WO = CX * S, HO = CY * S;                      // padded outputs
  static constexpr int HI = HO + 2 * K, WI = WO + 2 * K;
  static constexpr int PI = WI | 1, PM = WO + 1;
  static constexpr size_t kLds = (size_t)(HI * PI + HI * PM) * sizeof(T);
  static_assert(WI <= 128, "a lane loads at most two columns of the region");
};

template <typename T, int BC, int NT, int RH, int RW>
__device__ __forceinline__ void prefilter_region(int nc, const T* __restrict__ in, int pi, int ry0,
                                                 int rx0, T* out, int po, T* smem) {
  using C = PreRegion<T, RH, RW>;
  constexpr int kWaves = NT / 64;
  __shared__ int rtab[C::HI], ctab[C::WI];
  T* si = smem;
  T* sm = si + C::HI * C::PI;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int k = t; k < C::HI + C::WI; k += NT) {
    bool neg;
    if (k < C::HI) {
      const int r = ext_node_any<BC>(ry0 - C::K + k, nc, &neg);
      rtab[k] = neg ? ~r : r;
    } else {
      const int c = ext_node_any<BC>(rx0 - C::K + (k - C::HI), nc, &neg);
      ctab[k - C::HI] = neg ? ~c : c;
    }
  }
  __syncthreads();
  constexpr int kRows = (C::HI + kWaves - 1) / kWaves;
  const int lx1 = lane + 64 < C::WI ? lane + 64 : C::WI - 1;
  const int ce0 = ctab[lane < C::WI ? lane : C::WI - 1], ce1 = ctab[lx1];
  const int c0 = ce0 < 0 ? ~ce0 : ce0, c1 = ce1 < 0 ? ~ce1 : ce1;
  T v0[kRows], v1[kRows];
  int re[kRows];
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int ly = wave + i * kWaves;
    re[i] = rtab[ly < C::HI ? ly : C::HI - 1];
  }
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const T* row = in + (size_t)(re[i] < 0 ? ~re[i] : re[i]) * pi;
    v0[i] = row[c0];
    v1[i] = row[c1];
  }
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int ly = wave + i * kWaves;
    if (ly < C::HI) {
      if (lane < C::WI) si[ly * C::PI + lane] = ((re[i] ^ ce0) < 0) ? -v0[i] : v0[i];
      if (lane + 64 < C::WI) si[ly * C::PI + lane + 64] = ((re[i] ^ ce1) < 0) ? -v1[i] : v1[i];
    }
  }
  __syncthreads();
  auto boundary = [&](int e) {  // table entry of a node: a Dirichlet boundary node?
    const int j = e < 0 ? ~e : e;
    return BC == kDirichlet && (j == 0 || j == nc - 1);
  };
  for (int w = t; w < C::HI * C::CX; w += NT) {
    const int ly = w % C::HI, q = (w / C::HI) * C::S;
    T y[C::S];
    chunk_iir<T, C::S, C::K>(si + ly * C::PI + q, 1, y);
#pragma unroll
    for (int k = 0; k < C::S; ++k)
      sm[ly * C::PM + q + k] = boundary(ctab[C::K + q + k]) ? T(0) : y[k];
  }
  __syncthreads();
  for (int w = t; w < RW * C::CY; w += NT) {
    const int x = w % RW, q = (w / RW) * C::S;
    T y[C::S];
    chunk_iir<T, C::S, C::K>(sm + q * C::PM + x, C::PM, y);
#pragma unroll
    for (int k = 0; k < C::S; ++k)
      if (q + k < RH) out[(q + k) * po + x] = boundary(rtab[C::K + q + k]) ? T(0) : y[k];
  }
  __syncthreads();
}

// Prefilter of the tail grids by per-thread chunks.  A thread takes S
// consecutive coefficients q0 .. q0 + S - 1 of one line: the causal
// recursion starts K nodes before the chunk from a zero state and runs K
// nodes past it, the anti-causal one starts there from a zero state (the
// truncation of the level prefilter, chunk_iir).  Extended-sequence
// nodes come from a table built once per call: entry q + K, q in
// [-K, nc + S + K), holds the stored node of ext_node_any, complemented
// (~index) where the extension negates the value.
template <typename T>
struct TailPre {
  static constexpr int K = PreCfg<T>::K;
  static constexpr int S = sizeof(T) == 8 ? 8 : 16;
  static constexpr int kTable = kTailMaxSide + S + 2 * K;
};

template <typename T, int BC>
__device__ __forceinline__ void tail_chunk(const T* src, int ss, T* dst, int ds, int nc, int q0,
                                           const int* tbl) {
  constexpr int K = TailPre<T>::K, S = TailPre<T>::S;
  const T z = T(kZ), g = T(kG);
  auto at = [&](int k) {  // node q0 - K + k of the extended line
    const int e = tbl[q0 + k];
    const T x = src[(e < 0 ? ~e : e) * ss];
    return e < 0 ? -x : x;
  };
  T p = T(0);
#pragma unroll
  for (int k = 0; k < K; ++k) p = at(k) + z * p;
  T v[S + K];
#pragma unroll
  for (int k = 0; k < S + K; ++k) {
    p = at(K + k) + z * p;
    v[k] = p;
  }
  T m = T(0);
#pragma unroll
  for (int k = S + K - 1; k >= 0; --k) {
    m = v[k] + z * m;
    v[k] = m;
  }
  const int M = BC == kPeriodic ? nc - 1 : nc;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const int q = q0 + k;
    if (q < M) {
      T y = g * v[k];
      if (BC == kDirichlet && (q == 0 || q == nc - 1)) y = T(0);
      dst[q * ds] = y;
      if (BC == kPeriodic && q == 0) dst[(nc - 1) * ds] = y;
    }
  }
}

// Sides 5 to 33: the prefilter as a dense matrix M (side NC, in LDS; see
// prefilter_matrix: the exact inverse, every extension folded onto the
// stored nodes), rows then columns, two barrier phases in all.  On these
// sides chunked recursions are all latency.
template <typename T, int BC, int TR, int NC>
__device__ __forceinline__ void tail_prefilter_mat(const T* src, T* tmp, T* dst, int pd,
                                                   const T* M) {
  const int t = tail_tid();
  constexpr int rows = BC == kPeriodic ? NC - 1 : NC;  // the seam row is never read
  for (int w = t; w < rows * NC; w += 32 * TR) {
    const int line = w / NC, q = w - line * NC;
    T acc = T(0);
#pragma unroll 11
    for (int k = 0; k < NC; ++k) acc += M[q * NC + k] * src[line * NC + k];
    tmp[line * NC + q] = acc;
  }
  __syncthreads();
  for (int w = t; w < NC * NC; w += 32 * TR) {
    const int q = w / NC, line = w - q * NC;
    T acc = T(0);
#pragma unroll 11
    for (int k = 0; k < rows; ++k) acc += M[q * NC + k] * tmp[k * NC + line];
    dst[q * pd + line] = acc;
  }
  __syncthreads();
}

// Prefilter a tail grid src (side nc, pitch nc): rows into the scratch grid
// tmp, then columns into dst (pitch pd; may be src).  MAT = false leaves the
// matrix form out of a call site that only sees the top side.  mat: the
// dense matrices of the sides 5, 9, 17, 33 (LDS, tail_mat_offset).
template <typename T, int BC, int TR, bool MAT = true>
__device__ __forceinline__ void tail_prefilter(const T* src, T* tmp, T* dst, int pd, int nc,
                                               const T* mat) {
  if (MAT) {
    if (nc == 5) return tail_prefilter_mat<T, BC, TR, 5>(src, tmp, dst, pd, mat);
    if (nc == 9) return tail_prefilter_mat<T, BC, TR, 9>(src, tmp, dst, pd, mat + tail_mat_offset(9));
    if (nc == 17)
      return tail_prefilter_mat<T, BC, TR, 17>(src, tmp, dst, pd, mat + tail_mat_offset(17));
    if (nc == 33)
      return tail_prefilter_mat<T, BC, TR, 33>(src, tmp, dst, pd, mat + tail_mat_offset(33));
  }
  using C = TailPre<T>;
  __shared__ int tbl[C::kTable];
  const int t = tail_tid();
  for (int q = t; q < nc + C::S + 2 * C::K; q += 32 * TR) {
    bool neg;
    const int j = ext_node_any<BC>(q - C::K, nc, &neg);
    tbl[q] = neg ? ~j : j;
  }
  __syncthreads();
  // Rows: the periodic seam row is never read by the column pass.
  const int rows = BC == kPeriodic ? nc - 1 : nc;
  const int chunks = (nc + C::S - 1) / C::S;
  for (int w = t; w < rows * chunks; w += 32 * TR) {
    const int line = w % rows, q0 = (w / rows) * C::S;
    tail_chunk<T, BC>(src + line * nc, 1, tmp + line * nc, 1, nc, q0, tbl);
  }
  __syncthreads();
  for (int w = t; w < nc * chunks; w += 32 * TR) {
    const int line = w % nc, q0 = (w / nc) * C::S;
    tail_chunk<T, BC>(tmp + line, nc, dst + line, pd, nc, q0, tbl);
  }
  __syncthreads();
}

// u += P c on a tail grid of side n from coefficients c of side nc, in two
// separable passes through the scratch grid t: first along x for every
// coarse row of the extension that the y taps reach (rows -1 .. nc), then
// along y.
template <typename T, int BC, int TR>
__device__ __forceinline__ void tail_prolong_add(T* u, const T* c, T* t, int n) {
  const int nc = (n - 1) / 2 + 1;
  const int ty = tail_tid() >> 5, tx = tail_tid() & 31;
  // The unknowns of a side n <= 65 lie in rows and columns 0 .. 63: fine
  // columns 2J, 2J + 1 for J < 32, read from coarse rows -1 .. nc (scratch
  // rows 0 .. nc + 1).  Each thread makes both fine columns of its J from
  // the four coarse values J - 1 .. J + 2.
  static_assert(kTailMaxSide <= 65, "fine columns 2J, 2J + 1 with J < 32");
  for (int a = 0; a < (kTailMaxSide / 2 + 3 + TR - 1) / TR; ++a) {
    const int r = ty + TR * a;
    if (r < nc + 2 && tx < nc) {
      bool ni, n0, n1, n2, n3;
      const int Ie = tail_ext<BC>(r - 1, nc, &ni);
      const T* cr = c + Ie * nc;
      const int j0 = ext_node<BC>(tx - 1, nc, &n0), j1 = ext_node<BC>(tx, nc, &n1);
      const int j2 = ext_node<BC>(tx + 1, nc, &n2), j3 = ext_node<BC>(tx + 2, nc, &n3);
      T x0 = cr[j0], x1 = cr[j1], x2 = cr[j2], x3 = cr[j3];
      x0 = (n0 != ni) ? -x0 : x0;
      x1 = (n1 != ni) ? -x1 : x1;
      x2 = (n2 != ni) ? -x2 : x2;
      x3 = (n3 != ni) ? -x3 : x3;
      const int j = 2 * tx;
      t[r * n + j] = (T(1.0 / 6.0) * x0 + T(4.0 / 6.0) * x1) + T(1.0 / 6.0) * x2;
      if (j + 1 < n)
        t[r * n + j + 1] =
            ((T(1.0 / 48.0) * x0 + T(23.0 / 48.0) * x1) + T(23.0 / 48.0) * x2) + T(1.0 / 48.0) * x3;
    }
  }
  __syncthreads();
  // Fine rows 2I, 2I + 1 for I < 32 from scratch rows I .. I + 3 (coarse
  // rows I - 1 .. I + 2), columns 0 .. 63.
  for (int a = 0; a < (kTailMaxSide / 2 + TR - 1) / TR; ++a) {
    const int I = ty + TR * a;
    if (I < nc - 1) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = tx + 32 * b;
        if (j < n) {
          const T* tr = t + I * n + j;
          const T y0 = tr[0], y1 = tr[n], y2 = tr[2 * n], y3 = tr[3 * n];
          const int i = 2 * I;
          if (tail_unknown<BC>(i, j, n))
            u[i * n + j] += (T(1.0 / 6.0) * y0 + T(4.0 / 6.0) * y1) + T(1.0 / 6.0) * y2;
          if (tail_unknown<BC>(i + 1, j, n))
            u[(i + 1) * n + j] +=
                ((T(1.0 / 48.0) * y0 + T(23.0 / 48.0) * y1) + T(23.0 / 48.0) * y2) +
                T(1.0 / 48.0) * y3;
        }
      }
    }
  }
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

// Elements of the tail's scratch grid (defined with tail_bytes).
__host__ __device__ inline int tail_scratch_elems(int nt, size_t elem);

// The whole tail for one problem by one workgroup of 32 TR threads; sm =
// LDS of tail_bytes(nt) bytes.
template <typename T, int BC, int TR>
__device__ __forceinline__ void tail_block(int nt, const T* __restrict__ uin, int pui,
                                           T* __restrict__ uout, int puo, const T* __restrict__ f,
                                           int pf, T* __restrict__ cout, int pco,
                                           const double* __restrict__ inv, T* sm) {
  const int L = tail_levels(nt);
  T* tmp = sm + tail_offu(nt, L);
  T* mat = tmp + tail_scratch_elems(nt, sizeof(T));
  MG_TAIL_FOR(nt, i, j, {
    sm[i * nt + j] = uin ? uin[(size_t)i * pui + j] : T(0);
    sm[nt * nt + i * nt + j] = f[(size_t)i * pf + j];
  });
  for (int q = tail_tid(); q < kTailMatElems; q += 32 * TR) mat[q] = T(inv[kTailMatOffset + q]);
  __syncthreads();
  for (int l = 0; l + 1 < L; ++l) {
    const int n = tail_side(nt, l);
    T* u = sm + tail_offu(nt, l);
    T* ff = sm + tail_offf(nt, l);
    if (l > 0) {
      MG_TAIL_FOR(n, i, j, { u[i * n + j] = T(0); });
      __syncthreads();
    }
    tail_sweeps<T, BC, TR>(u, ff, n, 4);
    tail_restrict<T, BC, TR>(u, ff, tmp, sm + tail_offf(nt, l + 1), n);
  }
  {
    // 5 x 5 direct solve in FP64.
    T* u = sm + tail_offu(nt, L - 1);
    const T* ff = sm + tail_offf(nt, L - 1);
    constexpr int m = BC == kDirichlet ? 9 : 16;
    const int t = tail_tid();
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
    tail_prefilter<T, BC, TR>(uc, tmp, uc, nc, nc, mat);
    tail_prolong_add<T, BC, TR>(sm + tail_offu(nt, l), uc, tmp, n);
    tail_sweeps<T, BC, TR>(sm + tail_offu(nt, l), sm + tail_offf(nt, l), n, 4);
  }
  if (uout)
    MG_TAIL_FOR(nt, i, j, {
      if (tail_unknown<BC>(i, j, nt)) uout[(size_t)i * puo + j] = sm[i * nt + j];
    });
  if (cout) {
    __syncthreads();
    tail_prefilter<T, BC, TR, false>(sm, tmp, cout, pco, nt, mat);
  }
}

// u and f of every tail level, then the scratch grid of at least nt x nt
// (the residual of the top level, the x-interpolated rows of a prolongation
// ((nt+1)/2 + 2 rows of nt), or the row pass of the prefilter), then the
// dense prefilter matrices of the sides 5, 9, 17 and 33.
__host__ __device__ inline size_t tail_bytes(int nt, size_t elem) {
  size_t tot = 0;
  for (int n = nt;; n = (n - 1) / 2 + 1) {
    tot += 2 * (size_t)n * n;
    if (n == 5) break;
  }
  return (tot + (size_t)tail_scratch_elems(nt, elem) + kTailMatElems) * elem;
}
__host__ __device__ inline int tail_scratch_elems(int nt, size_t elem) {
  (void)elem;
  return nt * nt;
}

}  // namespace dev
}  // namespace mg
