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

// Along y: one wavefront filters 64 consecutive columns [c0, c0 + 64) over
// one segment of PreCfg<T>::S rows, one column per lane (coalesced).
template <typename T, int BC>
__device__ __forceinline__ void prey_wave(int nc, const T* __restrict__ in, int pi,
                                          T* __restrict__ out, int po, int c0, int seg, int lane) {
  using C = PreCfg<T>;
  const int col = c0 + lane;
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
template <typename T, int BC, int TR>
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

// Node q of the extended sequence of a tail line for q in [-Q - 1, 2Q)
// (Q the period of the extension; the prolongation reaches one node
// outside the line).
template <int BC>
__device__ __forceinline__ int tail_ext(int q, int nc, bool* neg) {
  return ext_node<BC>(q, nc, neg);
}

// Prefilter a tail grid: rows of src (in place), then columns into dst
// (pitch pd); each wavefront takes every (TR/2)-th line, with its own slice
// of the scratch grid for the causal values.
template <typename T, int BC, int TR>
__device__ __forceinline__ void tail_prefilter(T* src, T* tmp, T* dst, int pd, int nc) {
  const int t = tail_tid();
  const int lane = t & 63, wave = t >> 6;
  constexpr int kLineWaves = TR / 2;
  const ScanWeights<T> w(lane);
  T* buf = tmp + wave * (nc + 128);
  for (int line = wave; line < nc; line += kLineWaves)
    wave_line_prefilter<T, BC>(src + line * nc, 1, buf, src + line * nc, 1, nc, w, lane);
  __syncthreads();
  for (int line = wave; line < nc; line += kLineWaves)
    wave_line_prefilter<T, BC>(src + line, nc, buf, dst + line, pd, nc, w, lane);
  __syncthreads();
}

// u += P c on a tail grid of side n from coefficients c of side nc, in two
// separable passes through the scratch grid t: first along x for every
// coarse row of the extension that the y taps reach (rows -1 .. nc), then
// along y.
template <typename T, int BC, int TR>
__device__ __forceinline__ void tail_prolong_add(T* u, const T* c, T* t, int n) {
  const int nc = (n - 1) / 2 + 1;
  const int rows = nc + 2;  // coarse rows -1 .. nc
  for (int q = tail_tid(); q < rows * n; q += 32 * TR) {
    const int I = q / n - 1, j = q % n;
    bool ni;
    const int Ie = tail_ext<BC>(I, nc, &ni);
    int bj;
    T wj[4];
    const int nj = bspline_taps<T>(j, &bj, wj);
    T row = T(0);
    for (int b = 0; b < nj; ++b) {
      bool nb;
      const int J = ext_node<BC>(bj + b, nc, &nb);
      const T x = c[Ie * nc + J];
      row += wj[b] * (nb ? -x : x);
    }
    t[q] = ni ? -row : row;
  }
  __syncthreads();
  MG_TAIL_FOR(n, i, j, {
    if (tail_unknown<BC>(i, j, n)) {
      int bi;
      T wi[4];
      const int ni = bspline_taps<T>(i, &bi, wi);
      T v = T(0);
      for (int a = 0; a < ni; ++a) v += wi[a] * t[(bi + a + 1) * n + j];
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

// The whole tail for one problem by one workgroup of 32 TR threads; sm =
// LDS of tail_bytes(nt) bytes.
template <typename T, int BC, int TR>
__device__ __forceinline__ void tail_block(int nt, const T* __restrict__ uin, int pui,
                                           T* __restrict__ uout, int puo, const T* __restrict__ f,
                                           int pf, T* __restrict__ cout, int pco,
                                           const double* __restrict__ inv, T* sm) {
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
    tail_prefilter<T, BC, TR>(uc, tmp, uc, nc, nc);
    tail_prolong_add<T, BC, TR>(sm + tail_offu(nt, l), uc, tmp, n);
    tail_sweeps<T, BC, TR>(sm + tail_offu(nt, l), sm + tail_offf(nt, l), n, 4);
  }
  if (uout)
    MG_TAIL_FOR(nt, i, j, {
      if (tail_unknown<BC>(i, j, nt)) uout[(size_t)i * puo + j] = sm[i * nt + j];
    });
  if (cout) {
    __syncthreads();
    tail_prefilter<T, BC, TR>(sm, tmp, cout, pco, nt);
  }
}

// u and f of every tail level, then the scratch grid: the residual of the
// top level, the x-interpolated rows of a prolongation ((nt+1)/2 + 2 rows of
// nt), or the per-wavefront line buffers of the prefilter (TR/2 <= 16 of
// them).
__host__ __device__ inline size_t tail_bytes(int nt, size_t elem) {
  size_t tot = 0;
  for (int n = nt;; n = (n - 1) / 2 + 1) {
    tot += 2 * (size_t)n * n;
    if (n == 5) break;
  }
  const size_t scratch = ((size_t)nt * nt > (size_t)16 * (nt + 128) ? (size_t)nt * nt : (size_t)16 * (nt + 128));
  return (tot + scratch) * elem;
}

}  // namespace dev
}  // namespace mg
