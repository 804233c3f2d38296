// Device-side helpers shared by the fused kernels.
#pragma once

#include "mg_internal.h"

namespace mg {

// Workgroups of a launch are dispatched round-robin over the 8 XCDs of the
// MI355X (workgroup b runs on XCD b % 8), each with its own L2.  Renumber
// them so that every XCD receives one contiguous run of tiles: neighbouring
// tiles, whose halos overlap, then share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  constexpr int kXcds = 8;
  const int per = nblocks / kXcds, rem = nblocks % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x * per + (x < rem ? x : rem) + k;
}

// Node q of the extended sequence of a level with nc nodes per side, for q
// in [-Q, 2Q): periodic grids wrap over N = nc-1 nodes (Q = N); Dirichlet
// grids use the odd extension about nodes 0 and nc-1 (period Q = 2(nc-1)).
// Returns the stored node index; *neg is set when the value changes sign.
template <int BC>
__device__ __forceinline__ int ext_node(int q, int nc, bool* neg) {
  if constexpr (BC == kPeriodic) {
    const int N = nc - 1;
    q = q < 0 ? q + N : q;
    q = q >= N ? q - N : q;
    q = q >= N ? q - N : q;
    *neg = false;
    return q;
  } else {
    const int Q = 2 * (nc - 1);
    bool s = false;
    if (q < 0) {
      q = -q;
      s = true;
    }
    q = q >= Q ? q - Q : q;
    if (q > nc - 1) {
      q = Q - q;
      s = !s;
    }
    *neg = s;
    return q;
  }
}

// Same mapping for any q (slower: uses a modulo).
template <int BC>
__device__ __forceinline__ int ext_node_any(int q, int nc, bool* neg) {
  const int Q = BC == kPeriodic ? nc - 1 : 2 * (nc - 1);
  int r = q % Q;
  r = r < 0 ? r + Q : r;
  return ext_node<BC>(r, nc, neg);
}

// Cubic B-spline evaluation on one axis at fine node x (unwrapped index):
// coincident nodes use (1, 4, 1)/6 on coefficients base..base+2, midpoints
// (1, 23, 23, 1)/48 on base..base+3.  Returns the number of taps.
template <typename T>
__device__ __forceinline__ int bspline_taps(int x, int* base, T* w) {
  if ((x & 1) == 0) {
    *base = (x >> 1) - 1;
    w[0] = T(1.0 / 6.0);
    w[1] = T(4.0 / 6.0);
    w[2] = T(1.0 / 6.0);
    w[3] = T(0);
    return 3;
  }
  *base = ((x - 1) >> 1) - 1;
  w[0] = T(1.0 / 48.0);
  w[1] = T(23.0 / 48.0);
  w[2] = T(23.0 / 48.0);
  w[3] = T(1.0 / 48.0);
  return 4;
}

// ------------------------------------------------------------------------
// Wavefront-wide first-order recursion (the B-spline prefilter along a line).
//
// For z = sqrt(3) - 2 the causal recursion p_k = x_k + z p_{k-1} over 64
// consecutive nodes held one per lane is a weighted prefix sum,
// p_l = sum_{j <= l} z^(l-j) x_j + z^(l+1) p_in: four in-row steps with DPP
// row shifts by 1, 2, 4, 8 lanes, then the carries of rows 0, 1, 2 of 16
// lanes passed on with readlane, then the carry from the previous chunk.

template <int CTRL>
__device__ __forceinline__ float dpp_row(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_row(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

constexpr double kPrefZ = -0.26794919243112270647;  // sqrt(3) - 2
constexpr double kPrefG = 1.60769515458673623882;   // 12 - 6 sqrt(3)

template <typename T>
struct ScanWeights {
  T z1, z2, z4, z8;  // z^1, z^2, z^4, z^8
  T row;             // z^(lane % 16 + 1)
  T all;             // z^(lane + 1)
  __device__ explicit ScanWeights(int lane) {
    const double z = kPrefZ;
    z1 = T(z);
    z2 = T(z * z);
    z4 = T((z * z) * (z * z));
    z8 = T(((z * z) * (z * z)) * ((z * z) * (z * z)));
    double p = z;
    for (int k = 0; k < (lane & 15); ++k) p *= z;
    row = T(p);
    double q = z;
    for (int k = 0; k < lane; ++k) q *= z;
    all = T(q);
  }
};

// Inclusive weighted scan of one value per lane with carry-in `carry`
// (the recursion's value just before lane 0).  All 64 lanes must call it.
template <typename T>
__device__ __forceinline__ T wave_recursion(T x, T carry, const ScanWeights<T>& w, int lane) {
  T q = x;
  q += w.z1 * dpp_row<0x111>(q);  // row_shr:1
  q += w.z2 * dpp_row<0x112>(q);  // row_shr:2
  q += w.z4 * dpp_row<0x114>(q);  // row_shr:4
  q += w.z8 * dpp_row<0x118>(q);  // row_shr:8
  const T c15 = read_lane(q, 15);
  if ((lane >> 4) == 1) q += w.row * c15;
  const T c31 = read_lane(q, 31);
  if ((lane >> 4) == 2) q += w.row * c31;
  const T c47 = read_lane(q, 47);
  if ((lane >> 4) == 3) q += w.row * c47;
  return q + w.all * carry;
}

// Prefilter one line of a level with nc nodes per side (the extended
// sequence of ext_node_any) by one wavefront: src / dst with element
// strides ss / ds (dst may alias src), buf = scratch of >= M + 128 values,
// M = stored nodes of one period.  Causal pass left to right storing p in
// buf (starting 64 nodes before the line from a zero state, and running 64
// nodes past its end), then the anti-causal pass right to left.
template <typename T, int BC>
__device__ __forceinline__ void wave_line_prefilter(const T* src, int ss, T* buf, T* dst, int ds, int nc,
                                    const ScanWeights<T>& w, int lane) {
  const int M = BC == kPeriodic ? nc - 1 : nc;
  auto ext = [&](int q) {
    bool neg;
    const int j = ext_node_any<BC>(q, nc, &neg);
    const T v = src[j * ss];
    return neg ? -v : v;
  };
  T carry = T(0);
  {
    const T p = wave_recursion<T>(ext(lane - 64), T(0), w, lane);
    carry = read_lane(p, 63);
  }
  for (int k0 = 0; k0 < M + 64; k0 += 64) {
    const int q = k0 + lane;
    const T x = q < M ? src[q * ss] : ext(q);
    const T p = wave_recursion<T>(x, carry, w, lane);
    carry = read_lane(p, 63);
    buf[q] = p;
  }
  carry = T(0);
  const T g = T(kPrefG);
  for (int k1 = M + 64; k1 > 0; k1 -= 64) {
    const int q = k1 - 1 - lane;
    const T x = q >= 0 ? buf[q] : T(0);
    const T m = wave_recursion<T>(x, carry, w, lane);
    carry = read_lane(m, 63);
    if (q >= 0 && q < M) {
      T y = g * m;
      if (BC == kDirichlet && (q == 0 || q == nc - 1)) y = T(0);
      dst[q * ds] = y;
      if (BC == kPeriodic && q == 0) dst[(nc - 1) * ds] = y;
    }
  }
}

}  // namespace mg
