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
// B-spline prefilter constants: the pole z of (1, 4, 1)/6 and the gain g.
constexpr double kPrefZ = -0.26794919243112270647;  // sqrt(3) - 2
constexpr double kPrefG = 1.60769515458673623882;   // 12 - 6 sqrt(3)

}  // namespace mg
