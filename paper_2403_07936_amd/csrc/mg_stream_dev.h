// Register-streaming down and up passes (device functions) for gfx950.
// Used by the standalone kernels (mg_stream.hip) and the persistent cycle
// kernel (mg_persist.hip).
//
// Each 64-lane wavefront owns a band of columns, two adjacent columns per
// lane (x0 = even, x1 = x0 + 1), and marches down a segment of rows.  With
// two columns per lane every red-black half-sweep updates exactly one node
// per lane per row, and which of the two it is depends only on the row, so
// the wavefront never diverges.  The steps of a pass are pipelined over the
// rows with fixed lags, each row held in registers for the few steps that
// need it:
//   down pass, at the step that loads row t:
//     red sweep on row t-1, black on t-2, red on t-3, black on t-4 (u final),
//     residual on row t-5, full weighting on the coarse row at fine row t-6;
//   up pass, at the step that loads row t:
//     u += P e_c on row t, red sweep on t-1, black on t-2, red on t-3,
//     black on t-4 (u final).
// Horizontal neighbours come from the adjacent lane by a cross-lane shuffle.
// The lanes at the band edges see no neighbour, and the error this causes
// moves inward one column per step, so only the inner columns of a band are
// written (the rest is a halo that the neighbouring band owns); the top and
// bottom of a segment likewise load halo rows.  The arithmetic and its
// order are those of the per-operation kernels.

#pragma once

#include "mg_device.h"

namespace mg {
namespace stream {

constexpr int kWaves = 4;           // independent wavefronts per workgroup
constexpr int kDownHalo = 6;        // columns on each side a down band does not own
constexpr int kDownOwned = 128 - 2 * kDownHalo;
constexpr int kUpHalo = 6;          // up pass: spline support + 4 half-sweeps
constexpr int kUpOwned = 112;       // owned columns [xw + 6, xw + 118)
// Rows are loaded this many steps before the step that first uses them.  The
// 16-slot row rings bound it: the down pass keeps rows t-6 .. t live (at
// most 9 ahead), the up pass rows t-5 .. t and its 8-slot FP64 ring rows
// t-4 .. (at most 7 ahead).  The wavefronts of a large level together keep
// enough loads in flight with a few rows each; 5 to 9 rows measured up to
// 2 % slower on 4097^2 than these.
constexpr int kAheadDown = 3;
constexpr int kAheadUp = 4;
static_assert(kAheadDown <= 9 && kAheadUp <= 7, "row rings hold the rows in flight");

// Cross-lane moves by one lane with DPP wavefront shifts (GFX9 family):
// wave_shr:1 gives lane l the value of lane l - 1, wave_shl:1 that of lane
// l + 1.  Lanes with no source lane receive 0 (bound control: no old value
// to keep); they are band-edge lanes whose results are never written.
// 64-bit values move as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kWaveShr1 = 0x138;
constexpr int kWaveShl1 = 0x130;

// A value that is the same in every lane of the wavefront (derived from the
// wavefront's index), moved to a scalar register.  Branches on it then stay
// scalar: without this the compiler treats the row parity of a half-sweep as
// per-lane and runs both colours' code under exec masks.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <typename T>
__device__ __forceinline__ T from_left(T v) {  // value of lane - 1
  return dpp_move<kWaveShr1>(v);
}
template <typename T>
__device__ __forceinline__ T from_right(T v) {  // value of lane + 1
  return dpp_move<kWaveShl1>(v);
}

// Two adjacent elements of a row, moved by one 8-byte (FP32) or 16-byte
// (FP64) access.  Only element alignment is assumed: rows of an odd pitch
// start at odd elements.
template <typename T>
struct PairOf;
template <>
struct PairOf<float> {
  typedef float type __attribute__((ext_vector_type(2), aligned(4)));
};
template <>
struct PairOf<double> {
  typedef double type __attribute__((ext_vector_type(2), aligned(8)));
};

// Column data of one lane.  Loads read the stored pair (pc, pc + 1): the
// lane's columns x0, x0 + 1 where both exist (always on a periodic grid:
// x0 and n - 1 are even, so x0 + 1 never wraps apart from x0).  On a
// Dirichlet grid the lane holding the last column n - 1 reads the pair
// ending there and takes it from the second element (sw); lanes outside the
// grid read columns 0 and 1, values that only feed results that are never
// written.
template <int BC>
struct Cols {
  int pc;            // first stored column of the pair that is loaded
  bool sw;           // the lane's column x0 is the pair's second element
  bool unk0, unk1;   // column holds unknowns
  __device__ Cols(int x0, int n) {
    if constexpr (BC == kPeriodic) {
      const int N = n - 1;
      pc = x0 % N;
      if (pc < 0) pc += N;
      sw = false;
      unk0 = unk1 = true;
    } else {
      pc = (x0 >= 0 && x0 <= n - 2) ? x0 : (x0 == n - 1 ? n - 2 : 0);
      sw = x0 == n - 1;
      unk0 = x0 >= 1 && x0 <= n - 2;
      unk1 = x0 + 1 >= 1 && x0 + 1 <= n - 2;
    }
  }
};

// Interior forms of a pass (template argument IN): 0 general; 1 every row
// index the wavefront item forms lies inside the grid (no row clamps or
// wraps, every row holds unknowns); 2 the same for its columns as well, so
// that the column masks, pair selection and coefficient-column extension
// are compile-time constants and drop out of the code.
template <int BC, int IN>
__device__ __forceinline__ Cols<BC> make_cols(int x0, int n) {
  Cols<BC> c(x0, n);
  if constexpr (IN == 2) {
    c.pc = x0;
    c.sw = false;
    c.unk0 = c.unk1 = true;
  }
  return c;
}

// Columns xw .. xw + 127 of a band all hold unknowns (periodic: none is the
// seam copy), so the band may run with IN = 2.
template <int BC>
__device__ __forceinline__ bool band_inside(int xw, int n) {
  return (BC == kPeriodic ? xw >= 0 : xw >= 1) && xw + 127 <= n - 2;
}

template <typename T>
__device__ __forceinline__ void load_pair(T (&dst)[2], const T* __restrict__ row, int pc,
                                          bool sw) {
  const typename PairOf<T>::type v = *reinterpret_cast<const typename PairOf<T>::type*>(row + pc);
  dst[0] = sw ? v.y : v.x;
  dst[1] = v.y;
}

// Store a and b at p[0], p[1] where w0, w1 hold: one pair store for the
// lanes that write both.
template <typename T>
__device__ __forceinline__ void store_pair(T* p, bool w0, bool w1, T a, T b) {
  if (w0 && w1) {
    typename PairOf<T>::type v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<typename PairOf<T>::type*>(p) = v;
  } else {
    if (w0) p[0] = a;
    if (w1) p[1] = b;
  }
}

template <int BC>
__device__ __forceinline__ int row_index(int t, int n, bool* in) {
  if constexpr (BC == kPeriodic) {
    const int N = n - 1;
    *in = true;
    return t < 0 ? t + N : (t >= N ? t - N : t);
  } else {
    *in = t >= 0 && t < n;
    return *in ? t : 0;
  }
}

template <int BC>
__device__ __forceinline__ bool row_unknown(int t, int n) {
  return BC == kPeriodic || (t >= 1 && t <= n - 2);
}

// Loads are unconditional: rows and columns outside a Dirichlet grid are
// clamped to node 0 of that axis (a boundary node), and such values only
// feed results at nodes outside the grid or in the halo, which are never
// written.  Conditional loads would leave the compiler unable to count the
// loads in flight, and every use of a row would then wait for all of them,
// the prefetched rows included.
// IN (interior segment): every row index a pass forms lies inside the grid,
// so rows are neither clamped nor wrapped and every row holds unknowns.
template <typename T, int BC, int IN = 0>
__device__ __forceinline__ void load_row(T (&dst)[2], const T* __restrict__ a, int pa, int t, int n,
                                         const Cols<BC>& col) {
  bool rin;
  const int r = IN ? t : row_index<BC>(t, n, &rin);
  load_pair<T>(dst, a + (size_t)r * pa, col.pc, col.sw);
}

template <typename T>
__device__ __forceinline__ T fused_mul_add(T a, T b, T c) {
  if constexpr (sizeof(T) == sizeof(float))
    return __builtin_fmaf(a, b, c);
  else
    return __builtin_fma(a, b, c);
}

// Red-black half-sweep on one row: the node of the half-sweep's colour among
// the lane's two columns (column x0 + odd, odd = (colour + row) & 1) solves
// its equation with its four neighbours fixed.  Callers pass odd as a value
// the unrolled row loop makes a constant (rows of a segment start at an even
// row), so only one column's code is emitted; updates are selects, not
// branches, which keeps the row ring in place in registers.
template <typename T, int BC, int IN = 0>
__device__ __forceinline__ void sweep_row(const T (&um)[2], T (&u0)[2], const T (&up)[2],
                                          const T (&f0)[2], int row, int odd, int n,
                                          const Cols<BC>& col, T h2) {
  // h2 f + s as one fused multiply-add, written out: left to the compiler,
  // whether it fuses depends on how often the unrolled code reuses h2 f,
  // and the same sweep in two kernels could round differently.
  const bool rok = IN || row_unknown<BC>(row, n);
  if (odd == 0) {
    const T left = from_left(u0[1]);
    const T s = ((um[0] + up[0]) + left) + u0[1];
    const T v = fused_mul_add(h2, f0[0], s) * T(0.25);
    u0[0] = (rok && col.unk0) ? v : u0[0];
  } else {
    const T right = from_right(u0[0]);
    const T s = ((um[1] + up[1]) + u0[0]) + right;
    const T v = fused_mul_add(h2, f0[1], s) * T(0.25);
    u0[1] = (rok && col.unk1) ? v : u0[1];
  }
}

template <typename T, int BC, int IN = 0>
__device__ __forceinline__ void residual_row(const T (&um)[2], const T (&u0)[2], const T (&up)[2],
                                             const T (&f0)[2], T (&r)[2], int row, int n,
                                             const Cols<BC>& col, T inv_h2) {
  const T left = from_left(u0[1]);
  const T right = from_right(u0[0]);
  const T s0 = ((um[0] + up[0]) + left) + u0[1];
  const T s1 = ((um[1] + up[1]) + u0[0]) + right;
  const T r0 = f0[0] - (T(4) * u0[0] - s0) * inv_h2;
  const T r1 = f0[1] - (T(4) * u0[1] - s1) * inv_h2;
  const bool rok = IN || row_unknown<BC>(row, n);
  r[0] = (rok && col.unk0) ? r0 : T(0);
  r[1] = (rok && col.unk1) ? r1 : T(0);
}

// Down pass of one wavefront item: band `band` (128 columns) and row segment
// `seg` (hs rows) of a level with n nodes per side.  lane = threadIdx & 63.
// UIN: 1 reads the initial u from uin, 0 starts from u = 0 (uin unused),
// -1 decides at run time (uin == nullptr: zero).
// RES (mixed path, level 0, from u = 0): the right-hand side is not read
// but made here, a row at a time just before the pipeline needs it, as the
// FP64 residual r = f64 - A u64 of the FP64 iterate (u64, f64: pitch p64,
// pf64), rounded to FP32; the rows and columns the wavefront owns are also
// stored to rout (pitch pro; f is not used), where the up pass reads them.  The same
// arithmetic as residual_wave, so r32 is bitwise what that writes on the
// nodes the up pass reads.  NORM (RES, or UIN = 1): returns the lane's sum
// of r^2 (x) and, with NORM = 2, of f^2 (y) in FP64 over the unknowns it owns
// (periodic: the unique nodes), the residual norm of the iterate the pass
// starts from and the norm it is measured against; zeros otherwise.  With
// UIN = 1 the residual of row t is formed at step t, before that step's
// sweeps, from rows t - 1 .. t + 1 as they were read (the sweeps reach row
// t - 1 only at that step).
template <typename T, int BC, int UIN, bool RES, int IN, bool SB = true, bool REV = false,
          int NORM = 0>
__device__ __forceinline__ double2 down_wave_rows(int n, const T* __restrict__ uin, int pui,
                                          T* __restrict__ uout, int puo, const T* __restrict__ f,
                                          int pf, T* __restrict__ fc, int pfc, int band, int seg,
                                          int hs, T h2, T inv_h2, int lane,
                                          const double* __restrict__ u64, int p64,
                                          const double* __restrict__ f64, int pf64,
                                          double inv_h2d, T* __restrict__ rout, int pro) {
  static_assert(!RES || (UIN == 0 && sizeof(T) == sizeof(float)), "RES: FP32 cycle from u = 0");
  static_assert(!REV || IN >= 1, "a reversed segment lies inside the grid");
  static_assert(!NORM || RES || UIN == 1, "the norm is of the iterate the pass reads");
  const int xw = band * kDownOwned - kDownHalo;
  const int x0 = xw + 2 * lane;
  // REV: the segment's rows [seg hs, seg hs + hs) are walked upwards, as
  // rows v of a mirrored grid, row v = C - (grid row) with C = 2 seg hs + hs
  // even (so row parities, and with them the colours and the even rows the
  // restriction reads, are the same in both).  The mirrored segment then
  // starts at the odd row seg hs + 1.
  const int ys = REV ? seg * hs + 1 : seg * hs;
  const int C = 2 * seg * hs + hs;
  auto ra = [&](int v) { return REV ? C - v : v; };  // grid row of pipeline row v
  const Cols<BC> col = make_cols<BC, IN>(x0, n);
  const int N = n - 1, nc = (n - 1) / 2 + 1;
  const bool lane_owns = lane >= kDownHalo / 2 && lane < 64 - kDownHalo / 2;
  const bool wr0 = lane_owns && (BC == kPeriodic ? x0 < N : col.unk0);
  const bool wr1 = lane_owns && (BC == kPeriodic ? x0 + 1 < N : col.unk1);
  const int J = x0 >> 1;
  const bool wrc = lane_owns && (BC == kPeriodic ? J < nc - 1 : (J >= 1 && J <= nc - 2));
  const int row_end = BC == kPeriodic ? N : n;  // rows [0, row_end) are owned by some segment

  // Rows live in a ring of register slots; row t0 + s is in slot s & RM and
  // is loaded kAheadDown steps before the step that first uses it.  RES
  // loads nothing ahead into these rings (rows t - 6 .. t are live), so 8
  // slots hold them.
  constexpr int RM = RES ? 7 : 15;
  T U[RM + 1][2], F[RM + 1][2], R[4][2];
#pragma unroll
  for (int k = 0; k <= RM; ++k) U[k][0] = U[k][1] = F[k][0] = F[k][1] = T(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) R[k][0] = R[k][1] = T(0);

  const int t0 = ys - 6;  // even (hs is even); odd when REV
  constexpr int P = REV ? 1 : 0;  // parity of t - k
  // The restriction of even row i runs at step i + 6; mirrored, the last
  // even row the segment owns is ys + hs - 1, one step later than forward.
  const int steps = hs + 11 + P;
  const bool read_u = UIN == 1 || (UIN == -1 && uin != nullptr);
  // RES: u64 row t0 - 1 + q in RU[q & 7], f64 row t0 + q in RF[q & 3],
  // loaded kAheadR + 1 and kAheadR rows before their residual row.
  constexpr int kAheadR = 3;
  double RU[RES ? 8 : 1][2], RF[RES ? 4 : 1][2];
  const int tl = t0 + steps - 1;  // last row a step uses
  const bool rw0 = lane_owns && x0 < n, rw1 = lane_owns && x0 + 1 < n;
  double acc = 0.0, accf = 0.0;
  if constexpr (RES) {
#pragma unroll
    for (int q = 0; q < kAheadR + 2; ++q) {
      const int r = t0 - 1 + q;
      load_row<double, BC, IN>(RU[q], u64, p64, ra(r < tl + 1 ? r : tl + 1), n, col);
    }
#pragma unroll
    for (int q = 0; q < kAheadR; ++q) {
      const int r = t0 + q;
      load_row<double, BC, IN>(RF[q], f64, pf64, ra(r < tl ? r : tl), n, col);
    }
  } else {
#pragma unroll
    for (int k = 0; k < kAheadDown; ++k) {
      if (UIN == 1 || (UIN == -1 && read_u)) load_row<T, BC, IN>(U[k], uin, pui, ra(t0 + k), n, col);
      load_row<T, BC, IN>(F[k], f, pf, ra(t0 + k), n, col);
    }
  }
  for (int sb = 0; sb < steps; sb += 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int s = sb + k;
      // (NORM: the sum of r^2 lives past the loop, and the early exit then
      // keeps the compiler from unrolling it; skipping the remaining steps
      // instead does not.)
      if (s >= steps) {
        if constexpr (NORM) continue;
        else break;
      }
      const int t = t0 + s;
      // Rows kAheadDown ahead; past the last row a step uses, that row again
      // (a cache hit instead of a row of HBM traffic; never used).
      if constexpr (RES) {
        // Right-hand side row t (first used at the next step) from u64 rows
        // t - 1 .. t + 1 and f64 row t.
        const int tu = t + kAheadR + 1 < tl + 1 ? t + kAheadR + 1 : tl + 1;
        const int tf = t + kAheadR < tl ? t + kAheadR : tl;
        load_row<double, BC, IN>(RU[(k + kAheadR + 2) & 7], u64, p64, ra(tu), n, col);
        load_row<double, BC, IN>(RF[(k + kAheadR) & 3], f64, pf64, ra(tf), n, col);
        const double(&um)[2] = RU[k & 7];
        const double(&u0)[2] = RU[(k + 1) & 7];
        const double(&up)[2] = RU[(k + 2) & 7];
        const double(&ff)[2] = RF[k & 3];
        const double left = from_left(u0[1]);
        const double right = from_right(u0[0]);
        const double s0 = ((um[0] + up[0]) + left) + u0[1];
        const double s1 = ((um[1] + up[1]) + u0[0]) + right;
        double r0 = ff[0] - (4.0 * u0[0] - s0) * inv_h2d;
        double r1 = ff[1] - (4.0 * u0[1] - s1) * inv_h2d;
        if constexpr (BC == kDirichlet) {
          const bool rok = IN || row_unknown<BC>(t, n);
          r0 = (rok && col.unk0) ? r0 : 0.0;
          r1 = (rok && col.unk1) ? r1 : 0.0;
        }
        F[k & RM][0] = (T)r0;
        F[k & RM][1] = (T)r1;
        const bool own_row = t >= ys && t < ys + hs && (IN || t < row_end);
        if (own_row) store_pair<T>(rout + (size_t)ra(t) * pro + x0, rw0, rw1, (T)r0, (T)r1);
        if constexpr (NORM) {
          // r is 0 on the Dirichlet boundary rows already; f is not.
          const bool fr = own_row && (BC == kPeriodic || IN || row_unknown<BC>(t, n));
          const double q0 = (own_row && wr0) ? r0 : 0.0, q1 = (own_row && wr1) ? r1 : 0.0;
          const double g0 = (fr && wr0) ? ff[0] : 0.0, g1 = (fr && wr1) ? ff[1] : 0.0;
          acc += q0 * q0;
          acc += q1 * q1;
          if constexpr (NORM >= 2) {
            accf += g0 * g0;
            accf += g1 * g1;
          }
        }
        U[k & RM][0] = U[k & RM][1] = T(0);  // row t starts from 0
      } else {
        if constexpr (NORM) {
          static_assert(kAheadDown >= 2, "row t + 1 is in the ring at step t");
          T rr[2];
          residual_row<T, BC, IN>(U[(k + 15) & RM], U[k & RM], U[(k + 1) & RM], F[k & RM], rr, t,
                                  n, col, inv_h2);
          const bool own_row = t >= ys && t < ys + hs && (IN || t < row_end);
          const bool fr = own_row && (BC == kPeriodic || IN || row_unknown<BC>(t, n));
          const double q0 = (own_row && wr0) ? (double)rr[0] : 0.0;
          const double q1 = (own_row && wr1) ? (double)rr[1] : 0.0;
          const double g0 = (fr && wr0) ? (double)F[k & RM][0] : 0.0;
          const double g1 = (fr && wr1) ? (double)F[k & RM][1] : 0.0;
          acc += q0 * q0;
          acc += q1 * q1;
          if constexpr (NORM >= 2) {
            accf += g0 * g0;
            accf += g1 * g1;
          }
        }
        const int ta = t + kAheadDown < t0 + steps - 1 ? t + kAheadDown : t0 + steps - 1;
        T(&nu)[2] = U[(k + kAheadDown) & RM];
        if (UIN == 1 || (UIN == -1 && read_u)) load_row<T, BC, IN>(nu, uin, pui, ra(ta), n, col);
        else nu[0] = nu[1] = T(0);
        load_row<T, BC, IN>(F[(k + kAheadDown) & RM], f, pf, ra(ta), n, col);
      }
      // red (sweep 1) on t-1, black on t-2, red (sweep 2) on t-3, black on
      // t-4; t has the parity of k + P (t0 - P and sb are even).
      sweep_row<T, BC, IN>(U[(k + 14) & RM], U[(k + 15) & RM], U[k & RM], F[(k + 15) & RM], t - 1,
                       (k + 1 + P) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(k + 13) & RM], U[(k + 14) & RM], U[(k + 15) & RM], F[(k + 14) & RM],
                       t - 2, (k + 1 + P) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(k + 12) & RM], U[(k + 13) & RM], U[(k + 14) & RM], F[(k + 13) & RM],
                       t - 3, (k + 1 + P) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(k + 11) & RM], U[(k + 12) & RM], U[(k + 13) & RM], F[(k + 12) & RM],
                       t - 4, (k + 1 + P) & 1, n, col, h2);
      const int tu = t - 4;
      if (SB && tu >= ys && tu < ys + hs && (IN || tu < row_end)) {
        T* p = uout + (size_t)ra(tu) * puo;
        store_pair<T>(p + x0, wr0, wr1, U[(k + 12) & RM][0], U[(k + 12) & RM][1]);
      }
      residual_row<T, BC, IN>(U[(k + 10) & RM], U[(k + 11) & RM], U[(k + 12) & RM], F[(k + 11) & RM],
                          R[(k + 3) & 3], t - 5, n, col, inv_h2);
      const int i = t - 6;
      if ((i & 1) == 0 && i >= ys && i < ys + hs) {
        const int I = ra(i) >> 1;
        const bool rowc = IN || (BC == kPeriodic ? I < nc - 1 : (I >= 1 && I <= nc - 2));
        const T(&rm)[2] = R[(k + 1) & 3];
        const T(&r0)[2] = R[(k + 2) & 3];
        const T(&rp)[2] = R[(k + 3) & 3];
        const T am = from_left(rm[1]), a0 = from_left(r0[1]), ap = from_left(rp[1]);
        // Sums symmetric in rm and rp (pairs added first), so that a segment
        // walked upwards rounds as one walked downwards.
        const T edges = ((rm[0] + rp[0]) + a0) + r0[1];
        const T corners = (am + rm[1]) + (ap + rp[1]);
        const T v = ((T(4) * r0[0] + T(2) * edges) + corners) * T(0.0625);
        if (rowc && wrc) fc[(size_t)I * pfc + J] = v;
      }
    }
  }
  return make_double2(acc, accf);
}

// SB = false (RES only): the pre-smoothed iterate is not stored (the up pass
// makes it again from the stored right-hand side, up_pre_wave).  NORM: see
// down_wave_rows (the lane's parts of ||f - A u||^2 and ||f||^2).
template <typename T, int BC, int UIN = -1, bool RES = false, bool SB = true, int NORM = 0>
__device__ __forceinline__ double2 down_wave(int n, const T* __restrict__ uin, int pui,
                                          T* __restrict__ uout, int puo, const T* __restrict__ f,
                                          int pf, T* __restrict__ fc, int pfc, int band, int seg,
                                          int hs, T h2, T inv_h2, int lane,
                                          const double* __restrict__ u64 = nullptr, int p64 = 0,
                                          const double* __restrict__ f64 = nullptr, int pf64 = 0,
                                          double inv_h2d = 0.0, T* __restrict__ rout = nullptr,
                                          int pro = 0) {
  n = wave_uniform(n), band = wave_uniform(band), seg = wave_uniform(seg), hs = wave_uniform(hs);
  // Rows the segment touches: t0 - 1 .. t0 + hs + 11 (t0 = seg * hs - 6).
  // Inside rows 1 .. n - 2 (periodic: 0 .. n - 2) the interior form runs.
  const int lo = seg * hs - 7, hi = seg * hs + hs + 5;
  const bool in = BC == kPeriodic ? (lo >= 0 && hi <= n - 2) : (lo >= 1 && hi <= n - 2);
  static_assert(SB || RES, "only the residual-making down pass may skip its iterate");
  // The residual-making form stays at IN = 1 across columns: its IN = 2 code
  // (fewer instructions, loads kept in flight differently) measured 78 -> 87
  // us at 4097^2.
  // Odd segments inside the grid walk their rows upwards (REV), so that
  // neighbouring segments read the rows around their shared edge at the
  // same time (both at the start, or both at the end of their walk) and one
  // of the two reads finds them in cache.  Reversed, a segment touches rows
  // seg hs - 7 .. seg hs + hs + 6.
  const int lo_r = seg * hs - 7, hi_r = seg * hs + hs + 6;
  const bool in_r = BC == kPeriodic ? (lo_r >= 0 && hi_r <= n - 2) : (lo_r >= 1 && hi_r <= n - 2);
  if (RES && (seg & 1) && in_r)
    return down_wave_rows<T, BC, UIN, RES, 1, SB, true, NORM>(
        n, uin, pui, uout, puo, f, pf, fc, pfc, band, seg, hs, h2, inv_h2, lane, u64, p64, f64,
        pf64, inv_h2d, rout, pro);
  else if (!RES && in && band_inside<BC>(band * kDownOwned - kDownHalo, n))
    return down_wave_rows<T, BC, UIN, RES, 2, SB, false, NORM>(
        n, uin, pui, uout, puo, f, pf, fc, pfc, band, seg, hs, h2, inv_h2, lane, u64, p64, f64,
        pf64, inv_h2d, rout, pro);
  else if (in)
    return down_wave_rows<T, BC, UIN, RES, 1, SB, false, NORM>(
        n, uin, pui, uout, puo, f, pf, fc, pfc, band, seg, hs, h2, inv_h2, lane, u64, p64, f64,
        pf64, inv_h2d, rout, pro);
  else
    return down_wave_rows<T, BC, UIN, RES, 0, SB, false, NORM>(
        n, uin, pui, uout, puo, f, pf, fc, pfc, band, seg, hs, h2, inv_h2, lane, u64, p64, f64,
        pf64, inv_h2d, rout, pro);
}

// Spline along x at the lane's two columns from coarse row values held one
// coarse column per lane (lane L holds coefficient column x0/2).
// The weighted sums of the spline are written as explicit fused multiply-
// adds (w0 a, then + w1 b, + w2 c, ... each fused), so that every kernel
// evaluating them rounds the same way.
template <typename T>
__device__ __forceinline__ T wsum3(T w0, T a, T w1, T b, T w2, T c) {
  return fused_mul_add(w2, c, fused_mul_add(w1, b, w0 * a));
}
template <typename T>
__device__ __forceinline__ T wsum4(T w0, T a, T w1, T b, T w2, T c, T w3, T d) {
  return fused_mul_add(w3, d, fused_mul_add(w2, c, fused_mul_add(w1, b, w0 * a)));
}

template <typename T>
__device__ __forceinline__ void spline_x(T cj, T (&out)[2]) {
  const T cl = from_left(cj), cr = from_right(cj), cr2 = from_right(cr);
  out[0] = wsum3(T(1.0 / 6.0), cl, T(4.0 / 6.0), cj, T(1.0 / 6.0), cr);
  out[1] = wsum4(T(1.0 / 48.0), cl, T(23.0 / 48.0), cj, T(23.0 / 48.0), cr, T(1.0 / 48.0), cr2);
}

template <typename T, int BC, int IN = 0>
__device__ __forceinline__ T load_coef(const T* __restrict__ c, int pc, int I, int J, int nc) {
  bool ni = false, nj = false;
  const int ii = IN ? I : ext_node_any<BC>(I, nc, &ni);
  const int jj = IN == 2 ? J : ext_node_any<BC>(J, nc, &nj);
  const T v = c[(size_t)ii * pc + jj];
  return (ni != nj) ? -v : v;
}

// Up pass of one wavefront item (see down_wave).  With ADD, the finished
// rows are added to u64 (the FP64 iterate of the mixed path, pitch p64) over
// the unknowns -- the refinement update -- instead of being written to uout.
template <typename T, int BC, bool ADD, int IN>
__device__ __forceinline__ void up_wave_rows(int n, const T* __restrict__ uin, int pui,
                                             T* __restrict__ uout, int puo,
                                             const T* __restrict__ f, int pf,
                                             const T* __restrict__ c, int pc, int band, int seg,
                                             int hs, T h2, int lane, double* __restrict__ u64,
                                             int p64) {
  const int xw = band * kUpOwned - kUpHalo;
  const int x0 = xw + 2 * lane;
  const int ys = seg * hs;
  const Cols<BC> col = make_cols<BC, IN>(x0, n);
  const int N = n - 1, nc = (n - 1) / 2 + 1;
  const bool lane_owns = lane >= kUpHalo / 2 && lane < kUpHalo / 2 + kUpOwned / 2;
  const bool wr0 = lane_owns && (BC == kPeriodic ? x0 < N : col.unk0);
  const bool wr1 = lane_owns && (BC == kPeriodic ? x0 + 1 < N : col.unk1);
  const int Jc = x0 >> 1;
  const int row_end = BC == kPeriodic ? N : n;

  T U[16][2], F[16][2], CX[4][2], CR[8];
#pragma unroll
  for (int k = 0; k < 16; ++k) U[k][0] = U[k][1] = F[k][0] = F[k][1] = T(0);

  const int t0 = ys - 4;            // even
  const int cbase = (t0 >> 1) - 1;  // coarse row q = 0 of the ring
  // Raw coefficients (lane L: column x0/2) of coarse row cbase + q live in
  // CR[q & 7], loaded 4 coarse rows ahead; CX[q & 3] holds their spline
  // along x at the lane's two columns.
#pragma unroll
  for (int q = 0; q < 7; ++q) CR[q] = load_coef<T, BC, IN>(c, pc, cbase + q, Jc, nc);
  CR[7] = T(0);
#pragma unroll
  for (int q = 0; q < 3; ++q) spline_x<T>(CR[q], CX[q]);
  CX[3][0] = CX[3][1] = T(0);
  const int steps = hs + 8;
  // With u64: its row written at step s (row t0 + s - 4) is read kAheadUp
  // steps earlier into UR[s & 7].
  double UR[ADD ? 8 : 1][2];
  // Only rows and columns the segment stores are read: other rows repeat its
  // first or last row, and the halo lanes read the first owned lane's pair
  // (cache hits; never used).
  const int ylast = (ys + hs < row_end ? ys + hs : row_end) - 1;
  const Cols<BC> col64 = make_cols<BC, IN>(lane_owns ? x0 : xw + kUpHalo, n);
  auto load_u64 = [&](int slot, int row) {
    if (ADD) {
      const int rr = row < ys ? ys : (row > ylast ? ylast : row);
      const double* q = u64 + (size_t)rr * p64;
      load_pair<double>(UR[slot], q, col64.pc, col64.sw);
    }
  };
#pragma unroll
  for (int k = 0; k < kAheadUp; ++k) {
    load_row<T, BC, IN>(U[k], uin, pui, t0 + k, n, col);
    load_row<T, BC, IN>(F[k], f, pf, t0 + k, n, col);
    load_u64(k & 7, t0 - 4 + k);
  }
  for (int sb = 0; sb < steps; sb += 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int s = sb + k;
      if (s >= steps) break;
      const int t = t0 + s;
      {  // rows kAheadUp ahead; past the last row a step uses, that row again
        const int ta = t + kAheadUp < t0 + steps - 1 ? t + kAheadUp : t0 + steps - 1;
        load_row<T, BC, IN>(U[(k + kAheadUp) & 15], uin, pui, ta, n, col);
        load_row<T, BC, IN>(F[(k + kAheadUp) & 15], f, pf, ta, n, col);
        load_u64((k + kAheadUp) & 7, t - 4 + kAheadUp);
      }
      // coarse row q = (s - 1)/2 + 3 is needed from the first odd step on
      if (k & 1) {
        const int qk = ((k - 1) >> 1) + 3;  // q mod 8
        spline_x<T>(CR[qk & 7], CX[qk & 3]);
        CR[(qk + 4) & 7] = load_coef<T, BC, IN>(c, pc, cbase + ((s - 1) >> 1) + 7, Jc, nc);
      }
      {
        // u += P e_c on row t: coincident rows (1, 4, 1)/6 on coarse rows
        // base..base+2, midpoints (1, 23, 23, 1)/48 on base..base+3.
        const int qb = (k >> 1);  // coarse row (t >> 1) - 1 relative to cbase, mod 8
        T v0, v1;
        const T(&a)[2] = CX[qb & 3];
        const T(&b)[2] = CX[(qb + 1) & 3];
        const T(&d)[2] = CX[(qb + 2) & 3];
        if ((k & 1) == 0) {
          v0 = wsum3(T(1.0 / 6.0), a[0], T(4.0 / 6.0), b[0], T(1.0 / 6.0), d[0]);
          v1 = wsum3(T(1.0 / 6.0), a[1], T(4.0 / 6.0), b[1], T(1.0 / 6.0), d[1]);
        } else {
          const T(&e)[2] = CX[(qb + 3) & 3];
          v0 = wsum4(T(1.0 / 48.0), a[0], T(23.0 / 48.0), b[0], T(23.0 / 48.0), d[0],
                     T(1.0 / 48.0), e[0]);
          v1 = wsum4(T(1.0 / 48.0), a[1], T(23.0 / 48.0), b[1], T(23.0 / 48.0), d[1],
                     T(1.0 / 48.0), e[1]);
        }
        const bool rok = IN || row_unknown<BC>(t, n);
        U[k][0] = (rok && col.unk0) ? U[k][0] + v0 : U[k][0];
        U[k][1] = (rok && col.unk1) ? U[k][1] + v1 : U[k][1];
      }
      // t has the parity of k (t0 and sb are even)
      sweep_row<T, BC, IN>(U[(k + 14) & 15], U[(k + 15) & 15], U[k], F[(k + 15) & 15], t - 1,
                       (k + 1) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(k + 13) & 15], U[(k + 14) & 15], U[(k + 15) & 15], F[(k + 14) & 15],
                       t - 2, (k + 1) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(k + 12) & 15], U[(k + 13) & 15], U[(k + 14) & 15], F[(k + 13) & 15],
                       t - 3, (k + 1) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(k + 11) & 15], U[(k + 12) & 15], U[(k + 13) & 15], F[(k + 12) & 15],
                       t - 4, (k + 1) & 1, n, col, h2);
      const int tu = t - 4;
      if (tu >= ys && tu < ys + hs && (IN || tu < row_end)) {
        if (ADD) {
          double* q = u64 + (size_t)tu * p64;
          const bool r = IN || row_unknown<BC>(tu, n);
          store_pair<double>(q + x0, wr0 && col.unk0 && r, wr1 && col.unk1 && r,
                             UR[k & 7][0] + (double)U[(k + 12) & 15][0],
                             UR[k & 7][1] + (double)U[(k + 12) & 15][1]);
        } else {
          T* p = uout + (size_t)tu * puo;
          store_pair<T>(p + x0, wr0, wr1, U[(k + 12) & 15][0], U[(k + 12) & 15][1]);
        }
      }
    }
  }
}

template <typename T, int BC, bool ADD = false>
__device__ __forceinline__ void up_wave(int n, const T* __restrict__ uin, int pui,
                                        T* __restrict__ uout, int puo, const T* __restrict__ f,
                                        int pf, const T* __restrict__ c, int pc, int band, int seg,
                                        int hs, T h2, int lane, double* __restrict__ u64 = nullptr,
                                        int p64 = 0) {
  n = wave_uniform(n), band = wave_uniform(band), seg = wave_uniform(seg), hs = wave_uniform(hs);
  // Fine rows touched: seg * hs - 4 .. seg * hs + hs + 3; coarse rows up to
  // (seg * hs + hs) / 2 + 7.  Inside the grid (and coarse rows from 0) the
  // interior form runs.
  const int lo = seg * hs - 4, hi = seg * hs + hs + 15;
  const bool in = lo >= 2 && hi <= n - 1;
  if (in && band_inside<BC>(band * kUpOwned - kUpHalo, n))
    up_wave_rows<T, BC, ADD, 2>(n, uin, pui, uout, puo, f, pf, c, pc, band, seg, hs, h2, lane, u64,
                                p64);
  else if (in)
    up_wave_rows<T, BC, ADD, 1>(n, uin, pui, uout, puo, f, pf, c, pc, band, seg, hs, h2, lane, u64,
                                p64);
  else
    up_wave_rows<T, BC, ADD, 0>(n, uin, pui, uout, puo, f, pf, c, pc, band, seg, hs, h2, lane, u64,
                                p64);
}

// Up pass of the mixed path's level 0 when its down pass started from e = 0
// and did not store its pre-smoothed iterate: the iterate is made again here
// from the stored right-hand side f (the same two sweeps from zero, so
// bitwise the same values), and neither pass moves it through memory.  At
// the step that loads row t: red sweep on t-1, black t-2, red t-3, black
// t-4 (the pre-smoothed row t-4); then the up pass proper on row tv = t-5:
// u += P e_c on tv, red tv-1, black tv-2, red tv-3, black tv-4, added into
// the FP64 iterate u64.  The lag of five keeps the correction of a row after
// the last pre-smoothing sweep that reads it (the black sweep of row tv + 1,
// made at the same step just before).  Rows above the segment start from
// zero with f = 0 there; that error reaches at most 6 rows below the first
// loaded one, which is 8 above the segment.  A band owns columns
// [xw + 8, xw + 120): the edge lanes' missing neighbours spoil one column
// per half-sweep (eight) and the spline's right support two lanes.
constexpr int kUpPreLeft = 8;
constexpr int kUpPreOwned = 112;

template <int BC, int IN>
__device__ __forceinline__ void up_pre_wave_rows(int n, const float* __restrict__ f, int pf,
                                                 const float* __restrict__ c, int pc, int band,
                                                 int seg, int hs, float h2, int lane,
                                                 double* __restrict__ u64, int p64) {
  using T = float;
  const int xw = band * kUpPreOwned - kUpPreLeft;
  const int x0 = xw + 2 * lane;
  const int ys = seg * hs;
  const Cols<BC> col = make_cols<BC, IN>(x0, n);
  const int N = n - 1, nc = (n - 1) / 2 + 1;
  const bool lane_owns = lane >= kUpPreLeft / 2 && lane < kUpPreLeft / 2 + kUpPreOwned / 2;
  const bool wr0 = lane_owns && (BC == kPeriodic ? x0 < N : col.unk0);
  const bool wr1 = lane_owns && (BC == kPeriodic ? x0 + 1 < N : col.unk1);
  const int Jc = x0 >> 1;
  const int row_end = BC == kPeriodic ? N : n;

  T U[16][2], F[16][2], CX[4][2], CR[8];
#pragma unroll
  for (int k = 0; k < 16; ++k) U[k][0] = U[k][1] = F[k][0] = F[k][1] = T(0);

  // Row r sits in ring slot (r - t0) & 15.  The correction starts at row
  // tv0 = ys - 4 (as in up_wave_rows), at step 9; its own step index
  // sv = s - 9 drives the coarse-row ring exactly as there.
  const int t0 = ys - 8;             // first row of the pre-smoothing stage (even)
  const int tv0 = ys - 4;
  const int cbase = (tv0 >> 1) - 1;  // coarse row q = 0 of the ring
#pragma unroll
  for (int q = 0; q < 7; ++q) CR[q] = load_coef<T, BC, IN>(c, pc, cbase + q, Jc, nc);
  CR[7] = T(0);
#pragma unroll
  for (int q = 0; q < 3; ++q) spline_x<T>(CR[q], CX[q]);
  CX[3][0] = CX[3][1] = T(0);
  const int steps = hs + 17;
  const int tlast = t0 + steps - 1;
  // u64 row written at step s (row t0 + s - 9) is read kAheadU64 steps
  // earlier into UR[s & 3]; only rows and columns the segment stores.
  constexpr int kAheadU64 = 3;
  double UR[4][2];
  const int ylast = (ys + hs < row_end ? ys + hs : row_end) - 1;
  const Cols<BC> col64 = make_cols<BC, IN>(lane_owns ? x0 : xw + kUpPreLeft, n);
  auto load_u64 = [&](int slot, int row) {
    const int rr = row < ys ? ys : (row > ylast ? ylast : row);
    load_pair<double>(UR[slot], u64 + (size_t)rr * p64, col64.pc, col64.sw);
  };
#pragma unroll
  for (int k = 0; k < kAheadUp; ++k) load_row<T, BC, IN>(F[k], f, pf, t0 + k, n, col);
#pragma unroll
  for (int k = 0; k < kAheadU64; ++k) load_u64(k, t0 - 9 + k);
  for (int sb = 0; sb < steps; sb += 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int s = sb + k;
      if (s >= steps) break;
      const int t = t0 + s;
      {  // rows kAheadUp ahead; past the last row a step uses, that row again
        const int ta = t + kAheadUp < tlast ? t + kAheadUp : tlast;
        load_row<T, BC, IN>(F[(k + kAheadUp) & 15], f, pf, ta, n, col);
        load_u64((k + kAheadU64) & 3, t - 9 + kAheadU64);
      }
      U[k][0] = U[k][1] = T(0);  // row t starts from zero
      // pre-smoothing from zero (t has the parity of k: t0 and sb are even)
      sweep_row<T, BC, IN>(U[(k + 14) & 15], U[(k + 15) & 15], U[k], F[(k + 15) & 15], t - 1,
                           (k + 1) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(k + 13) & 15], U[(k + 14) & 15], U[(k + 15) & 15],
                           F[(k + 14) & 15], t - 2, (k + 1) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(k + 12) & 15], U[(k + 13) & 15], U[(k + 14) & 15],
                           F[(k + 13) & 15], t - 3, (k + 1) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(k + 11) & 15], U[(k + 12) & 15], U[(k + 13) & 15],
                           F[(k + 12) & 15], t - 4, (k + 1) & 1, n, col, h2);
      if (s < 9) continue;
      // The up pass on row tv = t - 5: ring slot kv of row tv; kq = sv mod 16
      // for the coarse ring (sv = s - 9, t has the parity of k, so tv and sv
      // have the parity of k + 1).
      const int kv = (k + 11) & 15, kq = (k + 7) & 15;
      const int sv = s - 9, tv = t - 5;
      if (kq & 1) {
        const int qk = ((kq - 1) >> 1) + 3;
        spline_x<T>(CR[qk & 7], CX[qk & 3]);
        CR[(qk + 4) & 7] = load_coef<T, BC, IN>(c, pc, cbase + ((sv - 1) >> 1) + 7, Jc, nc);
      }
      {
        const int qb = (kq >> 1);
        T v0, v1;
        const T(&a)[2] = CX[qb & 3];
        const T(&b)[2] = CX[(qb + 1) & 3];
        const T(&d)[2] = CX[(qb + 2) & 3];
        if ((kq & 1) == 0) {
          v0 = wsum3(T(1.0 / 6.0), a[0], T(4.0 / 6.0), b[0], T(1.0 / 6.0), d[0]);
          v1 = wsum3(T(1.0 / 6.0), a[1], T(4.0 / 6.0), b[1], T(1.0 / 6.0), d[1]);
        } else {
          const T(&e)[2] = CX[(qb + 3) & 3];
          v0 = wsum4(T(1.0 / 48.0), a[0], T(23.0 / 48.0), b[0], T(23.0 / 48.0), d[0],
                     T(1.0 / 48.0), e[0]);
          v1 = wsum4(T(1.0 / 48.0), a[1], T(23.0 / 48.0), b[1], T(23.0 / 48.0), d[1],
                     T(1.0 / 48.0), e[1]);
        }
        const bool rok = IN || row_unknown<BC>(tv, n);
        U[kv][0] = (rok && col.unk0) ? U[kv][0] + v0 : U[kv][0];
        U[kv][1] = (rok && col.unk1) ? U[kv][1] + v1 : U[kv][1];
      }
      sweep_row<T, BC, IN>(U[(kv + 14) & 15], U[(kv + 15) & 15], U[kv], F[(kv + 15) & 15], tv - 1,
                           (kv + 1) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(kv + 13) & 15], U[(kv + 14) & 15], U[(kv + 15) & 15],
                           F[(kv + 14) & 15], tv - 2, (kv + 1) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(kv + 12) & 15], U[(kv + 13) & 15], U[(kv + 14) & 15],
                           F[(kv + 13) & 15], tv - 3, (kv + 1) & 1, n, col, h2);
      sweep_row<T, BC, IN>(U[(kv + 11) & 15], U[(kv + 12) & 15], U[(kv + 13) & 15],
                           F[(kv + 12) & 15], tv - 4, (kv + 1) & 1, n, col, h2);
      const int tu = tv - 4;
      if (tu >= ys && tu < ys + hs && (IN || tu < row_end)) {
        double* q = u64 + (size_t)tu * p64;
        const bool r = IN || row_unknown<BC>(tu, n);
        store_pair<double>(q + x0, wr0 && col.unk0 && r, wr1 && col.unk1 && r,
                           UR[k & 3][0] + (double)U[(kv + 12) & 15][0],
                           UR[k & 3][1] + (double)U[(kv + 12) & 15][1]);
      }
    }
  }
}

template <int BC>
__device__ __forceinline__ void up_pre_wave(int n, const float* __restrict__ f, int pf,
                                            const float* __restrict__ c, int pc, int band, int seg,
                                            int hs, float h2, int lane, double* __restrict__ u64,
                                            int p64) {
  n = wave_uniform(n), band = wave_uniform(band), seg = wave_uniform(seg), hs = wave_uniform(hs);
  // Fine rows touched: seg * hs - 10 .. seg * hs + hs + 8; coarse rows up to
  // (seg * hs + hs) / 2 + 7.
  const int lo = seg * hs - 10, hi = seg * hs + hs + 19;
  const bool in = lo >= 2 && hi <= n - 1;
  if (in && band_inside<BC>(band * kUpPreOwned - kUpPreLeft, n))
    up_pre_wave_rows<BC, 2>(n, f, pf, c, pc, band, seg, hs, h2, lane, u64, p64);
  else if (in)
    up_pre_wave_rows<BC, 1>(n, f, pf, c, pc, band, seg, hs, h2, lane, u64, p64);
  else
    up_pre_wave_rows<BC, 0>(n, f, pf, c, pc, band, seg, hs, h2, lane, u64, p64);
}

// Mixed path, level 0: r32 = fl32(f - A u) with f, u and the arithmetic in
// FP64, at every node of rows [ys, ys + hs) (0 on the Dirichlet boundary;
// periodic seam row and column = node 0), for the wavefront of (band, seg):
// lanes 1 .. 62 own the band's kResOwned columns, lanes 0 and 63 only supply
// neighbours.  Rows stream through 8-slot rings, u loaded kAheadRes + 1 rows
// and f kAheadRes rows before use.  Returns the lane's sum of r^2 over the
// unknowns it owns.
constexpr int kResOwned = 124;
constexpr int kAheadRes = 4;
static_assert(kAheadRes <= 5, "u ring holds rows t-1 .. t+1+kAheadRes");

template <int BC>
__device__ __forceinline__ double residual_wave(int n, const double* __restrict__ u, int pu,
                                                const double* __restrict__ f, int pf,
                                                float* __restrict__ r32, int pr, int band, int seg,
                                                int hs, double inv_h2, int lane) {
  n = wave_uniform(n), band = wave_uniform(band), seg = wave_uniform(seg), hs = wave_uniform(hs);
  const int x0 = band * kResOwned - 2 + 2 * lane;
  const Cols<BC> col(x0, n);
  const int N = n - 1;
  const bool owns = lane >= 1 && lane <= 62;
  const bool w0 = owns && x0 < n, w1 = owns && x0 + 1 < n;
  // Unknowns counted in the norm (periodic: the unique nodes).
  const bool k0 = owns && (BC == kPeriodic ? x0 < N : col.unk0);
  const bool k1 = owns && (BC == kPeriodic ? x0 + 1 < N : col.unk1);
  const int ys = seg * hs;
  const int steps = (ys + hs < n ? ys + hs : n) - ys;

  double U[8][2], F[8][2];
#pragma unroll
  for (int k = 0; k < 8; ++k) U[k][0] = U[k][1] = F[k][0] = F[k][1] = 0.0;
  // u row ys - 1 + q in U[q & 7], f row ys + q in F[q & 7].
  // Rows past the last ones the segment uses (u: ys + steps <= n, f: one
  // less) repeat them: cache hits, never used, and a periodic row index
  // wraps at most once.
  const int ulast = ys + steps, flast = ys + steps - 1;
#pragma unroll
  for (int q = 0; q < kAheadRes + 2; ++q) {
    const int r = ys - 1 + q;
    load_row<double, BC>(U[q], u, pu, r < ulast ? r : ulast, n, col);
  }
#pragma unroll
  for (int q = 0; q < kAheadRes; ++q) {
    const int r = ys + q;
    load_row<double, BC>(F[q], f, pf, r < flast ? r : flast, n, col);
  }
  double acc = 0.0;
  for (int sb = 0; sb < steps; sb += 8) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int s = sb + k;
      if (s >= steps) break;
      const int t = ys + s;
      const int tu = t + kAheadRes + 1, tf = t + kAheadRes;
      load_row<double, BC>(U[(k + kAheadRes + 2) & 7], u, pu, tu < ulast ? tu : ulast, n, col);
      load_row<double, BC>(F[(k + kAheadRes) & 7], f, pf, tf < flast ? tf : flast, n, col);
      const double(&um)[2] = U[k & 7];
      const double(&u0)[2] = U[(k + 1) & 7];
      const double(&up)[2] = U[(k + 2) & 7];
      const double(&f0)[2] = F[k & 7];
      const double left = from_left(u0[1]);
      const double right = from_right(u0[0]);
      const double s0 = ((um[0] + up[0]) + left) + u0[1];
      const double s1 = ((um[1] + up[1]) + u0[0]) + right;
      double r0 = f0[0] - (4.0 * u0[0] - s0) * inv_h2;
      double r1 = f0[1] - (4.0 * u0[1] - s1) * inv_h2;
      if constexpr (BC == kDirichlet) {
        const bool rok = row_unknown<BC>(t, n);
        r0 = (rok && col.unk0) ? r0 : 0.0;
        r1 = (rok && col.unk1) ? r1 : 0.0;
      }
      store_pair<float>(r32 + (size_t)t * pr + x0, w0, w1, (float)r0, (float)r1);
      if (BC == kDirichlet || t < N) {
        acc += k0 ? r0 * r0 : 0.0;
        acc += k1 ? r1 * r1 : 0.0;
      }
    }
  }
  return acc;
}

}  // namespace stream
}  // namespace mg
