// The paper's controlled two-level experiment (Section 4.1; Table 1: N_grid,
// r_min, N_step, N_smooth, N_smooth,pre; appendix V-CYCLE with a single
// coarse level that is relaxed, not solved), batched: one workgroup per
// problem, the whole iteration in one launch.
//
// Per iteration and problem (periodic N x N unique nodes, coarse side
// Nc = N / F):
//   n_smooth red-black Gauss-Seidel sweeps on A p = f (red = (i+j) even first);
//   r = f - A p;  r_c = R_F r (1-D weights (F - |a|)/F^2, x then y);
//   d_c = 0, coarse_sweeps red-black sweeps on A_c d_c = r_c (spacing F h);
//   p += P_F d_c (periodic tensor cubic spline by the factor F);
//   change = ||p_new - p_old||_2 over the unique nodes.
//
// Layout.  1024 threads = 32 x 32 patches of P x P nodes (N = 32 P, P even,
// so every patch starts on a red node and the colour pattern inside a patch
// is the same for every thread).  A thread keeps its patch of p in
// registers for the whole launch.  A half-sweep of colour C reads only
// nodes of the other colour; those on the patch's edge come from the four
// neighbouring patches through LDS (each thread publishes its edge values
// of that colour, one barrier, then reads its neighbours'; a second barrier
// frees the buffer).  h^2 f is packed per thread and colour (k_tl_pack) so
// that a thread's values for one half-sweep are one contiguous run.  The
// sweeps, residual, restriction and coarse sweeps evaluate the same
// expressions in the same order as the definition (no contraction), so they
// are bitwise those of a plain loop; the prolongation uses B-spline
// coefficients (exact periodic inverse of (1,4,1)/6 as a dense Nc x Nc
// matrix) and the 4 x 4-tap evaluation at t = q/F, which is the same spline
// up to rounding.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "mg.h"
#include "mg_internal.h"

namespace mg {
namespace {

// 512 threads = 32 rows x 16 columns of patches, PY x PX nodes each
// (N = 32 PY = 16 PX): two waves per SIMD, so a wave may hold its patch
// (PY PX doubles) in up to 256 registers.
constexpr int kTlThreads = 512;
constexpr int kTlRows = 32, kTlCols = 16;

struct TlArgs {
  int N, F, Nc;
  int n_smooth, coarse_sweeps;
  int sweeps;       // smoothing-only launch: this many sweeps and no iteration
  double tol;       // stop a problem once its change is <= tol; < 0: never
  double h2, h2c;   // h^2 of the fine and the coarse grid
  double* p;        // [batch][N+1][N+1]
  const double* f;  // [batch][N+1][N+1]
  const double* g;  // [batch][2][512][PY * PX/2] packed h^2 f
  double* ps;       // [batch][N][N] smoothed p
  double* r;        // [batch][N][N] residual
  const double* m;  // Nc x Nc periodic prefilter matrix
  const double* w;  // [F][4] B-spline weights at t = q/F
  int* active;      // [batch]
  int* iters;       // [batch]
  double* change;   // [batch]
};

__device__ __forceinline__ int wrapi(int i, int m) { return i < 0 ? i + m : (i >= m ? i - m : i); }

// The same index, opaque to the compiler: the addresses of a phase are
// formed from their own copy of the patch's offset, so that the compiler does
// not keep one phase's per-node addresses live through the next ones (the
// patch itself already fills most of the registers).
__device__ __forceinline__ int fresh(int i) {
  asm volatile("" : "+v"(i));
  return i;
}

// h^2 f packed per (problem, colour, entry, thread), the thread index
// fastest (a wave's loads of one entry are one contiguous run): entry
// i * PX/2 + k of colour c is the node (y0 + i, x0 + ((i + c) & 1) + 2k) of
// the thread's patch.
template <int PY, int PX>
__global__ __launch_bounds__(256) void k_tl_pack(int batch, const double* __restrict__ f,
                                                 double h2, double* __restrict__ g) {
#pragma clang fp contract(off)
  constexpr int HX = PX / 2, L = PY * HX, N = 32 * PY, n = N + 1;
  const long total = (long)batch * 2 * kTlThreads * L;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int tid = (int)(e % kTlThreads);
    const long rest = e / kTlThreads;
    const int k = (int)(rest % L);
    const int c = (int)((rest / L) % 2);
    const long b = rest / (2 * L);
    const int i = k / HX, m = k % HX;
    const int y = (tid / kTlCols) * PY + i, x = (tid % kTlCols) * PX + ((i + c) & 1) + 2 * m;
    g[e] = h2 * f[b * n * n + (long)y * n + x];
  }
}

// Edge values of colour C that the neighbouring patches read, into the
// colour-C exchange buffer: top row, bottom row (PX/2 each), left and
// right column (PY/2 each).
template <int PY, int PX, int C>
__device__ __forceinline__ void tl_publish(const double (&u)[PY][PX], double* B, int tid) {
  constexpr int HX = PX / 2, HY = PY / 2;
  double* Bt = B;
  double* Bb = B + kTlThreads * HX;
  double* Bl = B + 2 * kTlThreads * HX;
  double* Br = B + 2 * kTlThreads * HX + kTlThreads * HY;
#pragma unroll
  for (int k = 0; k < HX; ++k) {
    Bt[tid * HX + k] = u[0][C + 2 * k];
    Bb[tid * HX + k] = u[PY - 1][((PY - 1 + C) & 1) + 2 * k];
  }
#pragma unroll
  for (int k = 0; k < HY; ++k) {
    Bl[tid * HY + k] = u[C + 2 * k][0];
    Br[tid * HY + k] = u[((PX - 1 + C) & 1) + 2 * k][PX - 1];
  }
}

// Rows of h^2 f in flight: the row of step t (t = colour * PY + row, 2 PY
// steps per sweep) sits in slot t % S, S = tl_slots<PY>() dividing 2 PY, so
// a step's slot is the same in every sweep and known at compile time.  Each
// step loads the row S - 1 steps ahead (into the next sweep for the last
// steps: h^2 f does not change between sweeps).
// Three slots for the 6 x 12 patch (its 144 registers leave room for no
// more), four otherwise.
template <int PY>
constexpr int tl_slots() { return PY == 6 ? 3 : 4; }

// One row of one half-sweep (step T of the sweep) on the patch u: reads the
// other colour's edge values of the neighbouring patches from that colour's
// exchange buffer.
template <int PY, int PX, int T>
__device__ __forceinline__ void tl_row(double (&u)[PY][PX], double (&ring)[tl_slots<PY>()][PX / 2],
                                       const double* E, const double* g0, const double* g1,
                                       int up, int dn, int lf, int rt) {
#pragma clang fp contract(off)
  constexpr int HX = PX / 2, HY = PY / 2;
  constexpr int C = T / PY, i = T % PY, O = 1 - C;
  constexpr int BUF = kTlThreads * (PX + PY);
  constexpr int kTlSlots = tl_slots<PY>();
  // Prefetch the row kTlSlots - 1 steps ahead.
  constexpr int TA = (T + kTlSlots - 1) % (2 * PY);
  {
    // The row's offset is formed afresh at every step: otherwise the compiler
    // keeps the addresses of all 2 PY rows live across the sweep loop.
    const double* ga = (TA / PY ? g1 : g0) + fresh((TA % PY) * HX * kTlThreads);
#pragma unroll
    for (int k = 0; k < HX; ++k) ring[TA % kTlSlots][k] = ga[k * kTlThreads];
  }
  const double* B = E + O * BUF;
  const double* Bt = B;
  const double* Bb = B + kTlThreads * HX;
  const double* Bl = B + 2 * kTlThreads * HX;
  const double* Br = B + 2 * kTlThreads * HX + kTlThreads * HY;
#pragma unroll
  for (int k = 0; k < HX; ++k) {
    const int j = ((i + C) & 1) + 2 * k;
    const double vu = i == 0 ? Bb[up * HX + (j >> 1)] : u[i > 0 ? i - 1 : 0][j];
    const double vd = i == PY - 1 ? Bt[dn * HX + (j >> 1)] : u[i < PY - 1 ? i + 1 : 0][j];
    const double vl = j == 0 ? Br[lf * HY + (i >> 1)] : u[i][j > 0 ? j - 1 : 0];
    const double vr = j == PX - 1 ? Bl[rt * HY + (i >> 1)] : u[i][j < PX - 1 ? j + 1 : 0];
    const double s = ((vu + vd) + vl) + vr;
    u[i][j] = (ring[T % kTlSlots][k] + s) * 0.25;
  }
  __builtin_amdgcn_sched_barrier(0);
}

template <int PY, int PX, int T>
__device__ __forceinline__ void tl_steps(double (&u)[PY][PX],
                                         double (&ring)[tl_slots<PY>()][PX / 2],
                                         double* E, const double* g0, const double* g1, int tid,
                                         int up, int dn, int lf, int rt) {
  if constexpr (T < 2 * PY) {
    tl_row<PY, PX, T>(u, ring, E, g0, g1, up, dn, lf, rt);
    if constexpr (T % PY == PY - 1) {
      // End of a half-sweep: publish this colour's edges (its buffer was last
      // read before the previous barrier), then one barrier.
      constexpr int C = T / PY;
      tl_publish<PY, PX, C>(u, E + C * kTlThreads * (PX + PY), tid);
      __syncthreads();
    }
    tl_steps<PY, PX, T + 1>(u, ring, E, g0, g1, tid, up, dn, lf, rt);
  }
}

template <int PY, int PX>
__device__ __forceinline__ void tl_smooth(double (&u)[PY][PX], double* E, const double* gb,
                                          int sweeps, int tid, int tx, int ty) {
  constexpr int HX = PX / 2, L = PY * HX, kTlSlots = tl_slots<PY>();
  static_assert((2 * PY) % kTlSlots == 0, "the ring must divide the steps of a sweep");
  const double* g0 = gb + tid;
  const double* g1 = gb + (size_t)L * kTlThreads + tid;
  const int up = ((ty + kTlRows - 1) % kTlRows) * kTlCols + tx;
  const int dn = ((ty + 1) % kTlRows) * kTlCols + tx;
  const int lf = ty * kTlCols + (tx + kTlCols - 1) % kTlCols;
  const int rt = ty * kTlCols + (tx + 1) % kTlCols;
  double ring[kTlSlots][HX];
#pragma unroll
  for (int t = 0; t < kTlSlots - 1; ++t)
#pragma unroll
    for (int k = 0; k < HX; ++k)
      ring[t][k] = (t / PY ? g1 : g0)[((t % PY) * HX + k) * kTlThreads];
  // The red half-sweep reads black edges: publish them first; the red ones
  // too, so that both buffers hold the patch's edges even after no sweep
  // (the residual reads them).
  tl_publish<PY, PX, 0>(u, E, tid);
  tl_publish<PY, PX, 1>(u, E + kTlThreads * (PX + PY), tid);
  __syncthreads();
#pragma unroll 1
  for (int s = 0; s < sweeps; ++s) tl_steps<PY, PX, 0>(u, ring, E, g0, g1, tid, up, dn, lf, rt);
}

// Patch store to the caller's grid, seam included (row and column N repeat
// row and column 0).
template <int PY, int PX>
__device__ __forceinline__ void tl_store(const double (&u)[PY][PX], double* p, int n, int tx,
                                         int ty) {
  const int N = n - 1, y0 = ty * PY, x0 = tx * PX;
  const int o = fresh(y0 * n + x0);
#pragma unroll
  for (int i = 0; i < PY; ++i)
#pragma unroll
    for (int j = 0; j < PX; ++j) p[o + i * n + j] = u[i][j];
  if (ty == 0)
#pragma unroll
    for (int j = 0; j < PX; ++j) p[(size_t)N * n + x0 + j] = u[0][j];
  if (tx == 0)
#pragma unroll
    for (int i = 0; i < PY; ++i) p[(size_t)(y0 + i) * n + N] = u[i][0];
  if (tx == 0 && ty == 0) p[(size_t)N * n + N] = u[0][0];
}

// One launch = one iteration of every active problem (or, with
// a.sweeps > 0, that many smoothing sweeps and nothing else).
template <int PY, int PX, int F>
__global__ __launch_bounds__(kTlThreads) void k_twolevel(TlArgs a) {
#pragma clang fp contract(off)
  extern __shared__ double lds[];
  constexpr int N = 32 * PY, n = N + 1, L = PY * (PX / 2), Nc = N / F;
  const int b = blockIdx.x;
  if (a.sweeps == 0 && !a.active[b]) return;  // the same value for the whole workgroup
  const int tid = threadIdx.x, tx = tid % kTlCols, ty = tid / kTlCols;
  const int y0 = ty * PY, x0 = tx * PX;
  double* p = a.p + (size_t)b * n * n;
  const double* f = a.f + (size_t)b * n * n;
  const double* gb = a.g + (size_t)b * 2 * kTlThreads * L;
  double* ps = a.ps + (size_t)b * N * N;
  double* rr = a.r + (size_t)b * N * N;
  double* E = lds;                 // smoothing: the two colours' edge buffers
  double* S = lds;                 // transfers: N x Nc x-sums, then d_c and t
  double* RC = lds + N * Nc;       // Nc x Nc restricted residual, then the coefficients
  double* DC = S;
  double* T = S + Nc * Nc;
  double* CC = RC;
  double* XR = S;                  // Nc x N: the coefficients interpolated along x
  double* red = lds + (2 * kTlThreads * (PX + PY) > N * Nc + Nc * Nc
                           ? 2 * kTlThreads * (PX + PY) : N * Nc + Nc * Nc);
  double* W = red + kTlThreads;    // 4F B-spline weights
  double* M = S + 2 * Nc * Nc;     // Nc x Nc prefilter matrix (loaded in phase 5)
  static_assert(3 * Nc * Nc <= N * Nc, "d_c, t and the matrix must fit over the x-sums");
  for (int t = threadIdx.x; t < 4 * F; t += kTlThreads) W[t] = a.w[t];

  {
    // Smoothing: the patch lives in registers only here.
    double u[PY][PX];
    const int o = fresh(y0 * n + x0);
#pragma unroll
    for (int i = 0; i < PY; ++i)
#pragma unroll
      for (int j = 0; j < PX; ++j) u[i][j] = p[o + i * n + j];
    if (a.sweeps > 0) {
      tl_smooth<PY, PX>(u, E, gb, a.sweeps, tid, tx, ty);
      tl_store<PY, PX>(u, p, n, tx, ty);
      return;
    }
    // 1. pre-smoothing (the appendix relaxes at the start of an iteration)
    tl_smooth<PY, PX>(u, E, gb, a.n_smooth, tid, tx, ty);
    // The smoothed patch, thread index fastest (for the correction in 7).
    double* pt = ps + tid;
#pragma unroll
    for (int i = 0; i < PY; ++i)
#pragma unroll
      for (int j = 0; j < PX; ++j) pt[(i * PX + j) * kTlThreads] = u[i][j];
    // 2. r = f - A p with A p = (4 p - (up + down + left + right)) N^2.
    //    Neighbours across the patch's edges come from the exchange buffers,
    //    which hold both colours' edge values after the last sweep.
    constexpr int HX = PX / 2, HY = PY / 2, BUF = kTlThreads * (PX + PY);
    const int up = ((ty + kTlRows - 1) % kTlRows) * kTlCols + tx;
    const int dn = ((ty + 1) % kTlRows) * kTlCols + tx;
    const int lf = ty * kTlCols + (tx + kTlCols - 1) % kTlCols;
    const int rt = ty * kTlCols + (tx + 1) % kTlCols;
    const double inv_h2 = (double)N * (double)N;
#pragma unroll
    for (int i = 0; i < PY; ++i) {
      const int y = y0 + i;
      const double* frow = f + fresh(y * n + x0);
      double* rrow = rr + fresh(y * N + x0);
#pragma unroll
      for (int j = 0; j < PX; ++j) {
        const double* Bu = E + ((1 + j) & 1) * BUF + kTlThreads * HX;          // bottom rows
        const double* Bd = E + (j & 1) * BUF;                                  // top rows
        const double* Bl = E + ((1 + i) & 1) * BUF + 2 * kTlThreads * HX + kTlThreads * HY;
        const double* Br = E + (i & 1) * BUF + 2 * kTlThreads * HX;            // left columns
        const double vu = i > 0 ? u[i > 0 ? i - 1 : 0][j] : Bu[up * HX + (j >> 1)];
        const double vd = i < PY - 1 ? u[i < PY - 1 ? i + 1 : 0][j] : Bd[dn * HX + (j >> 1)];
        const double vl = j > 0 ? u[i][j > 0 ? j - 1 : 0] : Bl[lf * HY + (i >> 1)];
        const double vr = j < PX - 1 ? u[i][j < PX - 1 ? j + 1 : 0] : Br[rt * HY + (i >> 1)];
        const double s = ((vu + vd) + vl) + vr;
        const double au = (4.0 * u[i][j] - s) * inv_h2;
        rrow[j] = frow[j] - au;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();
  // 3. restriction: along x for every fine row, then along y
  const double wden = (double)(F * F);
#pragma unroll 1
  for (int t = tid; t < N * Nc; t += kTlThreads) {
    const int i = t / Nc, J = t % Nc;
    const double* row = rr + (size_t)i * N;
    double acc = 0.0;
#pragma unroll
    for (int q = -(F - 1); q <= F - 1; ++q) {
      const double wq = (double)(F - (q < 0 ? -q : q)) / wden;
      acc += wq * row[wrapi(F * J + q, N)];
    }
    S[t] = acc;
  }
  __syncthreads();
#pragma unroll 1
  for (int t = tid; t < Nc * Nc; t += kTlThreads) {
    const int I = t / Nc, J = t % Nc;
    double acc = 0.0;
#pragma unroll
    for (int q = -(F - 1); q <= F - 1; ++q) {
      const double wq = (double)(F - (q < 0 ? -q : q)) / wden;
      acc += wq * S[wrapi(F * I + q, N) * Nc + J];
    }
    RC[t] = acc;
  }
  __syncthreads();
  // 4. coarse sweeps from zero (the appendix relaxes the coarsest level)
#pragma unroll 1
  for (int t = tid; t < Nc * Nc; t += kTlThreads) DC[t] = 0.0;
  __syncthreads();
  const int hc = Nc / 2;
#pragma unroll 1
  for (int sw = 0; sw < 2 * a.coarse_sweeps; ++sw) {
    const int c = sw & 1;
#pragma unroll 1
    for (int t = tid; t < Nc * hc; t += kTlThreads) {
      const int I = t / hc, J = ((I + c) & 1) + 2 * (t % hc);
      const double sn = ((DC[wrapi(I - 1, Nc) * Nc + J] + DC[wrapi(I + 1, Nc) * Nc + J]) +
                         DC[I * Nc + wrapi(J - 1, Nc)]) + DC[I * Nc + wrapi(J + 1, Nc)];
      DC[I * Nc + J] = (a.h2c * RC[I * Nc + J] + sn) * 0.25;
    }
    __syncthreads();
  }
  // 5. B-spline coefficients of d_c (rows, then columns)
  for (int t = tid; t < Nc * Nc; t += kTlThreads) M[t] = a.m[t];
  __syncthreads();
#pragma unroll 1
  for (int t = tid; t < Nc * Nc; t += kTlThreads) {
    const int I = t / Nc, J = t % Nc;
    double acc = 0.0;
#pragma unroll 1
    for (int k = 0; k < Nc; ++k) acc += M[J * Nc + k] * DC[I * Nc + k];
    T[t] = acc;
  }
  __syncthreads();
#pragma unroll 1
  for (int t = tid; t < Nc * Nc; t += kTlThreads) {
    const int I = t / Nc, J = t % Nc;
    double acc = 0.0;
#pragma unroll 1
    for (int k = 0; k < Nc; ++k) acc += M[I * Nc + k] * T[k * Nc + J];
    CC[t] = acc;
  }
  __syncthreads();
  // 6. the spline along x for every coarse row at every fine column
#pragma unroll 1
  for (int t = tid; t < Nc * N; t += kTlThreads) {
    const int I = t / N, x = t % N, J0 = x / F;
    const double* wx = W + 4 * (x % F);
    const double* row = CC + I * Nc;
    double h = 0.0;
#pragma unroll
    for (int ax = 0; ax < 4; ++ax) h += wx[ax] * row[wrapi(J0 - 1 + ax, Nc)];
    XR[t] = h;
  }
  __syncthreads();
  // 7. then along y per node: p += P_F d_c from the smoothed iterate; the
  //    iteration's change against the previous iterate (still in p); store
  double ch = 0.0;
#pragma unroll 2
  for (int i = 0; i < PY; ++i) {
    const int y = y0 + i, I0 = y / F;
    const double* wy = W + 4 * (y % F);
    const double w0 = wy[0], w1 = wy[1], w2 = wy[2], w3 = wy[3];
    const double* r0 = XR + wrapi(I0 - 1, Nc) * N + x0;
    const double* r1 = XR + I0 * N + x0;
    const double* r2 = XR + wrapi(I0 + 1, Nc) * N + x0;
    const double* r3 = XR + wrapi(I0 + 2, Nc) * N + x0;
    const double* srow = ps + tid + i * PX * kTlThreads;
    double* prow = p + (size_t)y * n + x0;
    double nv[PX];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
      const double v = ((w0 * r0[j] + w1 * r1[j]) + w2 * r2[j]) + w3 * r3[j];
      nv[j] = srow[j * kTlThreads] + v;
      const double d = nv[j] - prow[j];
      ch += d * d;
    }
#pragma unroll
    for (int j = 0; j < PX; ++j) prow[j] = nv[j];
    if (tx == 0) p[(size_t)y * n + N] = nv[0];
    if (y == 0) {
#pragma unroll
      for (int j = 0; j < PX; ++j) p[(size_t)N * n + x0 + j] = nv[j];
      if (tx == 0) p[(size_t)N * n + N] = nv[0];
    }
  }
  red[tid] = ch;
  __syncthreads();
#pragma unroll 1
  for (int w = kTlThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    const double c = sqrt(red[0]);
    a.change[b] = c;
    a.iters[b] += 1;
    if ((a.tol >= 0.0 && c <= a.tol) || !(c == c)) a.active[b] = 0;
  }
}

// LDS: the larger of the two colour buffers and the transfers' arrays,
// then the reduction slots.
size_t tl_lds_bytes(int N, int Nc) {
  const int PY = N / 32, PX = N / 16;
  const size_t e = (size_t)2 * kTlThreads * (PX + PY);
  const size_t t = (size_t)N * Nc + (size_t)Nc * Nc;
  return (std::max(e, t) + kTlThreads + 4 * 32) * sizeof(double);
}

template <int PY, int PX, int F>
hipError_t tl_prepare(size_t lds) {
  static bool done = false;
  if (done) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_twolevel<PY, PX, F>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
  if (e == hipSuccess) done = true;
  return e;
}

}  // namespace
}  // namespace mg

struct mg_twolevel_s {
  int N = 0, F = 0, Nc = 0, batch = 0, n_smooth = 0, coarse_sweeps = 0, device = 0;
  hipStream_t stream = nullptr;
  double *g = nullptr, *ps = nullptr, *r = nullptr, *table = nullptr, *change = nullptr;
  int *active = nullptr, *iters = nullptr;
  double* host_change = nullptr;  // pinned
  int* host_iters = nullptr;      // pinned
  int* host_active = nullptr;     // pinned
};

namespace mg {
namespace {

int32_t tl_fail(int32_t st, const std::string& why) { return set_last_error(st, why.c_str()); }

#define TL_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return tl_fail(MG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

void tl_free(mg_twolevel_s* c) {
  (void)hipFree(c->g);
  (void)hipFree(c->ps);
  (void)hipFree(c->r);
  (void)hipFree(c->table);
  (void)hipFree(c->change);
  (void)hipFree(c->active);
  (void)hipFree(c->iters);
  (void)hipHostFree(c->host_change);
  (void)hipHostFree(c->host_iters);
  (void)hipHostFree(c->host_active);
  delete c;
}

TlArgs tl_args(const mg_twolevel_s* c, double* p, const double* f) {
  TlArgs a{};
  a.N = c->N;
  a.F = c->F;
  a.Nc = c->Nc;
  a.n_smooth = c->n_smooth;
  a.coarse_sweeps = c->coarse_sweeps;
  const double hd = 1.0 / (double)c->N, hc = 1.0 / (double)c->Nc;
  a.h2 = hd * hd;
  a.h2c = hc * hc;
  a.p = p;
  a.f = f;
  a.g = c->g;
  a.ps = c->ps;
  a.r = c->r;
  a.m = c->table;
  a.w = c->table + (size_t)c->Nc * c->Nc;
  a.active = c->active;
  a.iters = c->iters;
  a.change = c->change;
  a.tol = -1.0;
  return a;
}

template <int PY, int PX, int F>
int32_t tl_launch(mg_twolevel_s* c, const TlArgs& a, bool pack) {
  if (pack) {
    const long total = (long)c->batch * 2 * kTlThreads * PY * (PX / 2);
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL((k_tl_pack<PY, PX>), dim3(blocks), dim3(256), 0, c->stream, c->batch,
                       a.f, a.h2, const_cast<double*>(a.g));
    TL_HIP(hipGetLastError());
  }
  const size_t lds = tl_lds_bytes(c->N, c->Nc);
  TL_HIP((tl_prepare<PY, PX, F>(lds)));
  hipLaunchKernelGGL((k_twolevel<PY, PX, F>), dim3(c->batch), dim3(kTlThreads), lds, c->stream,
                     a);
  TL_HIP(hipGetLastError());
  return MG_OK;
}

template <int PY, int PX>
int32_t tl_launch_f(mg_twolevel_s* c, const TlArgs& a, bool pack) {
  switch (c->F) {
    case 4: return tl_launch<PY, PX, 4>(c, a, pack);
    case 8: return tl_launch<PY, PX, 8>(c, a, pack);
    case 16: return tl_launch<PY, PX, 16>(c, a, pack);
    default: return tl_launch<PY, PX, 32>(c, a, pack);
  }
}

// One launch: smoothing only (a.sweeps > 0) or one iteration.
int32_t tl_run(mg_twolevel_s* c, const TlArgs& a, bool pack) {
  switch (c->N) {
    case 64: return tl_launch_f<2, 4>(c, a, pack);
    case 128: return tl_launch_f<4, 8>(c, a, pack);
    default: return tl_launch_f<6, 12>(c, a, pack);
  }
}

int32_t tl_check(mg_twolevel_s* c, double* p, const double* f) {
  if (!c) return tl_fail(MG_ERR_INVALID_ARG, "NULL context");
  if (!p || !f) return tl_fail(MG_ERR_INVALID_ARG, "NULL array");
  if ((const void*)p == (const void*)f) return tl_fail(MG_ERR_INVALID_ARG, "p aliases f");
  if (hipSetDevice(c->device) != hipSuccess) return tl_fail(MG_ERR_HIP, "hipSetDevice");
  return MG_OK;
}

// Sets every problem active with a zero iteration count.
int32_t tl_reset(mg_twolevel_s* c) {
  std::vector<int> ones(c->batch, 1);
  TL_HIP(hipMemcpyAsync(c->active, ones.data(), sizeof(int) * c->batch, hipMemcpyHostToDevice,
                        c->stream));
  TL_HIP(hipMemsetAsync(c->iters, 0, sizeof(int) * c->batch, c->stream));
  return MG_OK;
}

int32_t tl_read(mg_twolevel_s* c, int32_t* iters_out, double* change_out) {
  TL_HIP(hipMemcpyAsync(c->host_change, c->change, sizeof(double) * c->batch,
                        hipMemcpyDeviceToHost, c->stream));
  TL_HIP(hipMemcpyAsync(c->host_iters, c->iters, sizeof(int) * c->batch, hipMemcpyDeviceToHost,
                        c->stream));
  TL_HIP(hipStreamSynchronize(c->stream));
  for (int b = 0; b < c->batch; ++b) {
    if (change_out) change_out[b] = c->host_change[b];
    if (iters_out) iters_out[b] = c->host_iters[b];
  }
  return MG_OK;
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

int32_t mg_twolevel_setup(int32_t n_unique, int32_t factor, int32_t batch, int32_t n_smooth,
                          int32_t coarse_sweeps, void* hip_stream, mg_twolevel* out) {
  set_last_error(MG_OK, "");
  if (!out) return tl_fail(MG_ERR_INVALID_ARG, "NULL out");
  *out = nullptr;
  if (n_unique != 64 && n_unique != 128 && n_unique != 192)
    return tl_fail(MG_ERR_UNSUPPORTED, "unique side must be 64, 128 or 192");
  if (factor < 4 || factor > 32 || (factor & (factor - 1)) || n_unique % factor ||
      (n_unique / factor) % 2)
    return tl_fail(MG_ERR_INVALID_ARG, "factor must be 4, 8, 16 or 32 with N/F even");
  if (batch <= 0) return tl_fail(MG_ERR_INVALID_ARG, "batch <= 0");
  if (n_smooth < 0 || n_smooth > 1000 || coarse_sweeps < 0 || coarse_sweeps > 1000)
    return tl_fail(MG_ERR_INVALID_ARG, "sweep counts outside 0..1000");
  mg_twolevel_s* c = nullptr;
  try {
    c = new mg_twolevel_s();
  } catch (const std::bad_alloc&) {
    return tl_fail(MG_ERR_OOM, "host allocation failed");
  }
  c->N = n_unique;
  c->F = factor;
  c->Nc = n_unique / factor;
  c->batch = batch;
  c->n_smooth = n_smooth;
  c->coarse_sweeps = coarse_sweeps;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    tl_free(c);
    return tl_fail(MG_ERR_HIP, "hipGetDevice");
  }
  const size_t nn = (size_t)n_unique * n_unique * batch;
  const int Nc = c->Nc, F = factor;
  auto fail_oom = [&](const char* what) {
    tl_free(c);
    return tl_fail(MG_ERR_OOM, std::string("hipMalloc ") + what);
  };
  if (hipMalloc(&c->g, sizeof(double) * nn) != hipSuccess) return fail_oom("g");
  if (hipMalloc(&c->ps, sizeof(double) * nn) != hipSuccess) return fail_oom("ps");
  if (hipMalloc(&c->r, sizeof(double) * nn) != hipSuccess) return fail_oom("r");
  if (hipMalloc(&c->table, sizeof(double) * ((size_t)Nc * Nc + 4 * F)) != hipSuccess)
    return fail_oom("table");
  if (hipMalloc(&c->change, sizeof(double) * batch) != hipSuccess) return fail_oom("change");
  if (hipMalloc(&c->active, sizeof(int) * batch) != hipSuccess) return fail_oom("active");
  if (hipMalloc(&c->iters, sizeof(int) * batch) != hipSuccess) return fail_oom("iters");
  if (hipHostMalloc(&c->host_change, sizeof(double) * batch) != hipSuccess)
    return fail_oom("host change");
  if (hipHostMalloc(&c->host_iters, sizeof(int) * batch) != hipSuccess)
    return fail_oom("host iters");
  if (hipHostMalloc(&c->host_active, sizeof(int) * batch) != hipSuccess)
    return fail_oom("host active");
  // Exact periodic inverse of (1,4,1)/6 on Nc nodes (the whole period of
  // the spline prefilter's taps), then the cubic B-spline weights of the
  // four coarse coefficients around each of the F fine offsets.
  std::vector<double> tab((size_t)Nc * Nc + 4 * F);
  std::vector<double> full((size_t)(Nc + 1) * (Nc + 1));
  prefilter_matrix(Nc + 1, kPeriodic, full.data());
  for (int i = 0; i < Nc; ++i)
    for (int k = 0; k < Nc; ++k) tab[(size_t)i * Nc + k] = full[(size_t)i * (Nc + 1) + k];
  for (int q = 0; q < F; ++q) {
    const double t = (double)q / F, s = 1.0 - t;
    double* wq = tab.data() + (size_t)Nc * Nc + 4 * q;
    wq[0] = s * s * s / 6.0;
    wq[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
    wq[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
    wq[3] = t * t * t / 6.0;
  }
  if (hipMemcpy(c->table, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice) !=
      hipSuccess) {
    tl_free(c);
    return tl_fail(MG_ERR_HIP, "hipMemcpy table");
  }
  *out = c;
  return MG_OK;
}

int32_t mg_twolevel_smooth(mg_twolevel ctx, double* p, const double* f, int32_t sweeps) {
  set_last_error(MG_OK, "");
  int32_t st = tl_check(ctx, p, f);
  if (st != MG_OK) return st;
  if (sweeps < 0) return tl_fail(MG_ERR_INVALID_ARG, "sweeps < 0");
  if (sweeps == 0) return MG_OK;
  TlArgs a = tl_args(ctx, p, f);
  a.sweeps = sweeps;
  return tl_run(ctx, a, true);
}

int32_t mg_twolevel_cycle(mg_twolevel ctx, double* p, const double* f, int32_t ncycles,
                          double* change_out) {
  set_last_error(MG_OK, "");
  int32_t st = tl_check(ctx, p, f);
  if (st != MG_OK) return st;
  if (ncycles < 0) return tl_fail(MG_ERR_INVALID_ARG, "ncycles < 0");
  if (ncycles == 0) return MG_OK;
  st = tl_reset(ctx);
  if (st != MG_OK) return st;
  TlArgs a = tl_args(ctx, p, f);
  for (int k = 0; k < ncycles; ++k) {
    st = tl_run(ctx, a, k == 0);
    if (st != MG_OK) return st;
  }
  if (!change_out) return MG_OK;
  st = tl_read(ctx, nullptr, change_out);
  if (st != MG_OK) return st;
  for (int b = 0; b < ctx->batch; ++b)
    if (!std::isfinite(change_out[b])) return tl_fail(MG_ERR_NONFINITE, "non-finite change");
  return MG_OK;
}

int32_t mg_twolevel_solve(mg_twolevel ctx, double* p, const double* f, int32_t n_pre, double tol,
                          int32_t max_iter, int32_t* iters_out, double* change_out) {
  set_last_error(MG_OK, "");
  int32_t st = tl_check(ctx, p, f);
  if (st != MG_OK) return st;
  if (n_pre < 0 || max_iter < 0 || !(tol >= 0.0))
    return tl_fail(MG_ERR_INVALID_ARG, "n_pre < 0, max_iter < 0 or tol not >= 0");
  TlArgs a = tl_args(ctx, p, f);
  bool packed = false;
  if (n_pre > 0) {
    a.sweeps = n_pre;
    st = tl_run(ctx, a, true);
    if (st != MG_OK) return st;
    packed = true;
    a.sweeps = 0;
  }
  st = tl_reset(ctx);
  if (st != MG_OK) return st;
  a.tol = tol;
  // Iterations in chunks; a problem whose change reaches tol marks itself
  // inactive on the device and later launches skip it.  Between chunks the
  // host reads the flags and stops once none is left.
  constexpr int kChunk = 8;
  int done = 0;
  while (done < max_iter) {
    const int k = std::min(kChunk, max_iter - done);
    for (int j = 0; j < k; ++j) {
      st = tl_run(ctx, a, !packed);
      if (st != MG_OK) return st;
      packed = true;
    }
    done += k;
    TL_HIP(hipMemcpyAsync(ctx->host_active, ctx->active, sizeof(int) * ctx->batch,
                          hipMemcpyDeviceToHost, ctx->stream));
    TL_HIP(hipStreamSynchronize(ctx->stream));
    bool any = false;
    for (int b = 0; b < ctx->batch; ++b) any = any || ctx->host_active[b] != 0;
    if (!any) break;
  }
  std::vector<int32_t> it(ctx->batch);
  std::vector<double> ch(ctx->batch);
  st = tl_read(ctx, it.data(), ch.data());
  if (st != MG_OK) return st;
  int32_t result = MG_OK;
  for (int b = 0; b < ctx->batch; ++b) {
    if (iters_out) iters_out[b] = it[b];
    if (change_out) change_out[b] = max_iter > 0 ? ch[b] : NAN;
    if (max_iter > 0 && !std::isfinite(ch[b]))
      result = MG_ERR_NONFINITE;
    else if (result == MG_OK && (max_iter == 0 || !(ch[b] <= tol)))
      result = MG_ERR_NOT_CONVERGED;
  }
  if (result != MG_OK)
    tl_fail(result, result == MG_ERR_NONFINITE ? "non-finite change" : "max_iter reached above tol");
  return result;
}

int32_t mg_twolevel_destroy(mg_twolevel ctx) {
  if (!ctx) return MG_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  tl_free(ctx);
  return MG_OK;
}

}  // extern "C"
