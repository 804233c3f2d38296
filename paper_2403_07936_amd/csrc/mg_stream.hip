// Standalone register-streaming down and up kernels: one wavefront per
// (band, row segment) item; the work itself is in mg_stream_dev.h.

#include "mg_stream_dev.h"

namespace mg {
using namespace stream;
namespace {

template <typename T, int BC, int UIN>
__global__ void __launch_bounds__(64 * kWaves)
    k_down_s(int n, const T* __restrict__ uin, int pui, T* __restrict__ uout, int puo,
             const T* __restrict__ f, int pf, T* __restrict__ fc, int pfc, int nbands, int nitems,
             int hs, T h2, T inv_h2) {
  const int item = wave_uniform(xcd_tile(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (item >= nitems) return;
  down_wave<T, BC, UIN>(n, uin, pui, uout, puo, f, pf, fc, pfc, item % nbands, item / nbands, hs,
                        h2, inv_h2, threadIdx.x & 63);
}

template <typename T, int BC, bool ADD>
__global__ void __launch_bounds__(64 * kWaves)
    k_up_s(int n, const T* __restrict__ uin, int pui, T* __restrict__ uout, int puo,
           const T* __restrict__ f, int pf, const T* __restrict__ c, int pc, int nbands,
           int nitems, int hs, T h2, double* __restrict__ u64, int p64) {
  const int item = wave_uniform(xcd_tile(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (item >= nitems) return;
  up_wave<T, BC, ADD>(n, uin, pui, uout, puo, f, pf, c, pc, item % nbands, item / nbands, hs, h2,
                      threadIdx.x & 63, u64, p64);
}

// Mixed path, level 0: r32 = fl32(f - A u) with f, u and the arithmetic in
// FP64, at every node of rows [ys, ys + hs) (0 on the Dirichlet boundary;
// periodic seam row and column = node 0).  One wavefront per (band, row
// segment): lanes 1 .. 62 own the band's kResOwned columns, lanes 0 and 63
// only supply neighbours.  Rows stream through 8-slot rings, u loaded
// kAheadRes + 1 rows and f kAheadRes rows before use.  Each wavefront writes
// the sum of r^2 over the unknowns it owns to partials[item], in a fixed
// order.
constexpr int kResOwned = 124;
constexpr int kAheadRes = 4;
static_assert(kAheadRes <= 5, "u ring holds rows t-1 .. t+1+kAheadRes");

template <int BC>
__global__ void __launch_bounds__(64 * kWaves)
    k_residual_mixed_s(int n, const double* __restrict__ u, int pu, const double* __restrict__ f,
                       int pf, float* __restrict__ r32, int pr, double* __restrict__ partials,
                       int nbands, int nitems, int hs, double inv_h2) {
  const int item = wave_uniform(xcd_tile(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (item >= nitems) return;
  const int lane = threadIdx.x & 63;
  const int band = item % nbands, seg = item / nbands;
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
#pragma unroll
  for (int q = 0; q < kAheadRes + 2; ++q) {
    const int r = ys - 1 + q;
    load_row<double, BC>(U[q], u, pu, r < n ? r : n, n, col);
  }
#pragma unroll
  for (int q = 0; q < kAheadRes; ++q) {
    const int r = ys + q;
    load_row<double, BC>(F[q], f, pf, r < n ? r : n - 1, n, col);
  }
  double acc = 0.0;
  for (int sb = 0; sb < steps; sb += 8) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int s = sb + k;
      if (s >= steps) break;
      const int t = ys + s;
      // Rows past n feed no step of the segment: clamped, so that a periodic
      // row index wraps at most once.
      const int tu = t + kAheadRes + 1, tf = t + kAheadRes;
      load_row<double, BC>(U[(k + kAheadRes + 2) & 7], u, pu, tu < n ? tu : n, n, col);
      load_row<double, BC>(F[(k + kAheadRes) & 7], f, pf, tf < n ? tf : n - 1, n, col);
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
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
  if (lane == 0) partials[item] = acc;
}

}  // namespace

// Rows per wavefront segment: 64 on large grids; on small grids shorter, so
// that about 1024 wavefronts share the work (each segment also loads ~10 halo
// rows, which is cheap next to the latency a long serial segment costs).
int stream_segment_rows(int n, int bc, int owned_cols) {
  const int extent = bc == kPeriodic ? n - 1 : n;
  const int nb = (extent + owned_cols - 1) / owned_cols;
  int hs = 64;
  while (hs > 8 && (long)nb * ((extent + hs - 1) / hs) < 1024) hs -= 8;
  return hs;
}

int stream_down_owned() { return kDownOwned; }
int stream_up_owned() { return kUpOwned; }

template <typename T>
hipError_t launch_down_stream(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout,
                              int puo, const T* f, int pf, T* fc, int pfc, int hs) {
  // A periodic band wraps at most once only from n - 1 >= 128 on (levels
  // this small are in the tail); hs must be even (row parity of a segment).
  if ((bc == kPeriodic && n - 1 < 128) || (hs > 0 && (hs & 1))) return hipErrorInvalidValue;
  const int extent = bc == kPeriodic ? n - 1 : n;
  if (hs <= 0) hs = stream_segment_rows(n, bc, kDownOwned);
  const int nb = (extent + kDownOwned - 1) / kDownOwned;
  const int ns = (extent + hs - 1) / hs;
  const int items = nb * ns;
  const int blocks = (items + kWaves - 1) / kWaves;
  const double hd = 1.0 / (double)(n - 1);
  const T h2 = T(hd * hd), inv_h2 = T((double)(n - 1) * (double)(n - 1));
  if (bc == kDirichlet && uin)
    hipLaunchKernelGGL((k_down_s<T, kDirichlet, 1>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, fc, pfc, nb, items, hs, h2, inv_h2);
  else if (bc == kDirichlet)
    hipLaunchKernelGGL((k_down_s<T, kDirichlet, 0>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, fc, pfc, nb, items, hs, h2, inv_h2);
  else if (uin)
    hipLaunchKernelGGL((k_down_s<T, kPeriodic, 1>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, fc, pfc, nb, items, hs, h2, inv_h2);
  else
    hipLaunchKernelGGL((k_down_s<T, kPeriodic, 0>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, fc, pfc, nb, items, hs, h2, inv_h2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_up_stream(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout, int puo,
                            const T* f, int pf, const T* c, int pc, int hs, double* u64,
                            int p64) {
  if ((bc == kPeriodic && n - 1 < 128) || (hs > 0 && (hs & 1))) return hipErrorInvalidValue;
  const int extent = bc == kPeriodic ? n - 1 : n;
  if (hs <= 0) hs = stream_segment_rows(n, bc, kUpOwned);
  const int nb = (extent + kUpOwned - 1) / kUpOwned;
  const int ns = (extent + hs - 1) / hs;
  const int items = nb * ns;
  const int blocks = (items + kWaves - 1) / kWaves;
  const double hd = 1.0 / (double)(n - 1);
  const T h2 = T(hd * hd);
  if (bc == kDirichlet && u64)
    hipLaunchKernelGGL((k_up_s<T, kDirichlet, true>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, c, pc, nb, items, hs, h2, u64, p64);
  else if (bc == kDirichlet)
    hipLaunchKernelGGL((k_up_s<T, kDirichlet, false>), dim3(blocks), dim3(64 * kWaves), 0, s, n,
                       uin, pui, uout, puo, f, pf, c, pc, nb, items, hs, h2, u64, p64);
  else if (u64)
    hipLaunchKernelGGL((k_up_s<T, kPeriodic, true>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, c, pc, nb, items, hs, h2, u64, p64);
  else
    hipLaunchKernelGGL((k_up_s<T, kPeriodic, false>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, c, pc, nb, items, hs, h2, u64, p64);
  return hipGetLastError();
}

#define MG_STREAM_INSTANTIATE(T)                                                                \
  template hipError_t launch_down_stream<T>(hipStream_t, int, int, const T*, int, T*, int,      \
                                            const T*, int, T*, int, int);                        \
  template hipError_t launch_up_stream<T>(hipStream_t, int, int, const T*, int, T*, int,        \
                                          const T*, int, const T*, int, int, double*, int);

MG_STREAM_INSTANTIATE(double)
MG_STREAM_INSTANTIATE(float)

hipError_t launch_residual_mixed(hipStream_t s, int bc, int n, const double* u, int pu,
                                 const double* f, int pf, float* r32, int pr, double* partials,
                                 int* nblocks) {
  const double inv_h2 = (double)(n - 1) * (double)(n - 1);
  const int nb = (n + kResOwned - 1) / kResOwned;
  int hs = 64;
  while (hs > 8 && (long)nb * ((n + hs - 1) / hs) < 2048) hs -= 8;
  const int items = nb * ((n + hs - 1) / hs);
  const int blocks = (items + kWaves - 1) / kWaves;
  *nblocks = items;
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_residual_mixed_s<kDirichlet>), dim3(blocks), dim3(64 * kWaves), 0, s, n,
                       u, pu, f, pf, r32, pr, partials, nb, items, hs, inv_h2);
  else
    hipLaunchKernelGGL((k_residual_mixed_s<kPeriodic>), dim3(blocks), dim3(64 * kWaves), 0, s, n,
                       u, pu, f, pf, r32, pr, partials, nb, items, hs, inv_h2);
  return hipGetLastError();
}

}  // namespace mg
