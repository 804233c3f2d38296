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
             int hs, T h2, T inv_h2, const CallerArgs* ca) {
  const int item = wave_uniform(xcd_tile(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (item >= nitems) return;
  if constexpr (sizeof(T) == sizeof(double))
    if (ca) uin = ca->u, f = ca->f;
  down_wave<T, BC, UIN>(n, uin, pui, uout, puo, f, pf, fc, pfc, item % nbands, item / nbands, hs,
                        h2, inv_h2, threadIdx.x & 63);
}

// The FP64 down pass from the caller's iterate that also writes each
// wavefront's sum of r^2 of that iterate, over the unknowns it owns, to
// partials[item] (lanes reduced in a fixed order).  Held to three
// wavefronts per SIMD, as the plain pass runs.
template <int BC>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(3, 3)))
    k_down_norm_s(int n, const double* __restrict__ uin, int pui, double* __restrict__ uout,
                  int puo, const double* __restrict__ f, int pf, double* __restrict__ fc, int pfc,
                  int nbands, int nitems, int hs, double h2, double inv_h2, const CallerArgs* ca,
                  double* __restrict__ partials) {
  const int item = wave_uniform(xcd_tile(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (item >= nitems) return;
  if (ca) uin = ca->u, f = ca->f;
  double2 acc = down_wave<double, BC, 1, false, true, 1>(
      n, uin, pui, uout, puo, f, pf, fc, pfc, item % nbands, item / nbands, hs, h2, inv_h2,
      threadIdx.x & 63);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc.x += __shfl_down(acc.x, off);
  if ((threadIdx.x & 63) == 0) partials[item] = acc.x;
}

// Level-0 down pass of the mixed path with its right-hand side made from
// the FP64 iterate (down_wave with RES).
// SB = false: the pre-smoothed iterate is not stored (k_up_pre_s makes it
// again).  NORM: each wavefront also writes the sums of r^2 and of f^2 over
// the unknowns it owns to partials[item] and partials[nitems + item] (lanes
// reduced in a fixed order), so the pass yields ||f - A u|| of the iterate
// it starts from and ||f||.
template <int BC, bool SB, bool NORM = false>
__global__ void __launch_bounds__(64 * kWaves)
    k_down_res_s(int n, const double* __restrict__ u64, int p64, const double* __restrict__ f64,
                 int pf64, float* __restrict__ r32, int pr, float* __restrict__ uout, int puo,
                 float* __restrict__ fc, int pfc, int nbands, int nitems, int hs, float h2,
                 float inv_h2, double inv_h2d, const CallerArgs* ca,
                 double* __restrict__ partials = nullptr) {
  const int item = wave_uniform(xcd_tile(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (item >= nitems) return;
  if (ca) u64 = ca->u, f64 = ca->f;
  double2 acc = down_wave<float, BC, 0, true, SB, NORM ? 2 : 0>(
      n, nullptr, 0, uout, puo, nullptr, 0, fc, pfc, item % nbands, item / nbands, hs, h2, inv_h2,
      threadIdx.x & 63, u64, p64, f64, pf64, inv_h2d, r32, pr);
  if constexpr (NORM) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc.x += __shfl_down(acc.x, off);
      acc.y += __shfl_down(acc.y, off);
    }
    if ((threadIdx.x & 63) == 0) {
      partials[item] = acc.x;
      partials[nitems + item] = acc.y;
    }
  }
}

// Level-0 up pass of the mixed path after k_down_res_s<BC, false>: the
// pre-smoothed iterate made again from the right-hand side (up_pre_wave),
// the result added into the FP64 iterate.
template <int BC>
__global__ void __launch_bounds__(64 * kWaves)
    k_up_pre_s(int n, const float* __restrict__ f, int pf, const float* __restrict__ c, int pc,
               int nbands, int nitems, int hs, float h2, double* __restrict__ u64, int p64,
               const CallerArgs* ca) {
  const int item = wave_uniform(xcd_tile(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (item >= nitems) return;
  if (ca) u64 = ca->u;
  up_pre_wave<BC>(n, f, pf, c, pc, item % nbands, item / nbands, hs, h2, threadIdx.x & 63, u64,
                  p64);
}

template <typename T, int BC, bool ADD>
__global__ void __launch_bounds__(64 * kWaves)
    k_up_s(int n, const T* __restrict__ uin, int pui, T* __restrict__ uout, int puo,
           const T* __restrict__ f, int pf, const T* __restrict__ c, int pc, int nbands,
           int nitems, int hs, T h2, double* __restrict__ u64, int p64, const CallerArgs* ca) {
  const int item = wave_uniform(xcd_tile(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (item >= nitems) return;
  if (ca) {
    if constexpr (sizeof(T) == sizeof(double))
      uout = ca->u, f = ca->f;
    else
      u64 = ca->u;
  }
  up_wave<T, BC, ADD>(n, uin, pui, uout, puo, f, pf, c, pc, item % nbands, item / nbands, hs, h2,
                      threadIdx.x & 63, u64, p64);
}

// Mixed path, level 0: the FP64 residual by rows (residual_wave); each
// wavefront writes the sum of r^2 over the unknowns it owns to
// partials[item], reduced across its lanes in a fixed order.
template <int BC>
__global__ void __launch_bounds__(64 * kWaves)
    k_residual_mixed_s(int n, const double* __restrict__ u, int pu, const double* __restrict__ f,
                       int pf, float* __restrict__ r32, int pr, double* __restrict__ partials,
                       int nbands, int nitems, int hs, double inv_h2, const CallerArgs* ca) {
  const int item = wave_uniform(xcd_tile(blockIdx.x, gridDim.x) * kWaves + (threadIdx.x >> 6));
  if (item >= nitems) return;
  if (ca) u = ca->u, f = ca->f;
  const int lane = threadIdx.x & 63;
  double acc = residual_wave<BC>(n, u, pu, f, pf, r32, pr, item % nbands, item / nbands, hs,
                                 inv_h2, lane);
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

namespace {
int fit_rows(const void* fn, int extent, int owned) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kWaves, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const long slots = (long)per_cu * kWaves * cus;
  const int nb = (extent + owned - 1) / owned;
  for (int hs = 2; hs < extent; hs += 2)
    if ((long)nb * ((extent + hs - 1) / hs) <= slots) return hs;
  return 0;
}
}  // namespace

template <typename T>
int stream_fit_rows(StreamPass pass, int bc, int n) {
  const int extent = bc == kPeriodic ? n - 1 : n;
  const bool d = bc == kDirichlet;
  const void* fn = nullptr;
  int owned = kDownOwned;
  switch (pass) {
    case kFitDown:
      fn = d ? (const void*)&k_down_s<T, kDirichlet, 0> : (const void*)&k_down_s<T, kPeriodic, 0>;
      break;
    case kFitDownIn:
      fn = d ? (const void*)&k_down_s<T, kDirichlet, 1> : (const void*)&k_down_s<T, kPeriodic, 1>;
      break;
    case kFitDownRes:
      fn = d ? (const void*)&k_down_res_s<kDirichlet, false>
             : (const void*)&k_down_res_s<kPeriodic, false>;
      break;
    case kFitUp:
      fn = d ? (const void*)&k_up_s<T, kDirichlet, false> : (const void*)&k_up_s<T, kPeriodic, false>;
      owned = kUpOwned;
      break;
    case kFitUpPre:
      fn = d ? (const void*)&k_up_pre_s<kDirichlet> : (const void*)&k_up_pre_s<kPeriodic>;
      owned = kUpPreOwned;
      break;
  }
  return fit_rows(fn, extent, owned);
}
template int stream_fit_rows<float>(StreamPass, int, int);
template int stream_fit_rows<double>(StreamPass, int, int);

int stream_down_owned() { return kDownOwned; }
int stream_up_owned() { return kUpOwned; }
int stream_res_owned() { return kResOwned; }

template <typename T>
hipError_t launch_down_stream(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout,
                              int puo, const T* f, int pf, T* fc, int pfc, int hs,
                              const CallerArgs* ca, double* partials, int nparts, int* nitems) {
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
  if (nitems) *nitems = items;
  if (partials) {
    // The norm form: FP64, from the caller's iterate, one partial per
    // wavefront.
    if constexpr (sizeof(T) == sizeof(double)) {
      if (!uin || items > nparts) return hipErrorInvalidValue;
      if (bc == kDirichlet)
        hipLaunchKernelGGL((k_down_norm_s<kDirichlet>), dim3(blocks), dim3(64 * kWaves), 0, s, n,
                           uin, pui, uout, puo, f, pf, fc, pfc, nb, items, hs, h2, inv_h2, ca,
                           partials);
      else
        hipLaunchKernelGGL((k_down_norm_s<kPeriodic>), dim3(blocks), dim3(64 * kWaves), 0, s, n,
                           uin, pui, uout, puo, f, pf, fc, pfc, nb, items, hs, h2, inv_h2, ca,
                           partials);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (bc == kDirichlet && uin)
    hipLaunchKernelGGL((k_down_s<T, kDirichlet, 1>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, fc, pfc, nb, items, hs, h2, inv_h2, ca);
  else if (bc == kDirichlet)
    hipLaunchKernelGGL((k_down_s<T, kDirichlet, 0>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, fc, pfc, nb, items, hs, h2, inv_h2, ca);
  else if (uin)
    hipLaunchKernelGGL((k_down_s<T, kPeriodic, 1>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, fc, pfc, nb, items, hs, h2, inv_h2, ca);
  else
    hipLaunchKernelGGL((k_down_s<T, kPeriodic, 0>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, fc, pfc, nb, items, hs, h2, inv_h2, ca);
  return hipGetLastError();
}

hipError_t launch_down_res_stream(hipStream_t s, int bc, int n, const double* u64, int p64,
                                  const double* f64, int pf64, float* r32, int pr, float* uout,
                                  int puo, float* fc, int pfc, int hs, const CallerArgs* ca,
                                  double* partials, int nparts, int* nitems) {
  if ((bc == kPeriodic && n - 1 < 128) || (hs > 0 && (hs & 1))) return hipErrorInvalidValue;
  const int extent = bc == kPeriodic ? n - 1 : n;
  if (hs <= 0) hs = stream_segment_rows(n, bc, kDownOwned);
  const int nb = (extent + kDownOwned - 1) / kDownOwned;
  const int items = nb * ((extent + hs - 1) / hs);
  const int blocks = (items + kWaves - 1) / kWaves;
  if (nitems) *nitems = items;
  if (partials) {
    // The norm form stores no pre-smoothed iterate and writes one partial
    // per wavefront.
    if (uout || 2 * items > nparts) return hipErrorInvalidValue;
    const double hd = 1.0 / (double)(n - 1);
    const double inv_h2d = (double)(n - 1) * (double)(n - 1);
    const float h2 = (float)(hd * hd), inv_h2 = (float)inv_h2d;
    if (bc == kDirichlet)
      hipLaunchKernelGGL((k_down_res_s<kDirichlet, false, true>), dim3(blocks), dim3(64 * kWaves),
                         0, s, n, u64, p64, f64, pf64, r32, pr, uout, puo, fc, pfc, nb, items, hs,
                         h2, inv_h2, inv_h2d, ca, partials);
    else
      hipLaunchKernelGGL((k_down_res_s<kPeriodic, false, true>), dim3(blocks), dim3(64 * kWaves),
                         0, s, n, u64, p64, f64, pf64, r32, pr, uout, puo, fc, pfc, nb, items, hs,
                         h2, inv_h2, inv_h2d, ca, partials);
    return hipGetLastError();
  }
  const double hd = 1.0 / (double)(n - 1);
  const double inv_h2d = (double)(n - 1) * (double)(n - 1);
  const float h2 = (float)(hd * hd), inv_h2 = (float)inv_h2d;
#define MG_DOWN_RES(B, SB)                                                                     \
  hipLaunchKernelGGL((k_down_res_s<B, SB>), dim3(blocks), dim3(64 * kWaves), 0, s, n, u64, p64, \
                     f64, pf64, r32, pr, uout, puo, fc, pfc, nb, items, hs, h2, inv_h2, inv_h2d, ca)
  if (bc == kDirichlet && uout) MG_DOWN_RES(kDirichlet, true);
  else if (bc == kDirichlet) MG_DOWN_RES(kDirichlet, false);
  else if (uout) MG_DOWN_RES(kPeriodic, true);
  else MG_DOWN_RES(kPeriodic, false);
#undef MG_DOWN_RES
  return hipGetLastError();
}

hipError_t launch_up_pre_stream(hipStream_t s, int bc, int n, const float* f, int pf,
                                const float* c, int pc, int hs, double* u64, int p64,
                                const CallerArgs* ca) {
  if ((bc == kPeriodic && n - 1 < 128) || (hs > 0 && (hs & 1)) || !u64)
    return hipErrorInvalidValue;
  const int extent = bc == kPeriodic ? n - 1 : n;
  if (hs <= 0) hs = stream_segment_rows(n, bc, kUpPreOwned);
  const int nb = (extent + kUpPreOwned - 1) / kUpPreOwned;
  const int items = nb * ((extent + hs - 1) / hs);
  const int blocks = (items + kWaves - 1) / kWaves;
  const double hd = 1.0 / (double)(n - 1);
  const float h2 = (float)(hd * hd);
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_up_pre_s<kDirichlet>), dim3(blocks), dim3(64 * kWaves), 0, s, n, f, pf,
                       c, pc, nb, items, hs, h2, u64, p64, ca);
  else
    hipLaunchKernelGGL((k_up_pre_s<kPeriodic>), dim3(blocks), dim3(64 * kWaves), 0, s, n, f, pf,
                       c, pc, nb, items, hs, h2, u64, p64, ca);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_up_stream(hipStream_t s, int bc, int n, const T* uin, int pui, T* uout, int puo,
                            const T* f, int pf, const T* c, int pc, int hs, double* u64,
                            int p64, const CallerArgs* ca) {
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
                       pui, uout, puo, f, pf, c, pc, nb, items, hs, h2, u64, p64, ca);
  else if (bc == kDirichlet)
    hipLaunchKernelGGL((k_up_s<T, kDirichlet, false>), dim3(blocks), dim3(64 * kWaves), 0, s, n,
                       uin, pui, uout, puo, f, pf, c, pc, nb, items, hs, h2, u64, p64, ca);
  else if (u64)
    hipLaunchKernelGGL((k_up_s<T, kPeriodic, true>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, c, pc, nb, items, hs, h2, u64, p64, ca);
  else
    hipLaunchKernelGGL((k_up_s<T, kPeriodic, false>), dim3(blocks), dim3(64 * kWaves), 0, s, n, uin,
                       pui, uout, puo, f, pf, c, pc, nb, items, hs, h2, u64, p64, ca);
  return hipGetLastError();
}

#define MG_STREAM_INSTANTIATE(T)                                                                \
  template hipError_t launch_down_stream<T>(hipStream_t, int, int, const T*, int, T*, int,      \
                                            const T*, int, T*, int, int, const CallerArgs*,      \
                                            double*, int, int*);                                 \
  template hipError_t launch_up_stream<T>(hipStream_t, int, int, const T*, int, T*, int,        \
                                          const T*, int, const T*, int, int, double*, int,      \
                                          const CallerArgs*);

MG_STREAM_INSTANTIATE(double)
MG_STREAM_INSTANTIATE(float)

hipError_t launch_residual_mixed(hipStream_t s, int bc, int n, const double* u, int pu,
                                 const double* f, int pf, float* r32, int pr, double* partials,
                                 int* nblocks, const CallerArgs* ca) {
  const double inv_h2 = (double)(n - 1) * (double)(n - 1);
  const int nb = (n + kResOwned - 1) / kResOwned;
  int hs = 64;
  while (hs > 8 && (long)nb * ((n + hs - 1) / hs) < 2048) hs -= 8;
  const int items = nb * ((n + hs - 1) / hs);
  const int blocks = (items + kWaves - 1) / kWaves;
  *nblocks = items;
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_residual_mixed_s<kDirichlet>), dim3(blocks), dim3(64 * kWaves), 0, s, n,
                       u, pu, f, pf, r32, pr, partials, nb, items, hs, inv_h2, ca);
  else
    hipLaunchKernelGGL((k_residual_mixed_s<kPeriodic>), dim3(blocks), dim3(64 * kWaves), 0, s, n,
                       u, pu, f, pf, r32, pr, partials, nb, items, hs, inv_h2, ca);
  return hipGetLastError();
}

}  // namespace mg
