// Persistent cycle kernel: one launch runs a whole step (for the mixed path:
// FP64 residual, the FP32 V-cycle, FP64 update) for every problem of a batch.
//
// The host flattens the step into phases (mg_batch.hip): a phase is a list
// of items of one kind, and every item of a phase is independent of the
// others.  Phases are aligned from the coarsest level, so the tails of all
// problems fall in one phase whatever their sizes.  Workgroups take items
// round-robin (wavefront items by global wavefront index, tail items by
// workgroup index) and meet at a device-wide barrier between phases.  The
// grid is at most the number of co-resident workgroups; the barrier spins a
// bounded number of times, and on timeout sets an error flag and every
// workgroup leaves, so the kernel always ends.

#include "mg_stream_dev.h"
#include "mg_tail_dev.h"

namespace mg {
namespace {

using namespace stream;
using namespace dev;

constexpr int kWavesPerBlock = kPersistThreads / 64;
constexpr long kSpinLimit = 1L << 24;  // ~1 s of s_sleep: far longer than any phase

// Sense-reversing device-wide barrier.  Returns false (and every later call
// returns false) once any workgroup has timed out.
__device__ bool grid_barrier(PBarrier* bar, unsigned* gen_local) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = 1;
    __threadfence();
    const unsigned g = *gen_local;
    if (atomicAdd(&bar->count, 1u) == gridDim.x - 1) {
      atomicExch(&bar->count, 0u);
      __threadfence();
      atomicAdd(&bar->gen, 1u);
    } else {
      long k = 0;
      while (__hip_atomic_load(&bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(&bar->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
            ++k > kSpinLimit) {
          atomicOr(&bar->error, 1u);
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    *gen_local = g + 1;
    __threadfence();
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// u64 += e on the unknowns of rows [r0, r0 + kRowsPerItem).
template <int BC>
__device__ __forceinline__ void upd_rows(const PProblem& p, int r0, int lane) {
  const int n = p.lv[0].n, pu = p.pitch64, pe = p.lv[0].pitch_u;
  const float* e = static_cast<const float*>(p.lv[0].u);
  const int lo = BC == kDirichlet ? 1 : 0;
  for (int i = r0 < lo ? lo : r0; i < r0 + kRowsPerItem && i <= n - 2; ++i)
    for (int j = lo + lane; j <= n - 2; j += 64)
      p.u64[(size_t)i * pu + j] += (double)e[(size_t)i * pe + j];
}

// The items of one phase of kind KIND: workgroup items (tails, prefilter
// tiles) by workgroup index, wavefront items by global wavefront index,
// both striding by the grid.  sm: dynamic LDS (workgroup items only).
template <typename T, int BC, int KIND>
__device__ __forceinline__ void run_phase(const PProblem* __restrict__ probs, const PPhase& P,
                                          const PItem* __restrict__ items,
                                          const double* __restrict__ inv, T* sm) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // Consecutive items (neighbouring bands, then segments, of one level) go
  // to workgroups of one XCD, so the rows and columns they share come from
  // that XCD's L2 (xcd_tile permutes the workgroups).
  const int wg = xcd_tile(blockIdx.x, gridDim.x);
  const int gwave = wave_uniform(wg * kWavesPerBlock + wave);
  const int nwaves = gridDim.x * kWavesPerBlock;
  if constexpr (KIND == kItemTail) {
    for (int i = wg; i < P.count; i += gridDim.x) {
      const PItem it = items[P.first + i];
      const PProblem& p = probs[it.prob];
      if (!p.active) continue;
      const int t = it.level;
      const PLevel& L = p.lv[t];
      const bool top = t == 0;
      const T* uin = (top && !p.zero_guess) ? static_cast<const T*>(L.u) : nullptr;
      tail_block<T, BC, kPersistThreads / 32>(
          L.n, uin, L.pitch_u, top ? static_cast<T*>(L.u) : nullptr, L.pitch_u,
          static_cast<const T*>(L.f), L.pitch_f, top ? nullptr : static_cast<T*>(L.c), L.pitch,
          inv, sm);
      __syncthreads();
    }
  } else if constexpr (KIND == kItemPre) {
    for (int i = wg; i < P.count; i += gridDim.x) {
      const PItem it = items[P.first + i];
      const PProblem& p = probs[it.prob];
      if (!p.active) continue;
      const PLevel& L = p.lv[it.level];
      pre_tile_block<T, BC, kPersistThreads>(L.n, static_cast<const T*>(L.u), L.pitch_u,
                                             static_cast<T*>(L.c), L.pitch, it.a, it.b, sm);
      __syncthreads();
    }
  } else {
    for (int i = gwave; i < P.count; i += nwaves) {
      const PItem it = items[P.first + i];
      const PProblem& p = probs[it.prob];
      if (!p.active) continue;
      const PLevel& L = p.lv[it.level];
      if constexpr (KIND == kItemRes) {
        (void)residual_wave<BC>(L.n, p.u64, p.pitch64, p.f64, p.pitch64,
                                static_cast<float*>(L.f), L.pitch_f, it.a, it.b, kResSegRows,
                                (double)(L.n - 1) * (double)(L.n - 1), lane);
      } else if constexpr (KIND == kItemUpd) {
        upd_rows<BC>(p, it.a, lane);
      } else if constexpr (KIND == kItemDown) {
        const PLevel& C = p.lv[it.level + 1];
        const double hd = 1.0 / (double)(L.n - 1);
        // Mixed path, level 0 (from e = 0): the pass makes its FP32
        // right-hand side from the FP64 iterate itself and stores it for the
        // up pass, and stores no pre-smoothed iterate (the up pass makes it
        // again), as in the per-problem schedule.
        // Its sum of r^2 (the convergence check of the iterate the step
        // starts from) goes to the problem's partials, lanes reduced in a
        // fixed order.
        if constexpr (sizeof(T) == sizeof(float)) {
          if (it.level == 0 && p.zero_guess) {
            const double inv_h2d = (double)(L.n - 1) * (double)(L.n - 1);
            double2 q = down_wave<float, BC, 0, true, false, 1>(
                L.n, nullptr, 0, nullptr, 0, nullptr, 0, static_cast<float*>(C.f), C.pitch_f,
                it.a, it.b, L.hs_down, float(hd * hd), float(inv_h2d), lane, p.u64, p.pitch64,
                p.f64, p.pitch64, inv_h2d, static_cast<float*>(L.f), L.pitch_f);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) q.x += __shfl_down(q.x, off);
            if (lane == 0 && p.npart) p.npart[P.first + i - p.nfirst] = q.x;
            continue;
          }
        }
        const T* uin = (it.level == 0 && !p.zero_guess) ? static_cast<const T*>(L.u) : nullptr;
        down_wave<T, BC>(L.n, uin, L.pitch_u, static_cast<T*>(L.b), L.pitch,
                         static_cast<const T*>(L.f), L.pitch_f, static_cast<T*>(C.f), C.pitch_f,
                         it.a, it.b, L.hs_down, T(hd * hd),
                         T((double)(L.n - 1) * (double)(L.n - 1)), lane);
      } else if constexpr (KIND == kItemUp) {
        const PLevel& C = p.lv[it.level + 1];
        const double hd = 1.0 / (double)(L.n - 1);
        // Mixed path, level 0: the pre-smoothed iterate is made again from
        // the stored right-hand side and the finished rows go straight into
        // the FP64 iterate (the refinement update), as in the per-problem
        // schedule.
        if constexpr (sizeof(T) == sizeof(float)) {
          if (it.level == 0 && p.zero_guess) {
            up_pre_wave<BC>(L.n, static_cast<const float*>(L.f), L.pitch_f,
                            static_cast<const float*>(C.c), C.pitch, it.a, it.b, L.hs_up,
                            float(hd * hd), lane, p.u64, p.pitch64);
            continue;
          }
        }
        up_wave<T, BC>(L.n, static_cast<const T*>(L.b), L.pitch, static_cast<T*>(L.u),
                       L.pitch_u, static_cast<const T*>(L.f), L.pitch_f,
                       static_cast<const T*>(C.c), C.pitch, it.a, it.b, L.hs_up, T(hd * hd),
                       lane);
      }
    }
  }
}

template <typename T, int BC>
__global__ void __launch_bounds__(kPersistThreads)
    k_persistent(const PProblem* __restrict__ probs, const PPhase* __restrict__ phases,
                 int ph_begin, int ph_end, const PItem* __restrict__ items, PBarrier* bar,
                 const double* __restrict__ inv) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  __shared__ unsigned gen_local;
  if (threadIdx.x == 0)
    gen_local = __hip_atomic_load(&bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (__hip_atomic_load(&bar->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  for (int ph = ph_begin; ph < ph_end; ++ph) {
    const PPhase P = phases[ph];
    switch (P.kind) {
      case kItemTail: run_phase<T, BC, kItemTail>(probs, P, items, inv, sm); break;
      case kItemPre: run_phase<T, BC, kItemPre>(probs, P, items, inv, sm); break;
      case kItemRes: run_phase<T, BC, kItemRes>(probs, P, items, inv, sm); break;
      case kItemUpd: run_phase<T, BC, kItemUpd>(probs, P, items, inv, sm); break;
      case kItemDown: run_phase<T, BC, kItemDown>(probs, P, items, inv, sm); break;
      case kItemUp: run_phase<T, BC, kItemUp>(probs, P, items, inv, sm); break;
      default: break;
    }
    if (ph + 1 < ph_end && !grid_barrier(bar, &gen_local)) return;
  }
}

// One phase per launch (the kernel boundary orders the phases): the kernel
// holds only its kind's code, so its registers, and its LDS (none for
// wavefront items), are those of that kind alone.
template <typename T, int BC, int KIND>
__global__ void __launch_bounds__(kPersistThreads)
    k_phase(const PProblem* __restrict__ probs, PPhase P, const PItem* __restrict__ items,
            const double* __restrict__ inv) {
  // The phase record comes as an argument: a wavefront's first loads are
  // then its item and its problem's fields, one dependent load fewer.
  extern __shared__ __align__(16) unsigned char smem_raw[];
  run_phase<T, BC, KIND>(probs, P, items, inv, reinterpret_cast<T*>(smem_raw));
}

__global__ void k_resnorm_batched(int bc, const PProblem* __restrict__ probs, double* partials,
                                  int slots) {
  // Workgroup (256 threads) = (problem, slot): the unknowns of a run of
  // consecutive rows; a thread walks its columns j, j + 256, ... down the
  // run with the rows above and below its node in registers, so each row of
  // u is read once per column (plus its two neighbours in the row, which
  // the neighbouring lanes' reads bring into L1).
  __shared__ double sr[256], sf[256];
  const int pi = blockIdx.y, slot = blockIdx.x, t = threadIdx.x;
  const PProblem& p = probs[pi];
  double rr = 0.0, ff = 0.0;
  {
    const int n = p.lv[0].n, pu = p.pitch64;
    const double* u = p.u64;
    const double* f = p.f64;
    const double inv_h2 = (double)(n - 1) * (double)(n - 1);
    const int lo = bc == kDirichlet ? 1 : 0, hi = n - 2, N = n - 1;
    const int rows = hi - lo + 1, run = (rows + slots - 1) / slots;
    const int r0 = lo + slot * run, r1 = min(r0 + run, hi + 1);
    auto row_of = [&](int i) { return bc == kPeriodic ? (i < 0 ? i + N : (i >= N ? i - N : i)) : i; };
    for (int j = lo + t; j <= hi; j += 256) {
      const int jm = bc == kPeriodic && j == 0 ? N - 1 : j - 1;
      const int jp = bc == kPeriodic && j == N - 1 ? 0 : j + 1;
      if (r0 >= r1) break;
      double um = u[(size_t)row_of(r0 - 1) * pu + j], uc = u[(size_t)r0 * pu + j];
#pragma unroll 4
      for (int i = r0; i < r1; ++i) {
        const double up = u[(size_t)row_of(i + 1) * pu + j];
        const double* ui = u + (size_t)i * pu;
        const double s = ((um + up) + ui[jm]) + ui[jp];
        const double fv = f[(size_t)i * pu + j];
        const double r = fv - (4.0 * uc - s) * inv_h2;
        rr += r * r;
        ff += fv * fv;
        um = uc;
        uc = up;
      }
    }
  }
  sr[t] = rr;
  sf[t] = ff;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (t < s2) {
      sr[t] += sr[t + s2];
      sf[t] += sf[t + s2];
    }
    __syncthreads();
  }
  if (t == 0) {
    partials[((size_t)pi * slots + slot) * 2] = sr[0];
    partials[((size_t)pi * slots + slot) * 2 + 1] = sf[0];
  }
}

// One wavefront per problem: the sums its level-0 down items wrote, each
// lane over items lane, lane + 64, ..., then across the lanes.
__global__ void k_reduce_norms(const PProblem* __restrict__ probs, int nprob, double* sums) {
  const int b = blockIdx.x, lane = threadIdx.x;
  if (b >= nprob) return;
  const PProblem& p = probs[b];
  double a = 0.0;
  for (int j = lane; j < p.ncount; j += 64) a += p.npart[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off);
  if (lane == 0) sums[b] = a;
}

// Workgroup (256 threads) = (problem, slot): sums of a and a^2 over the
// unknowns of rows slot, slot + slots, ... of the problem's right-hand side
// (use_u = 0) or iterate (use_u = 1); zeros for inactive problems.
__global__ void k_moments_batched(const PProblem* __restrict__ probs, double* partials,
                                  int slots, int use_u) {
  __shared__ double sa[256], sb[256];
  const int pi = blockIdx.y, slot = blockIdx.x, t = threadIdx.x;
  const PProblem& p = probs[pi];
  double x = 0.0, x2 = 0.0;
  if (p.active) {
    const int n = p.lv[0].n, pf = p.pitch64;
    const double* f = use_u ? p.u64 : p.f64;
    const int lo = p.bc == kDirichlet ? 1 : 0;
    for (int i = lo + slot; i <= n - 2; i += slots)
      for (int j = lo + t; j <= n - 2; j += 256) {
        const double v = f[(size_t)i * pf + j];
        x += v;
        x2 += v * v;
      }
  }
  sa[t] = x;
  sb[t] = x2;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (t < s2) {
      sa[t] += sa[t + s2];
      sb[t] += sb[t + s2];
    }
    __syncthreads();
  }
  if (t == 0) {
    partials[((size_t)pi * slots + slot) * 2] = sa[0];
    partials[((size_t)pi * slots + slot) * 2 + 1] = sb[0];
  }
}

__global__ void k_reduce_problem(const double* __restrict__ partials, int slots, int nprob,
                                 double* sums) {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= nprob) return;
  double rr = 0.0, ff = 0.0;
  for (int s = 0; s < slots; ++s) {
    rr += partials[((size_t)pi * slots + s) * 2];
    ff += partials[((size_t)pi * slots + s) * 2 + 1];
  }
  sums[2 * pi] = rr;
  sums[2 * pi + 1] = ff;
}

// Periodic problems that are active: u -= sum(u) / N^2 on the unknowns
// (sums[2 b] = the sum), rows blockIdx.x, blockIdx.x + gridDim.x, ...
__global__ void k_remove_mean_batched(const PProblem* __restrict__ probs,
                                      const double* __restrict__ sums) {
  const PProblem& p = probs[blockIdx.y];
  if (p.bc != kPeriodic || !p.active) return;
  const int n = p.lv[0].n, N = n - 1, pu = p.pitch64;
  const double mean = sums[2 * blockIdx.y] / ((double)N * (double)N);
  double* u = p.u64;
  for (int i = blockIdx.x; i < N; i += gridDim.x)
    for (int j = threadIdx.x; j < N; j += blockDim.x) u[(size_t)i * pu + j] -= mean;
}

__global__ void k_seam_batched(const PProblem* __restrict__ probs) {
  const PProblem& p = probs[blockIdx.x];
  if (p.bc != kPeriodic) return;
  const int n = p.lv[0].n, pu = p.pitch64;
  double* u = p.u64;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    if (t < n - 1) {
      u[(size_t)t * pu + (n - 1)] = u[(size_t)t * pu];
      u[(size_t)(n - 1) * pu + t] = u[t];
    } else {
      u[(size_t)(n - 1) * pu + (n - 1)] = u[0];
    }
  }
}

}  // namespace

hipError_t persistent_init(size_t lds64, size_t lds32) {
  hipError_t e;
  e = hipFuncSetAttribute((const void*)k_persistent<double, kDirichlet>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds64);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_persistent<double, kPeriodic>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds64);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_persistent<float, kDirichlet>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds32);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_persistent<float, kPeriodic>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds32);
  if (e != hipSuccess) return e;
  const void* fns64[] = {(const void*)k_phase<double, kDirichlet, kItemTail>,
                         (const void*)k_phase<double, kPeriodic, kItemTail>,
                         (const void*)k_phase<double, kDirichlet, kItemPre>,
                         (const void*)k_phase<double, kPeriodic, kItemPre>};
  const void* fns32[] = {(const void*)k_phase<float, kDirichlet, kItemTail>,
                         (const void*)k_phase<float, kPeriodic, kItemTail>,
                         (const void*)k_phase<float, kDirichlet, kItemPre>,
                         (const void*)k_phase<float, kPeriodic, kItemPre>};
  for (const void* fn : fns64) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds64);
    if (e != hipSuccess) return e;
  }
  for (const void* fn : fns32) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds32);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t persistent_blocks(int bc, size_t lds, int* blocks) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const void* fn = bc == kDirichlet ? (const void*)k_persistent<T, kDirichlet>
                                    : (const void*)k_persistent<T, kPeriodic>;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kPersistThreads, lds);
  if (e != hipSuccess) return e;
  *blocks = cus * (per > 0 ? per : 0);
  return hipSuccess;
}

template <typename T>
hipError_t launch_persistent(hipStream_t s, int bc, const PProblem* probs, const PPhase* phases,
                             int ph_begin, int ph_end, const PItem* items, PBarrier* bar,
                             const double* inv, int blocks, size_t lds) {
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_persistent<T, kDirichlet>), dim3(blocks), dim3(kPersistThreads), lds, s,
                       probs, phases, ph_begin, ph_end, items, bar, inv);
  else
    hipLaunchKernelGGL((k_persistent<T, kPeriodic>), dim3(blocks), dim3(kPersistThreads), lds, s,
                       probs, phases, ph_begin, ph_end, items, bar, inv);
  return hipGetLastError();
}

hipError_t launch_reduce_norms(hipStream_t s, const PProblem* probs, int nprob, double* sums) {
  hipLaunchKernelGGL(k_reduce_norms, dim3(nprob), dim3(64), 0, s, probs, nprob, sums);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_phase(hipStream_t s, int bc, const PPhase& phase, const PProblem* probs,
                        const PItem* items, const double* inv, int blocks, size_t lds) {
  const int kind = phase.kind;
#define MG_PHASE(B, K)                                                                          \
  hipLaunchKernelGGL((k_phase<T, B, K>), dim3(blocks), dim3(kPersistThreads), lds, s, probs,     \
                     phase, items, inv)
#define MG_PHASE_BC(K)          \
  if (bc == kDirichlet)         \
    MG_PHASE(kDirichlet, K);    \
  else                          \
    MG_PHASE(kPeriodic, K)
  switch (kind) {
    case kItemTail: MG_PHASE_BC(kItemTail); break;
    case kItemPre: MG_PHASE_BC(kItemPre); break;
    case kItemRes: MG_PHASE_BC(kItemRes); break;
    case kItemUpd: MG_PHASE_BC(kItemUpd); break;
    case kItemDown: MG_PHASE_BC(kItemDown); break;
    case kItemUp: MG_PHASE_BC(kItemUp); break;
    default: return hipErrorInvalidValue;
  }
#undef MG_PHASE_BC
#undef MG_PHASE
  return hipGetLastError();
}

hipError_t launch_resnorm_batched(hipStream_t s, int bc, const PProblem* probs, int nprob,
                                  double* partials, int slots, double* sums) {
  hipLaunchKernelGGL(k_resnorm_batched, dim3(slots, nprob), dim3(256), 0, s, bc, probs, partials,
                     slots);
  hipLaunchKernelGGL(k_reduce_problem, dim3((nprob + 63) / 64), dim3(64), 0, s, partials, slots,
                     nprob, sums);
  return hipGetLastError();
}

hipError_t launch_moments_batched(hipStream_t s, const PProblem* probs, int nprob,
                                  double* partials, int slots, double* sums, bool use_u) {
  hipLaunchKernelGGL(k_moments_batched, dim3(slots, nprob), dim3(256), 0, s, probs, partials,
                     slots, (int)use_u);
  hipLaunchKernelGGL(k_reduce_problem, dim3((nprob + 63) / 64), dim3(64), 0, s, partials, slots,
                     nprob, sums);
  return hipGetLastError();
}

hipError_t launch_remove_mean_batched(hipStream_t s, const PProblem* probs, int nprob,
                                      const double* sums) {
  hipLaunchKernelGGL(k_remove_mean_batched, dim3(32, nprob), dim3(256), 0, s, probs, sums);
  return launch_seam_batched(s, probs, nprob);
}

hipError_t launch_seam_batched(hipStream_t s, const PProblem* probs, int nprob) {
  hipLaunchKernelGGL(k_seam_batched, dim3(nprob), dim3(256), 0, s, probs);
  return hipGetLastError();
}

template hipError_t launch_persistent<double>(hipStream_t, int, const PProblem*, const PPhase*,
                                              int, int, const PItem*, PBarrier*, const double*,
                                              int, size_t);
template hipError_t launch_persistent<float>(hipStream_t, int, const PProblem*, const PPhase*, int,
                                             int, const PItem*, PBarrier*, const double*, int,
                                             size_t);
template <typename T>
hipError_t phase_wave_slots(int bc, int kind, long* slots) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const bool d = bc == kDirichlet;
  const void* fn = nullptr;
  if (kind == kItemDown)
    fn = d ? (const void*)k_phase<T, kDirichlet, kItemDown> : (const void*)k_phase<T, kPeriodic, kItemDown>;
  else if (kind == kItemUp)
    fn = d ? (const void*)k_phase<T, kDirichlet, kItemUp> : (const void*)k_phase<T, kPeriodic, kItemUp>;
  else
    return hipErrorInvalidValue;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kPersistThreads, 0);
  if (e != hipSuccess) return e;
  *slots = (long)per * kWavesPerBlock * cus;
  return hipSuccess;
}
template hipError_t phase_wave_slots<double>(int, int, long*);
template hipError_t phase_wave_slots<float>(int, int, long*);

template hipError_t launch_phase<double>(hipStream_t, int, const PPhase&, const PProblem*,
                                         const PItem*, const double*, int, size_t);
template hipError_t launch_phase<float>(hipStream_t, int, const PPhase&, const PProblem*,
                                        const PItem*, const double*, int, size_t);
template hipError_t persistent_blocks<double>(int, size_t, int*);
template hipError_t persistent_blocks<float>(int, size_t, int*);

}  // namespace mg
