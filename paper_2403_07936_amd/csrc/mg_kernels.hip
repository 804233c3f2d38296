// Per-operation HIP kernels for the multigrid V-cycle on gfx950.
//
// One launch per step of the cycle (Section 2.2 and the appendix's V-cycle:
// Gauss-Seidel relaxation, residual, restriction, prolongation, coarse
// solve).  These are the reference GPU path: every step is a plain, fully
// parallel stencil pass, one thread per grid node, coalesced along x
// (64-wide wavefronts map to 64 consecutive x nodes).  The fused,
// LDS-tiled kernels in mg_fused.hip implement the same arithmetic.
//
// Layout: level arrays are n x n, row-major with a pitch in elements.
// Dirichlet unknowns are 1..n-2 per direction and boundary nodes hold 0;
// periodic unknowns are 0..n-2 and index n-1 is the seam copy of 0.

#include "mg_internal.h"

namespace mg {
namespace {

constexpr int TX = 64;  // one wavefront along x
constexpr int TY = 4;   // four wavefronts per workgroup

template <int BC>
__device__ __forceinline__ int prev_node(int i, int n) {
  if constexpr (BC == kPeriodic) return i == 0 ? n - 2 : i - 1;
  return i - 1;
}
template <int BC>
__device__ __forceinline__ int next_node(int i, int n) {
  if constexpr (BC == kPeriodic) return i == n - 2 ? 0 : i + 1;
  return i + 1;
}
template <int BC>
__device__ __forceinline__ constexpr int first_unknown() {
  return BC == kDirichlet ? 1 : 0;
}
// Periodic seam node n-1 is the same node as 0.
__device__ __forceinline__ int unwrap_seam(int i, int n) { return i == n - 1 ? 0 : i; }

template <typename T>
__device__ __forceinline__ T ld(const T* a, int p, int i, int j) {
  return a[(size_t)i * p + j];
}

// Deterministic block sum of one double per thread (256 threads).
__device__ double block_sum(double v, double* sh) {
  const int t = threadIdx.y * TX + threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = TX * TY / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

// ---------------------------------------------------------------- kernels --

template <typename T>
__global__ void __launch_bounds__(TX* TY) k_zero(int n, T* a, int pa) {
  const int j = blockIdx.x * TX + threadIdx.x;
  const int i = blockIdx.y * TY + threadIdx.y;
  if (i < n && j < n) a[(size_t)i * pa + j] = T(0);
}

template <typename T>
__global__ void k_seam(int n, T* a, int pa, const CallerArgs* ca) {
  if constexpr (sizeof(T) == sizeof(double))
    if (ca) a = ca->u;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n - 1) {
    a[(size_t)t * pa + (n - 1)] = a[(size_t)t * pa];
    a[(size_t)(n - 1) * pa + t] = a[t];
  } else if (t == n - 1) {
    a[(size_t)(n - 1) * pa + (n - 1)] = a[0];
  }
}

// One red-black half-sweep: nodes with (i + j) % 2 == colour solve their row
// of A u = f with the four neighbours (all of the other colour) fixed.
template <typename T, int BC>
__global__ void __launch_bounds__(TX* TY)
    k_relax(int n, T* __restrict__ u, int pu, const T* __restrict__ f, int pf, T h2, int colour) {
  constexpr int lo = first_unknown<BC>();
  const int j = lo + blockIdx.x * TX + threadIdx.x;
  const int i = lo + blockIdx.y * TY + threadIdx.y;
  if (i > n - 2 || j > n - 2 || ((i + j) & 1) != colour) return;
  const T s = ld(u, pu, prev_node<BC>(i, n), j) + ld(u, pu, next_node<BC>(i, n), j) +
              ld(u, pu, i, prev_node<BC>(j, n)) + ld(u, pu, i, next_node<BC>(j, n));
  u[(size_t)i * pu + j] = (h2 * ld(f, pf, i, j) + s) * T(0.25);
}

template <typename T, int BC>
__device__ __forceinline__ T residual_at(int n, const T* u, int pu, const T* f, int pf, int i,
                                         int j, T inv_h2) {
  const T s = ld(u, pu, prev_node<BC>(i, n), j) + ld(u, pu, next_node<BC>(i, n), j) +
              ld(u, pu, i, prev_node<BC>(j, n)) + ld(u, pu, i, next_node<BC>(j, n));
  return ld(f, pf, i, j) - (T(4) * ld(u, pu, i, j) - s) * inv_h2;
}

// r = f - A u at every node (0 on the Dirichlet boundary, seam = node 0).
template <typename T, int BC>
__global__ void __launch_bounds__(TX* TY)
    k_residual(int n, const T* __restrict__ u, int pu, const T* __restrict__ f, int pf,
               T* __restrict__ r, int pr, T inv_h2) {
  const int j = blockIdx.x * TX + threadIdx.x;
  const int i = blockIdx.y * TY + threadIdx.y;
  if (i >= n || j >= n) return;
  T v;
  if constexpr (BC == kDirichlet) {
    v = (i == 0 || j == 0 || i == n - 1 || j == n - 1)
            ? T(0)
            : residual_at<T, BC>(n, u, pu, f, pf, i, j, inv_h2);
  } else {
    v = residual_at<T, BC>(n, u, pu, f, pf, unwrap_seam(i, n), unwrap_seam(j, n), inv_h2);
  }
  r[(size_t)i * pr + j] = v;
}

// Full weighting onto the coarse node (I, J) = fine (2I, 2J).
template <typename T, int BC>
__global__ void __launch_bounds__(TX* TY)
    k_restrict(int n, const T* __restrict__ r, int pr, T* __restrict__ fc, int pfc) {
  const int nc = (n - 1) / 2 + 1;
  const int J = blockIdx.x * TX + threadIdx.x;
  const int I = blockIdx.y * TY + threadIdx.y;
  if (I >= nc || J >= nc) return;
  T v = T(0);
  const bool boundary = BC == kDirichlet && (I == 0 || J == 0 || I == nc - 1 || J == nc - 1);
  if (!boundary) {
    const int Iu = BC == kPeriodic ? unwrap_seam(I, nc) : I;
    const int Ju = BC == kPeriodic ? unwrap_seam(J, nc) : J;
    const int i = 2 * Iu, j = 2 * Ju;
    const int im = prev_node<BC>(i, n), ip = next_node<BC>(i, n);
    const int jm = prev_node<BC>(j, n), jp = next_node<BC>(j, n);
    const T centre = ld(r, pr, i, j);
    const T edges = ld(r, pr, im, j) + ld(r, pr, ip, j) + ld(r, pr, i, jm) + ld(r, pr, i, jp);
    const T corners = ld(r, pr, im, jm) + ld(r, pr, im, jp) + ld(r, pr, ip, jm) + ld(r, pr, ip, jp);
    v = (T(4) * centre + T(2) * edges + corners) * T(0.0625);
  }
  fc[(size_t)I * pfc + J] = v;
}

// Index of the extended sequence of a level with nc nodes: periodic wraps
// over nc-1 nodes; Dirichlet is the odd extension about 0 and nc-1 (period
// 2(nc-1)), returned as a node index and a sign.
template <int BC>
__device__ __forceinline__ int ext_index(int q, int nc, int period, int* sign) {
  int r = q % period;
  if (r < 0) r += period;
  if constexpr (BC == kPeriodic) {
    *sign = 1;
    return r;
  } else {
    if (r <= nc - 1) {
      *sign = 1;
      return r;
    }
    *sign = -1;
    return period - r;
  }
}

// One axis of the B-spline prefilter c = S^-1 e with S = (1, 4, 1)/6 applied
// as a convolution with the (exact or truncated) inverse kernel over the
// extended sequence.  AXIS 0 runs along x (within a row), 1 along y.
template <typename T, int BC, int AXIS>
__global__ void __launch_bounds__(TX* TY)
    k_prefilter(int nc, PrefilterTaps taps, const T* __restrict__ e, int pe, T* __restrict__ c,
                int pc) {
  const int J = blockIdx.x * TX + threadIdx.x;
  const int I = blockIdx.y * TY + threadIdx.y;
  if (I >= nc || J >= nc) return;
  const int along = AXIS == 0 ? J : I;
  T v = T(0);
  if (!(BC == kDirichlet && (along == 0 || along == nc - 1))) {
    double acc = 0.0;
    for (int t = 0; t < taps.count; ++t) {
      int sg;
      const int q = ext_index<BC>(along + t - taps.offset, nc, taps.period, &sg);
      const T x = AXIS == 0 ? ld(e, pe, I, q) : ld(e, pe, q, J);
      acc += taps.w[t] * (double)(sg > 0 ? x : -x);
    }
    v = T(acc);
  }
  c[(size_t)I * pc + J] = v;
}

// 1-D cubic B-spline evaluation weights at fine node i from coefficients of
// the coarse level: coincident nodes use (1, 4, 1)/6 on c_{I-1..I+1},
// midpoints (1, 23, 23, 1)/48 on c_{I-1..I+2}.
template <typename T>
__device__ __forceinline__ int spline_weights(int i, int* base, T* w) {
  if ((i & 1) == 0) {
    *base = i / 2 - 1;
    w[0] = T(1.0 / 6.0);
    w[1] = T(4.0 / 6.0);
    w[2] = T(1.0 / 6.0);
    w[3] = T(0);
    return 3;
  }
  *base = (i - 1) / 2 - 1;
  w[0] = T(1.0 / 48.0);
  w[1] = T(23.0 / 48.0);
  w[2] = T(23.0 / 48.0);
  w[3] = T(1.0 / 48.0);
  return 4;
}

// u (+)= P e_c at fine nodes, with c the prefiltered coefficients of e_c.
template <typename T, int BC>
__global__ void __launch_bounds__(TX* TY)
    k_prolong(int n, T* __restrict__ u, int pu, const T* __restrict__ c, int pc, int add) {
  const int j = blockIdx.x * TX + threadIdx.x;
  const int i = blockIdx.y * TY + threadIdx.y;
  if (i >= n || j >= n) return;
  const bool boundary = BC == kDirichlet && (i == 0 || j == 0 || i == n - 1 || j == n - 1);
  const bool seam = BC == kPeriodic && (i == n - 1 || j == n - 1);
  if (add && (boundary || seam)) return;
  T v = T(0);
  if (!boundary) {
    const int nc = (n - 1) / 2 + 1;
    const int period = BC == kPeriodic ? nc - 1 : 2 * (nc - 1);
    const int iu = BC == kPeriodic ? unwrap_seam(i, n) : i;
    const int ju = BC == kPeriodic ? unwrap_seam(j, n) : j;
    int bi, bj;
    T wi[4], wj[4];
    const int ni = spline_weights<T>(iu, &bi, wi);
    const int nj = spline_weights<T>(ju, &bj, wj);
    for (int a = 0; a < ni; ++a) {
      int si;
      const int I = ext_index<BC>(bi + a, nc, period, &si);
      T row = T(0);
      for (int b = 0; b < nj; ++b) {
        int sj;
        const int J = ext_index<BC>(bj + b, nc, period, &sj);
        const T x = ld(c, pc, I, J);
        row += wj[b] * (sj > 0 ? x : -x);
      }
      v += wi[a] * (si > 0 ? row : -row);
    }
  }
  T* dst = u + (size_t)i * pu + j;
  *dst = add ? *dst + v : v;
}

// 5 x 5 level: u = inv * f on the unknowns, in FP64.  One thread per node.
template <typename T, int BC>
__global__ void k_coarse(const T* __restrict__ f, int pf, T* __restrict__ u, int pu,
                         const double* __restrict__ inv) {
  __shared__ double fv[16];
  const int t = threadIdx.x;
  constexpr int m = BC == kDirichlet ? 9 : 16;
  if (t < m) {
    const int i = BC == kDirichlet ? t / 3 + 1 : t / 4;
    const int j = BC == kDirichlet ? t % 3 + 1 : t % 4;
    fv[t] = (double)ld(f, pf, i, j);
  }
  __syncthreads();
  if (t < 25) {
    const int i = t / 5, j = t % 5;
    double v = 0.0;
    int k = -1;
    if constexpr (BC == kDirichlet) {
      if (i >= 1 && i <= 3 && j >= 1 && j <= 3) k = (i - 1) * 3 + (j - 1);
    } else {
      k = (i % 4) * 4 + (j % 4);
    }
    if (k >= 0)
      for (int q = 0; q < m; ++q) v += inv[k * m + q] * fv[q];
    u[(size_t)i * pu + j] = T(v);
  }
}

template <int BC>
__global__ void __launch_bounds__(TX* TY)
    k_update_mixed(int n, double* __restrict__ u, int pu, const float* __restrict__ e, int pe,
                   const CallerArgs* ca) {
  if (ca) u = ca->u;
  constexpr int lo = first_unknown<BC>();
  const int j = lo + blockIdx.x * TX + threadIdx.x;
  const int i = lo + blockIdx.y * TY + threadIdx.y;
  if (i > n - 2 || j > n - 2) return;
  u[(size_t)i * pu + j] += (double)e[(size_t)i * pe + j];
}

// The norm kernels give each thread kNormRows rows of one column (rows
// q * TY + threadIdx.y of the block's band), so that a workgroup's share
// outweighs its tree reduction.
constexpr int kNormRows = 8;

template <int BC>
__global__ void __launch_bounds__(TX* TY)
    k_resnorm(int n, const double* __restrict__ u, int pu, const double* __restrict__ f, int pf,
              double* __restrict__ partials, int with_f, double inv_h2) {
  __shared__ double sh[TX * TY];
  constexpr int lo = first_unknown<BC>();
  const int j = lo + blockIdx.x * TX + threadIdx.x;
  double rr = 0.0, ff = 0.0;
  if (j <= n - 2) {
    for (int q = 0; q < kNormRows; ++q) {
      const int i = lo + (blockIdx.y * kNormRows + q) * TY + threadIdx.y;
      if (i > n - 2) break;
      const double v = residual_at<double, BC>(n, u, pu, f, pf, i, j, inv_h2);
      rr += v * v;
      const double fv = ld(f, pf, i, j);
      ff += fv * fv;
    }
  }
  const int b = blockIdx.y * gridDim.x + blockIdx.x;
  const double s = block_sum(rr, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[b] = s;
  if (with_f) {
    __syncthreads();
    const double s2 = block_sum(ff, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[gridDim.x * gridDim.y + b] = s2;
  }
}

// Per-block partial sums of a (slot 0) and a^2 (slot 1) over the unknowns.
template <int BC>
__global__ void __launch_bounds__(TX* TY)
    k_moments(int n, const double* __restrict__ a, int pa, double* __restrict__ partials,
              int with_sq) {
  __shared__ double sh[TX * TY];
  constexpr int lo = first_unknown<BC>();
  const int j = lo + blockIdx.x * TX + threadIdx.x;
  double x = 0.0, x2 = 0.0;
  if (j <= n - 2) {
    for (int q = 0; q < kNormRows; ++q) {
      const int i = lo + (blockIdx.y * kNormRows + q) * TY + threadIdx.y;
      if (i > n - 2) break;
      const double v = ld(a, pa, i, j);
      x += v;
      x2 += v * v;
    }
  }
  const int b = blockIdx.y * gridDim.x + blockIdx.x;
  const double s = block_sum(x, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[b] = s;
  if (with_sq) {
    __syncthreads();
    const double s2 = block_sum(x2, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[gridDim.x * gridDim.y + b] = s2;
  }
}

// Per-block partial sums of (u - prev)^2 over the unknowns, then prev = u
// there (the change one iteration made to the iterate).
template <int BC>
__global__ void __launch_bounds__(TX* TY)
    k_diffnorm(int n, const double* __restrict__ u, int pu, double* __restrict__ prev, int pp,
               double* __restrict__ partials) {
  __shared__ double sh[TX * TY];
  constexpr int lo = first_unknown<BC>();
  const int j = lo + blockIdx.x * TX + threadIdx.x;
  const int i = lo + blockIdx.y * TY + threadIdx.y;
  double d2 = 0.0;
  if (i <= n - 2 && j <= n - 2) {
    const double v = ld(u, pu, i, j);
    const double d = v - prev[(size_t)i * pp + j];
    d2 = d * d;
    prev[(size_t)i * pp + j] = v;
  }
  const int b = blockIdx.y * gridDim.x + blockIdx.x;
  const double s = block_sum(d2, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[b] = s;
}

// Sum of `count` partials per group (group g at partials + g * stride), one
// workgroup per group.  Each thread keeps 16 accumulators over its strided
// share so that 16 loads are in flight at once; the order of every addition
// is fixed, so the result is deterministic.
constexpr int kReduceThreads = 1024;
constexpr int kReduceLanes = 16;
__global__ void __launch_bounds__(kReduceThreads)
    k_reduce(const double* __restrict__ partials, int count, int stride, double* __restrict__ out) {
  __shared__ double sh[kReduceThreads];
  const int t = threadIdx.x;
  const double* p = partials + (size_t)blockIdx.x * stride;
  double acc[kReduceLanes];
#pragma unroll
  for (int q = 0; q < kReduceLanes; ++q) acc[q] = 0.0;
  int k = t;
  for (; k + (kReduceLanes - 1) * kReduceThreads < count; k += kReduceLanes * kReduceThreads) {
#pragma unroll
    for (int q = 0; q < kReduceLanes; ++q) acc[q] += p[k + q * kReduceThreads];
  }
  for (; k < count; k += kReduceThreads) acc[0] += p[k];
#pragma unroll
  for (int w = kReduceLanes / 2; w > 0; w >>= 1)
#pragma unroll
    for (int q = 0; q < w; ++q) acc[q] += acc[q + w];
  sh[t] = acc[0];
  __syncthreads();
  for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  if (t == 0) out[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(TX* TY)
    k_remove_mean(int n, double* __restrict__ u, int pu, const double* __restrict__ sum) {
  const int j = blockIdx.x * TX + threadIdx.x;
  const int i = blockIdx.y * TY + threadIdx.y;
  if (i > n - 2 || j > n - 2) return;
  const double N = (double)(n - 1);
  u[(size_t)i * pu + j] -= sum[0] / (N * N);
}

// ---------------------------------------------------------------- helpers --

inline dim3 grid_nodes(int n) { return dim3((n + TX - 1) / TX, (n + TY - 1) / TY); }
inline int unknowns_per_side(int n, int bc) { return bc == kDirichlet ? n - 2 : n - 1; }
inline dim3 grid_unknowns(int n, int bc) {
  const int m = unknowns_per_side(n, bc);
  return dim3((m + TX - 1) / TX, (m + TY - 1) / TY);
}
const dim3 kBlock(TX, TY);
// Grid of the norm kernels: kNormRows rows per thread.
inline dim3 grid_norm(int n, int bc) {
  const dim3 g = grid_unknowns(n, bc);
  return dim3(g.x, (g.y + kNormRows - 1) / kNormRows);
}

template <typename T>
constexpr double h2_of(int n) {
  return 1.0 / ((double)(n - 1) * (double)(n - 1));
}

}  // namespace

int blocks_for(int n, int bc) {
  const dim3 g = grid_unknowns(n, bc);
  return (int)(g.x * g.y);
}

template <typename T>
hipError_t launch_zero(hipStream_t s, int n, T* a, int pa) {
  hipLaunchKernelGGL(k_zero<T>, grid_nodes(n), kBlock, 0, s, n, a, pa);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_seam(hipStream_t s, int n, T* a, int pa, const CallerArgs* ca) {
  hipLaunchKernelGGL(k_seam<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, a, pa, ca);
  return hipGetLastError();
}

namespace {
__global__ void k_bind_caller(CallerArgs* slot, double* u, const double* f) {
  slot->u = u;
  slot->f = f;
}
}  // namespace

hipError_t launch_bind_caller(hipStream_t s, CallerArgs* slot, double* u, const double* f) {
  hipLaunchKernelGGL(k_bind_caller, dim3(1), dim3(1), 0, s, slot, u, f);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_relax(hipStream_t s, int bc, int n, T* u, int pu, const T* f, int pf, int colour,
                        int count) {
  const T h2 = T(h2_of<T>(n));
  const dim3 g = grid_unknowns(n, bc);
  for (int k = 0; k < count; ++k) {
    const int c = (colour + k) & 1;
    if (bc == kDirichlet)
      hipLaunchKernelGGL((k_relax<T, kDirichlet>), g, kBlock, 0, s, n, u, pu, f, pf, h2, c);
    else
      hipLaunchKernelGGL((k_relax<T, kPeriodic>), g, kBlock, 0, s, n, u, pu, f, pf, h2, c);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(hipStream_t s, int bc, int n, const T* u, int pu, const T* f, int pf,
                           T* r, int pr) {
  const T inv_h2 = T((double)(n - 1) * (double)(n - 1));
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_residual<T, kDirichlet>), grid_nodes(n), kBlock, 0, s, n, u, pu, f, pf,
                       r, pr, inv_h2);
  else
    hipLaunchKernelGGL((k_residual<T, kPeriodic>), grid_nodes(n), kBlock, 0, s, n, u, pu, f, pf, r,
                       pr, inv_h2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(hipStream_t s, int bc, int n, const T* r, int pr, T* fc, int pfc) {
  const int nc = (n - 1) / 2 + 1;
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_restrict<T, kDirichlet>), grid_nodes(nc), kBlock, 0, s, n, r, pr, fc,
                       pfc);
  else
    hipLaunchKernelGGL((k_restrict<T, kPeriodic>), grid_nodes(nc), kBlock, 0, s, n, r, pr, fc, pfc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prefilter(hipStream_t s, int bc, int nc, const PrefilterTaps& taps, const T* e,
                            int pe, T* tmp, int pt, T* c, int pc) {
  const dim3 g = grid_nodes(nc);
  if (bc == kDirichlet) {
    hipLaunchKernelGGL((k_prefilter<T, kDirichlet, 0>), g, kBlock, 0, s, nc, taps, e, pe, tmp, pt);
    hipLaunchKernelGGL((k_prefilter<T, kDirichlet, 1>), g, kBlock, 0, s, nc, taps, tmp, pt, c, pc);
  } else {
    hipLaunchKernelGGL((k_prefilter<T, kPeriodic, 0>), g, kBlock, 0, s, nc, taps, e, pe, tmp, pt);
    hipLaunchKernelGGL((k_prefilter<T, kPeriodic, 1>), g, kBlock, 0, s, nc, taps, tmp, pt, c, pc);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(hipStream_t s, int bc, int n, T* u, int pu, const T* c, int pc,
                          bool add) {
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_prolong<T, kDirichlet>), grid_nodes(n), kBlock, 0, s, n, u, pu, c, pc,
                       (int)add);
  else
    hipLaunchKernelGGL((k_prolong<T, kPeriodic>), grid_nodes(n), kBlock, 0, s, n, u, pu, c, pc,
                       (int)add);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse(hipStream_t s, int bc, const T* f, int pf, T* u, int pu,
                         const double* inv) {
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_coarse<T, kDirichlet>), dim3(1), dim3(64), 0, s, f, pf, u, pu, inv);
  else
    hipLaunchKernelGGL((k_coarse<T, kPeriodic>), dim3(1), dim3(64), 0, s, f, pf, u, pu, inv);
  return hipGetLastError();
}

hipError_t launch_update_mixed(hipStream_t s, int bc, int n, double* u, int pu, const float* e,
                               int pe, const CallerArgs* ca) {
  const dim3 g = grid_unknowns(n, bc);
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_update_mixed<kDirichlet>), g, kBlock, 0, s, n, u, pu, e, pe, ca);
  else
    hipLaunchKernelGGL((k_update_mixed<kPeriodic>), g, kBlock, 0, s, n, u, pu, e, pe, ca);
  return hipGetLastError();
}

hipError_t launch_resnorm(hipStream_t s, int bc, int n, const double* u, int pu, const double* f,
                          int pf, double* partials, bool with_f, int* nblocks) {
  const double inv_h2 = (double)(n - 1) * (double)(n - 1);
  const dim3 g = grid_norm(n, bc);
  *nblocks = (int)(g.x * g.y);
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_resnorm<kDirichlet>), g, kBlock, 0, s, n, u, pu, f, pf, partials,
                       (int)with_f, inv_h2);
  else
    hipLaunchKernelGGL((k_resnorm<kPeriodic>), g, kBlock, 0, s, n, u, pu, f, pf, partials,
                       (int)with_f, inv_h2);
  return hipGetLastError();
}

hipError_t launch_rhs_moments(hipStream_t s, int bc, int n, const double* f, int pf,
                              double* partials, int* nblocks) {
  const dim3 g = grid_norm(n, bc);
  *nblocks = (int)(g.x * g.y);
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_moments<kDirichlet>), g, kBlock, 0, s, n, f, pf, partials, 1);
  else
    hipLaunchKernelGGL((k_moments<kPeriodic>), g, kBlock, 0, s, n, f, pf, partials, 1);
  return hipGetLastError();
}

hipError_t launch_sum(hipStream_t s, int bc, int n, const double* a, int pa, double* partials,
                      int* nblocks) {
  const dim3 g = grid_norm(n, bc);
  *nblocks = (int)(g.x * g.y);
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_moments<kDirichlet>), g, kBlock, 0, s, n, a, pa, partials, 0);
  else
    hipLaunchKernelGGL((k_moments<kPeriodic>), g, kBlock, 0, s, n, a, pa, partials, 0);
  return hipGetLastError();
}

hipError_t launch_diffnorm(hipStream_t s, int bc, int n, const double* u, int pu, double* prev,
                           int pp, double* partials, int* nblocks) {
  const dim3 g = grid_unknowns(n, bc);
  *nblocks = (int)(g.x * g.y);
  if (bc == kDirichlet)
    hipLaunchKernelGGL((k_diffnorm<kDirichlet>), g, kBlock, 0, s, n, u, pu, prev, pp, partials);
  else
    hipLaunchKernelGGL((k_diffnorm<kPeriodic>), g, kBlock, 0, s, n, u, pu, prev, pp, partials);
  return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t s, const double* partials, int count, int stride, int groups,
                         double* out) {
  hipLaunchKernelGGL(k_reduce, dim3(groups), dim3(kReduceThreads), 0, s, partials, count, stride,
                     out);
  return hipGetLastError();
}

hipError_t launch_remove_mean(hipStream_t s, int n, double* u, int pu, const double* sum) {
  hipLaunchKernelGGL(k_remove_mean, grid_unknowns(n, kPeriodic), kBlock, 0, s, n, u, pu, sum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_seam<double>(s, n, u, pu);
}

#define MG_INSTANTIATE(T)                                                                        \
  template hipError_t launch_zero<T>(hipStream_t, int, T*, int);                                 \
  template hipError_t launch_seam<T>(hipStream_t, int, T*, int, const CallerArgs*);              \
  template hipError_t launch_relax<T>(hipStream_t, int, int, T*, int, const T*, int, int, int);  \
  template hipError_t launch_residual<T>(hipStream_t, int, int, const T*, int, const T*, int, T*, \
                                         int);                                                   \
  template hipError_t launch_restrict<T>(hipStream_t, int, int, const T*, int, T*, int);         \
  template hipError_t launch_prefilter<T>(hipStream_t, int, int, const PrefilterTaps&, const T*, \
                                          int, T*, int, T*, int);                                \
  template hipError_t launch_prolong<T>(hipStream_t, int, int, T*, int, const T*, int, bool);    \
  template hipError_t launch_coarse<T>(hipStream_t, int, const T*, int, T*, int, const double*);

MG_INSTANTIATE(double)
MG_INSTANTIATE(float)

}  // namespace mg
