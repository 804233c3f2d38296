// Pressure-projection steps around the Poisson solve on a periodic grid with
// the duplicated seam (unique nodes 0 .. N-1, N = n - 1, spacing h = 1/N, x
// along the columns):
//   * the source of the pressure-Poisson equation with zero viscosity
//     (Section 2.3, Eq. for f(x, y)): f = -div((u . grad) u);
//   * the explicit Euler step of the momentum equation (Section 2.1, first
//     line of the system): u <- u - dt ((u . grad) u + grad p).  The pressure
//     arrives as the Poisson solve returns it for that source, q = -p (the
//     solver's operator is the negative Laplacian), so the step evaluates
//     u - dt ((u . grad) u - grad q), bitwise the same as with p = -q.
// Every derivative is the central difference (a[j+1] - a[j-1]) / (2h) of the
// nodal values; 1 / (2h) = N / 2 is a power of two, so the products by it
// are exact and, with contraction off, each result is rounded exactly as
// the plain expression in the order written.
//
// Workgroups of 64 x 4 threads work on tiles of 64 columns x 16 (source) or
// 8 (update) rows.  The tile and a halo of 2 (source) or 1 (update) nodes of
// every input are staged in LDS with periodic wrap; each thread then makes
// 4 (2) rows of one column.  The source evaluates (u . grad) u at the four
// neighbours of its node from LDS, and each of its workgroups walks a
// contiguous run of tiles with the next tile's loads in flight; the update
// takes one tile per workgroup.  Tried and slower: forming (u . grad) u once
// per node in LDS behind a second barrier, and loading the tile row by row
// with the halo columns as extra masked loads.  Every XCD works through one
// contiguous run of tiles in row-major order, so the halos that neighbouring
// tiles share are hits in that XCD's L2.  Both passes are bound by HBM:
// algorithmic bytes per unique node are 3 values (source: read u_x, u_y,
// write f) and 5 values (update: read u_x, u_y, q, write both components).

#include "mg_device.h"
#include "mg_internal.h"

namespace mg {
namespace {

constexpr int kNsTX = 64, kNsTY = 4;
// Tile rows: 16 for the source (halo 2), 8 for the update (halo 1, three
// inputs), the faster of 8, 16 and 32 for each on 4097^2.
constexpr int kRowsRhs = 16, kRowsUpd = 8;
// Workgroups of the source's tile walk (16 per CU).
constexpr int kRhsGroups = 4096;

// Periodic index: more than one period away only on grids smaller than a
// tile.
__device__ __forceinline__ int ns_wrap(int i, int N) {
  while (i < 0) i += N;
  while (i >= N) i -= N;
  return i;
}

// Rows i0-H .. i0+ROWS+H-1 and columns j0-H .. j0+kNsTX+H-1 of `a`
// (wrapped) into sh (row length kNsTX + 2H), the threads running over the
// flattened tile so that every load instruction is a full wavefront of
// consecutive nodes.
template <typename T, int H, int ROWS>
__device__ __forceinline__ void ns_load_tile(const T* __restrict__ a, int pa, int N, int i0,
                                             int j0, T* __restrict__ sh) {
  constexpr int C = kNsTX + 2 * H, R = ROWS + 2 * H;
  const int t = threadIdx.y * kNsTX + threadIdx.x;
  for (int k = t; k < R * C; k += kNsTX * kNsTY) {
    const int r = k / C, c = k - r * C;
    sh[k] = a[(size_t)ns_wrap(i0 - H + r, N) * pa + ns_wrap(j0 - H + c, N)];
  }
}

// (u . grad) u at LDS position (r, c) of a tile with row length C.
template <typename T, int C>
__device__ __forceinline__ void ns_convection(const T* su, const T* sv, int r, int c, T inv2h,
                                              T* cx, T* cy) {
#pragma clang fp contract(off)
  const int k = r * C + c;
  const T u = su[k], v = sv[k];
  const T ux_x = (su[k + 1] - su[k - 1]) * inv2h, ux_y = (su[k + C] - su[k - C]) * inv2h;
  const T uy_x = (sv[k + 1] - sv[k - 1]) * inv2h, uy_y = (sv[k + C] - sv[k - C]) * inv2h;
  *cx = u * ux_x + v * ux_y;
  *cy = u * uy_x + v * uy_y;
}

// Writes node (i, j) and, on the first row / column, its seam copies.
template <typename T>
__device__ __forceinline__ void ns_store(T* a, int pa, int N, int i, int j, T val) {
  a[(size_t)i * pa + j] = val;
  if (i == 0) a[(size_t)N * pa + j] = val;
  if (j == 0) a[(size_t)i * pa + N] = val;
  if (i == 0 && j == 0) a[(size_t)N * pa + N] = val;
}

// Tile origin of this workgroup (XCD-contiguous row-major tile order).
template <int ROWS>
__device__ __forceinline__ void ns_tile(int N, int* i0, int* j0) {
  const int ntx = (N + kNsTX - 1) / kNsTX;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  *i0 = (t / ntx) * ROWS;
  *j0 = (t % ntx) * kNsTX;
}

// Registers holding one thread's share of a tile and halo (the flattened
// tile order of ns_load_tile), so that the next tile's loads are in flight
// while the current one is computed.
template <typename T, int H, int ROWS>
struct NsPrefetch {
  static constexpr int C = kNsTX + 2 * H, R = ROWS + 2 * H, E = R * C;
  static constexpr int NT = kNsTX * kNsTY, PER = (E + NT - 1) / NT;
  T v[PER];
  __device__ __forceinline__ void load(const T* __restrict__ a, int pa, int N, int i0, int j0) {
    const int t = threadIdx.y * kNsTX + threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = t + q * NT;
      if (k < E) {
        const int r = k / C, c = k - r * C;
        v[q] = a[(size_t)ns_wrap(i0 - H + r, N) * pa + ns_wrap(j0 - H + c, N)];
      }
    }
  }
  __device__ __forceinline__ void store(T* __restrict__ sh) const {
    const int t = threadIdx.y * kNsTX + threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = t + q * NT;
      if (k < E) sh[k] = v[q];
    }
  }
};

// Origin of tile t in row-major tile order.
template <int ROWS>
__device__ __forceinline__ void ns_origin(int t, int N, int* i0, int* j0) {
  const int ntx = (N + kNsTX - 1) / kNsTX;
  *i0 = (t / ntx) * ROWS;
  *j0 = (t % ntx) * kNsTX;
}

// The source walks a contiguous run of tiles per workgroup (XCD-contiguous
// runs), loading the next tile into registers while it computes the
// current one.
template <typename T>
__global__ void __launch_bounds__(kNsTX* kNsTY)
    k_ns_rhs(int N, const T* __restrict__ ux, const T* __restrict__ uy, int pu, T* __restrict__ f,
               T inv2h, int ntiles) {
#pragma clang fp contract(off)
  constexpr int H = 2, C = kNsTX + 2 * H, R = kRowsRhs + 2 * H;
  __shared__ T su[R * C], sv[R * C];
  const int w = xcd_tile(blockIdx.x, gridDim.x);
  const int tb = (int)((long long)w * ntiles / gridDim.x);
  const int te = (int)((long long)(w + 1) * ntiles / gridDim.x);
  NsPrefetch<T, H, kRowsRhs> fu, fv;
  int i0 = 0, j0 = 0;
  if (tb < te) {
    ns_origin<kRowsRhs>(tb, N, &i0, &j0);
    fu.load(ux, pu, N, i0, j0);
    fv.load(uy, pu, N, i0, j0);
  }
  for (int t = tb; t < te; ++t) {
    __syncthreads();
    fu.store(su); fv.store(sv);
    __syncthreads();
    const int ci0 = i0, cj0 = j0;
    if (t + 1 < te) {
      ns_origin<kRowsRhs>(t + 1, N, &i0, &j0);
      fu.load(ux, pu, N, i0, j0);
      fv.load(uy, pu, N, i0, j0);
    }
    const int j = cj0 + threadIdx.x, c = threadIdx.x + H;
    if (j < N) {
#pragma unroll
      for (int q = 0; q < kRowsRhs / kNsTY; ++q) {
        const int rl = threadIdx.y + q * kNsTY, i = ci0 + rl, r = rl + H;
        if (i < N) {
          T cxe, cye, cxw, cyw, cxn, cyn, cxs, cys;
          ns_convection<T, C>(su, sv, r, c + 1, inv2h, &cxe, &cye);
          ns_convection<T, C>(su, sv, r, c - 1, inv2h, &cxw, &cyw);
          ns_convection<T, C>(su, sv, r + 1, c, inv2h, &cxn, &cyn);
          ns_convection<T, C>(su, sv, r - 1, c, inv2h, &cxs, &cys);
          ns_store(f, pu, N, i, j, -((cxe - cxw) * inv2h + (cyn - cys) * inv2h));
        }
      }
    }
  }
}
template <typename T>
__global__ void __launch_bounds__(kNsTX* kNsTY)
    k_ns_update(int N, const T* __restrict__ ux, const T* __restrict__ uy,
                const T* __restrict__ q, int pu, T dt, T* __restrict__ ox, T* __restrict__ oy,
                T inv2h) {
#pragma clang fp contract(off)
  constexpr int H = 1, C = kNsTX + 2 * H, R = kRowsUpd + 2 * H;
  __shared__ T su[R * C], sv[R * C], sq[R * C];
  int i0, j0;
  ns_tile<kRowsUpd>(N, &i0, &j0);
  ns_load_tile<T, H, kRowsUpd>(ux, pu, N, i0, j0, su);
  ns_load_tile<T, H, kRowsUpd>(uy, pu, N, i0, j0, sv);
  ns_load_tile<T, H, kRowsUpd>(q, pu, N, i0, j0, sq);
  __syncthreads();
  const int j = j0 + threadIdx.x, c = threadIdx.x + H;
  if (j >= N) return;
#pragma unroll
  for (int q = 0; q < kRowsUpd / kNsTY; ++q) {
    const int rl = threadIdx.y + q * kNsTY, i = i0 + rl, r = rl + H;
    if (i >= N) break;
    T cx, cy;
    ns_convection<T, C>(su, sv, r, c, inv2h, &cx, &cy);
    const int k = r * C + c;
    // grad q = -grad p exactly, and c - g equals c + (-g) bit for bit.
    const T qx = (sq[k + 1] - sq[k - 1]) * inv2h, qy = (sq[k + C] - sq[k - C]) * inv2h;
    ns_store(ox, pu, N, i, j, su[k] - dt * (cx - qx));
    ns_store(oy, pu, N, i, j, sv[k] - dt * (cy - qy));
  }
}

dim3 ns_grid(int N, int rows) { return dim3(((N + kNsTX - 1) / kNsTX) * ((N + rows - 1) / rows)); }

}  // namespace

template <typename T>
hipError_t launch_ns_rhs(hipStream_t s, int n, const T* ux, const T* uy, T* f, int pitch) {
  const int N = n - 1;
  const int ntiles = (int)ns_grid(N, kRowsRhs).x;
  hipLaunchKernelGGL(k_ns_rhs<T>, dim3(std::min(ntiles, kRhsGroups)), dim3(kNsTX, kNsTY), 0, s, N,
                     ux, uy, pitch, f, (T)(0.5 * N), ntiles);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ns_update(hipStream_t s, int n, const T* ux, const T* uy, const T* q, double dt,
                            T* ox, T* oy, int pitch) {
  const int N = n - 1;
  hipLaunchKernelGGL(k_ns_update<T>, ns_grid(N, kRowsUpd), dim3(kNsTX, kNsTY), 0, s, N, ux, uy, q, pitch,
                     (T)dt, ox, oy, (T)(0.5 * N));
  return hipGetLastError();
}

template hipError_t launch_ns_rhs<double>(hipStream_t, int, const double*, const double*, double*,
                                          int);
template hipError_t launch_ns_rhs<float>(hipStream_t, int, const float*, const float*, float*, int);
template hipError_t launch_ns_update<double>(hipStream_t, int, const double*, const double*,
                                             const double*, double, double*, double*, int);
template hipError_t launch_ns_update<float>(hipStream_t, int, const float*, const float*,
                                            const float*, double, float*, float*, int);

}  // namespace mg
