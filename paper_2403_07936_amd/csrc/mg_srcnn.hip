// Super-resolution CNN prolongation (Section 3.1; the SR-Prolongation of the
// appendix, generator after Ledig et al.): coarse correction e_c on the N x N
// unique nodes of a periodic level -> fine correction on 2N x 2N.
//
//   s = max|e_c|;  x = bf16(e_c / s)
//   h = bf16(relu(conv_stem(x)))                          1 -> 64
//   8 x { t = bf16(relu(conv1(h)));  h = bf16(h + conv2(t)) }   64 -> 64
//   z = bf16(relu(shuffle2(conv_up(h))))                  64 -> 256 -> 64 @ 2N
//   u_fine (+)= s * conv_fin(z)                           64 -> 1
//
// All convolutions are 3x3 cross-correlations with circular padding and no
// bias.  Activations are bf16 in NHWC order (64 channels = 128 bytes per
// pixel); the 64-channel convolutions are implicit GEMMs on the bf16 matrix
// cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation): M = output channels,
// N = pixels, K = 9 taps x 64 input channels, with the weights and a
// (8+2) x (32+2)-pixel input tile staged in LDS.

#include "mg_internal.h"

namespace mg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kC = 64;            // channels
constexpr int kTH = 8;            // output rows per tile
constexpr int kTW = 32;           // output columns per tile
constexpr int kHW = kTW + 2;      // tile width with halo
constexpr int kTileChunks = (kTH + 2) * kHW * 8;  // 16-byte chunks of the input tile
constexpr int kWChunks = 9 * kC * 8;              // 16-byte chunks of one 64x64 weight set
constexpr int kConvThreads = 256;
constexpr int kPartials = 256;    // blocks of the max-abs pass

__device__ __forceinline__ unsigned short to_bf16(float x) {
  return __builtin_bit_cast(unsigned short, (__bf16)x);
}
__device__ __forceinline__ float from_bf16(unsigned short b) {
  return __builtin_bit_cast(float, (unsigned)b << 16);
}

// Bank-conflict-free placement of 16-byte chunk c (0..7) of row r: the
// eight chunks of eight consecutive rows land in distinct bank groups.
__device__ __forceinline__ int swz(int r, int c) { return r * 8 + (c ^ (r & 7)); }

// ---------------------------------------------------------------- max |e|
template <typename T>
__global__ void __launch_bounds__(256) k_cnn_absmax(int N, const T* __restrict__ e, int pe,
                                                    float* __restrict__ partials) {
  __shared__ float red[256];
  float m = 0.f;
  const long total = (long)N * N;
  for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < total; q += (long)gridDim.x * 256) {
    const int y = (int)(q / N), x = (int)(q % N);
    m = fmaxf(m, fabsf((float)e[(long)y * pe + x]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// Block-wide max of the partials (every thread gets it).
__device__ float block_scale(const float* __restrict__ partials, float* red) {
  red[threadIdx.x] = partials[threadIdx.x];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const float s = red[0];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- stem
// Thread = (pixel, group of 8 output channels).  stem_w: [64][9] floats.
template <typename T>
__global__ void __launch_bounds__(256)
    k_cnn_stem(int N, const T* __restrict__ e, int pe, const float* __restrict__ partials,
               const float* __restrict__ stem_w, unsigned short* __restrict__ h,
               float* __restrict__ scale_out) {
  __shared__ float red[256];
  const float s = block_scale(partials, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) scale_out[0] = s;
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  if (q >= (long)N * N * 8) return;
  const int g = (int)(q & 7);
  const long pix = q >> 3;
  const int y = (int)(pix / N), x = (int)(pix % N);
  float xv[9];
  for (int dy = 0; dy < 3; ++dy)
    for (int dx = 0; dx < 3; ++dx) {
      int yy = y + dy - 1, xx = x + dx - 1;
      yy = yy < 0 ? yy + N : (yy >= N ? yy - N : yy);
      xx = xx < 0 ? xx + N : (xx >= N ? xx - N : xx);
      const float v = (float)e[(long)yy * pe + xx];
      xv[dy * 3 + dx] = s > 0.f ? from_bf16(to_bf16(v / s)) : 0.f;
    }
  unsigned short o[8];
  for (int c = 0; c < 8; ++c) {
    const float* w = stem_w + (g * 8 + c) * 9;
    float acc = 0.f;
    for (int t = 0; t < 9; ++t) acc += w[t] * xv[t];
    o[c] = to_bf16(fmaxf(acc, 0.f));
  }
  uint4 pk;
  pk.x = o[0] | ((unsigned)o[1] << 16);
  pk.y = o[2] | ((unsigned)o[3] << 16);
  pk.z = o[4] | ((unsigned)o[5] << 16);
  pk.w = o[6] | ((unsigned)o[7] << 16);
  *reinterpret_cast<uint4*>(h + pix * kC + g * 8) = pk;
}

// ---------------------------------------------------------------- 64-channel conv
// MODE 0: out = bf16(relu(conv(in)))            [N][N][64]
// MODE 1: out = bf16(skip + conv(in))            [N][N][64] (out may alias skip)
// MODE 2: sub-pixel ab = blockIdx.y of the x2 shuffle: out[2y+a][2x+b] =
//         bf16(relu(conv(in))) with the 64 channels of weight set ab  [2N][2N][64]
// w: weight sets of [9 taps][64 out][64 in] bf16 (set blockIdx.y for MODE 2).
template <int MODE>
__global__ void __launch_bounds__(kConvThreads)
    k_cnn_conv(int N, const unsigned short* __restrict__ in, const unsigned short* __restrict__ w,
               unsigned short* out, const unsigned short* skip) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  uint4* wl = reinterpret_cast<uint4*>(lds);                    // kWChunks
  uint4* il = reinterpret_cast<uint4*>(lds) + kWChunks;         // kTileChunks
  const int tiles_x = N / kTW;
  const int tile = blockIdx.x;
  const int row0 = (tile / tiles_x) * kTH, col0 = (tile % tiles_x) * kTW;
  const uint4* wg = reinterpret_cast<const uint4*>(w) + (size_t)(MODE == 2 ? blockIdx.y : 0) * kWChunks;
  for (int q = threadIdx.x; q < kWChunks; q += kConvThreads) wl[swz(q >> 3, q & 7)] = wg[q];
  for (int q = threadIdx.x; q < kTileChunks; q += kConvThreads) {
    const int p = q >> 3, c = q & 7;
    const int ty = p / kHW, tx = p % kHW;
    int gy = row0 - 1 + ty, gx = col0 - 1 + tx;
    gy = gy < 0 ? gy + N : (gy >= N ? gy - N : gy);
    gx = gx < 0 ? gx + N : (gx >= N ? gx - N : gx);
    il[swz(p, c)] = reinterpret_cast<const uint4*>(in)[((size_t)gy * N + gx) * 8 + c];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 31, kh = lane >> 5;
  f32x16 acc[2][2];
  for (int j = 0; j < 2; ++j)
    for (int i = 0; i < 2; ++i)
      for (int v = 0; v < 16; ++v) acc[j][i][v] = 0.f;
#pragma unroll 1
  for (int tap = 0; tap < 9; ++tap) {
    const int ky = tap / 3, kx = tap % 3;
    const int p0 = (2 * wave + ky) * kHW + m + kx;
    const int p1 = p0 + kHW;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int c = kc * 2 + kh;
      const bf16x8 a0 = __builtin_bit_cast(bf16x8, wl[swz(tap * kC + m, c)]);
      const bf16x8 a1 = __builtin_bit_cast(bf16x8, wl[swz(tap * kC + 32 + m, c)]);
      const bf16x8 b0 = __builtin_bit_cast(bf16x8, il[swz(p0, c)]);
      const bf16x8 b1 = __builtin_bit_cast(bf16x8, il[swz(p1, c)]);
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
  }

  // Lane holds pixel column m and output channels 32j + 8g + 4kh + (0..3).
  for (int i = 0; i < 2; ++i) {
    const int y = row0 + 2 * wave + i, x = col0 + m;
    size_t base;
    if (MODE == 2) {
      const int a = blockIdx.y >> 1, b = blockIdx.y & 1;
      base = ((size_t)(2 * y + a) * (2 * N) + (2 * x + b)) * kC;
    } else {
      base = ((size_t)y * N + x) * kC;
    }
    for (int j = 0; j < 2; ++j)
      for (int g = 0; g < 4; ++g) {
        const int ch = 32 * j + 8 * g + 4 * kh;
        float v[4];
        for (int r = 0; r < 4; ++r) v[r] = acc[j][i][4 * g + r];
        if (MODE == 1) {
          const uint2 sk = *reinterpret_cast<const uint2*>(skip + base + ch);
          v[0] += from_bf16(sk.x & 0xffff);
          v[1] += from_bf16(sk.x >> 16);
          v[2] += from_bf16(sk.y & 0xffff);
          v[3] += from_bf16(sk.y >> 16);
        } else {
          for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r], 0.f);
        }
        uint2 pk;
        pk.x = to_bf16(v[0]) | ((unsigned)to_bf16(v[1]) << 16);
        pk.y = to_bf16(v[2]) | ((unsigned)to_bf16(v[3]) << 16);
        *reinterpret_cast<uint2*>(out + base + ch) = pk;
      }
  }
}

// ---------------------------------------------------------------- final conv
// 64 -> 1 at fine resolution M = 2N, times s, added to uin (nullable) and
// written to uout (the fine grid, M + 1 nodes per side; the seam row and
// column are written too).  Tile 16 x 16 fine pixels; fin_w: [9][64] floats.
constexpr int kFT = 16;
constexpr int kFHW = kFT + 2;
template <typename T>
__global__ void __launch_bounds__(256)
    k_cnn_final(int M, const unsigned short* __restrict__ z, const float* __restrict__ fin_w,
                const float* __restrict__ scale, const T* uin, int pui, T* uout, int puo) {
  __shared__ __attribute__((aligned(16))) uint4 tl[kFHW * kFHW * 8];
  __shared__ float wf[9 * kC];
  const int tiles_x = M / kFT;
  const int y0 = (blockIdx.x / tiles_x) * kFT, x0 = (blockIdx.x % tiles_x) * kFT;
  for (int q = threadIdx.x; q < 9 * kC; q += 256) wf[q] = fin_w[q];
  for (int q = threadIdx.x; q < kFHW * kFHW * 8; q += 256) {
    const int p = q >> 3, c = q & 7;
    int gy = y0 - 1 + p / kFHW, gx = x0 - 1 + p % kFHW;
    gy = gy < 0 ? gy + M : (gy >= M ? gy - M : gy);
    gx = gx < 0 ? gx + M : (gx >= M ? gx - M : gx);
    tl[swz(p, c)] = reinterpret_cast<const uint4*>(z)[((size_t)gy * M + gx) * 8 + c];
  }
  __syncthreads();
  const int ty = threadIdx.x / kFT, tx = threadIdx.x % kFT;
  float acc = 0.f;
  for (int tap = 0; tap < 9; ++tap) {
    const int p = (ty + tap / 3) * kFHW + tx + tap % 3;
    for (int c = 0; c < 8; ++c) {
      const uint4 v = tl[swz(p, c)];
      const float* wv = wf + tap * kC + c * 8;
      acc += wv[0] * from_bf16(v.x & 0xffff) + wv[1] * from_bf16(v.x >> 16) +
             wv[2] * from_bf16(v.y & 0xffff) + wv[3] * from_bf16(v.y >> 16) +
             wv[4] * from_bf16(v.z & 0xffff) + wv[5] * from_bf16(v.z >> 16) +
             wv[6] * from_bf16(v.w & 0xffff) + wv[7] * from_bf16(v.w >> 16);
    }
  }
  const T d = (T)(scale[0] * acc);
  const int y = y0 + ty, x = x0 + tx;
  auto put = [&](int yy, int xx) {
    const T base = uin ? uin[(size_t)yy * pui + xx] : T(0);
    uout[(size_t)yy * puo + xx] = base + d;
  };
  put(y, x);
  if (y == 0) put(M, x);
  if (x == 0) put(y, M);
  if (x == 0 && y == 0) put(M, M);
}

}  // namespace

size_t cnn_conv_lds() { return (size_t)(kWChunks + kTileChunks) * 16; }

hipError_t cnn_init() {
  hipError_t e = hipFuncSetAttribute((const void*)k_cnn_conv<0>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)cnn_conv_lds());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_cnn_conv<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)cnn_conv_lds());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_cnn_conv<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)cnn_conv_lds());
  return e;
}

int cnn_partials() { return kPartials; }

template <typename T>
hipError_t launch_cnn_head(hipStream_t s, int N, const T* e, int pe, float* partials,
                           const float* stem_w, unsigned short* h, float* scale) {
  hipLaunchKernelGGL(k_cnn_absmax<T>, dim3(kPartials), dim3(256), 0, s, N, e, pe, partials);
  const long threads = (long)N * N * 8;
  hipLaunchKernelGGL(k_cnn_stem<T>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, N, e,
                     pe, partials, stem_w, h, scale);
  return hipGetLastError();
}

hipError_t launch_cnn_conv(hipStream_t s, int mode, int N, const unsigned short* in,
                           const unsigned short* w, unsigned short* out, const unsigned short* skip) {
  const dim3 grid((unsigned)((N / kTW) * (N / kTH)), mode == 2 ? 4 : 1);
  const size_t lds = cnn_conv_lds();
  if (mode == 0)
    hipLaunchKernelGGL(k_cnn_conv<0>, grid, dim3(kConvThreads), lds, s, N, in, w, out, skip);
  else if (mode == 1)
    hipLaunchKernelGGL(k_cnn_conv<1>, grid, dim3(kConvThreads), lds, s, N, in, w, out, skip);
  else
    hipLaunchKernelGGL(k_cnn_conv<2>, grid, dim3(kConvThreads), lds, s, N, in, w, out, skip);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cnn_final(hipStream_t s, int N, const unsigned short* z, const float* fin_w,
                            const float* scale, const T* uin, int pui, T* uout, int puo) {
  const int M = 2 * N;
  hipLaunchKernelGGL(k_cnn_final<T>, dim3((unsigned)((M / kFT) * (M / kFT))), dim3(256), 0, s, M, z,
                     fin_w, scale, uin, pui, uout, puo);
  return hipGetLastError();
}

#define MG_CNN_INSTANTIATE(T)                                                                   \
  template hipError_t launch_cnn_head<T>(hipStream_t, int, const T*, int, float*, const float*, \
                                         unsigned short*, float*);                              \
  template hipError_t launch_cnn_final<T>(hipStream_t, int, const unsigned short*, const float*, \
                                          const float*, const T*, int, T*, int);
MG_CNN_INSTANTIATE(double)
MG_CNN_INSTANTIATE(float)

}  // namespace mg
