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

#include <algorithm>

namespace mg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kC = 64;            // channels
constexpr int kTH = 8;            // output rows per tile
constexpr int kTW = 32;           // output columns per tile
constexpr int kHW = kTW + 2;      // tile width with halo
constexpr int kTileChunks = (kTH + 2) * kHW * 8;  // 16-byte chunks of the input tile
constexpr int kWChunks = 9 * kC * 8;              // 16-byte chunks of one 64x64 weight set
constexpr int kConvThreads = 256;
constexpr int kPartials = 256;    // blocks of the max-abs pass
constexpr int kAheadK = 3;        // K-steps the operand reads run ahead of the products

__device__ __forceinline__ unsigned short to_bf16(float x) {
  return __builtin_bit_cast(unsigned short, (__bf16)x);
}
__device__ __forceinline__ float from_bf16(unsigned short b) {
  return __builtin_bit_cast(float, (unsigned)b << 16);
}

// Placement of 16-byte chunk c (0..7) of 128-byte row r.  The LDS serves a
// 16-byte read of 64 lanes from 64 banks (256 bytes per pass), so the
// chunks that 16 lanes reading 16 consecutive rows ask for must fill all 64
// banks: consecutive row pairs share a 256-byte bank row, and XOR-ing the
// chunk with r/2 spreads the eight pairs over its eight 32-byte slots.
// (XOR with r itself leaves rows r and r + 8 on the same banks: a 2-way
// conflict measured with SQ_LDS_BANK_CONFLICT.)
__device__ __forceinline__ int swz(int r, int c) { return r * 8 + (c ^ ((r >> 1) & 7)); }

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

// scale[0] = max of the partials (one workgroup).
__global__ void __launch_bounds__(256) k_cnn_scale(const float* __restrict__ partials,
                                                   float* __restrict__ scale) {
  __shared__ float red[256];
  red[threadIdx.x] = partials[threadIdx.x];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scale[0] = red[0];
}

// ---------------------------------------------------------------- stem
// Eight lanes per pixel, lane g of them computing output channels 8g..8g+7
// (16 bytes) from the pixel's 9 scaled, bf16-rounded inputs, so that the
// eight store the pixel's 128 bytes together (one pixel per thread, each
// writing its eight chunks, touched a cache line per lane: 25.9 us at
// 512^2).  stem_w: [64][9] floats, staged in LDS.
template <typename T>
__global__ void __launch_bounds__(256)
    k_cnn_stem(int N, const T* __restrict__ e, int pe, const float* __restrict__ scale,
               const float* __restrict__ stem_w, unsigned short* __restrict__ h) {
  __shared__ float sw[kC * 9];
  const long nq = (long)N * N * 8;
  const long q0 = (long)blockIdx.x * 256 + threadIdx.x;
  const bool live = q0 < nq;
  const long q = live ? q0 : nq - 1;  // past the end: a re-read, not stored
  const long pix = q >> 3;
  const int g = (int)(q & 7);
  const int y = (int)(pix / N), x = (int)(pix % N);
  // The inputs' reads go out before the weights' barrier, so that the two
  // latencies overlap.
  T ev[9];
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      int yy = y + dy - 1, xx = x + dx - 1;
      yy = yy < 0 ? yy + N : (yy >= N ? yy - N : yy);
      xx = xx < 0 ? xx + N : (xx >= N ? xx - N : xx);
      ev[dy * 3 + dx] = e[(long)yy * pe + xx];
    }
  for (int k = threadIdx.x; k < kC * 9; k += 256) sw[k] = stem_w[k];
  __syncthreads();
  if (!live) return;
  const float s = scale[0];
  float xv[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const float v = (float)ev[t];
    xv[t] = s > 0.f ? from_bf16(to_bf16(v / s)) : 0.f;
  }
  unsigned short o[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const float* w = sw + (g * 8 + c) * 9;
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) acc += w[t] * xv[t];
    o[c] = to_bf16(fmaxf(acc, 0.f));
  }
  uint4 pk;
  pk.x = o[0] | ((unsigned)o[1] << 16);
  pk.y = o[2] | ((unsigned)o[3] << 16);
  pk.z = o[4] | ((unsigned)o[5] << 16);
  pk.w = o[6] | ((unsigned)o[7] << 16);
  reinterpret_cast<uint4*>(h)[q] = pk;  // chunk g of pixel pix
}

// ---------------------------------------------------------------- 64-channel conv
// MODE 0: out = bf16(relu(conv(in)))            [N][N][64]
// MODE 1: out = bf16(skip + conv(in))            [N][N][64] (out may alias skip)
// MODE 2: sub-pixel ab = blockIdx.y of the x2 shuffle: out[2y+a][2x+b] =
//         bf16(relu(conv(in))) with the 64 channels of weight set ab  [2N][2N][64]
// w: weight sets of [9 taps][64 out][64 in] bf16 (set blockIdx.y for MODE 2).
//
// Each workgroup keeps its weight set in LDS and walks the tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...; the next tile's input is loaded
// into registers while the current tile is computed, then written to the
// other of two LDS tile buffers.  (Copying it with LDS-direct loads instead
// makes the compiler wait for every outstanding LDS read before each step
// of the product loop, which costs more than the registers.)
//
// LDS layouts are chunk-major: slot (c, row) holds 16-byte chunk c (input
// channels 8c .. 8c+7) of a weight row (tap * 64 + out channel) or of a
// tile pixel.  A fragment read by 32 lanes then covers 32 consecutive
// slots (no bank conflicts), and every read of a step is one per-lane base
// address plus a compile-time offset.  The weight chunks of one c lie
// kWStride = kWRows + 2 slots apart: a weight set is fetched a row's eight
// chunks by eight consecutive lanes (whole 128-byte rows from HBM), and
// with a stride of 32 mod 256 bytes the sixteen 16-byte bank groups each
// serve four lanes of a wavefront's store (at kWRows, 0 mod 256, eight
// lanes would share one).
constexpr int kWRows = 9 * kC;                  // weight rows (tap, out channel)
constexpr int kWStride = kWRows + 2;            // LDS slots between weight chunks c and c + 1
constexpr int kWSlots = 8 * kWStride;           // LDS slots of a weight set
constexpr int kTPix = (kTH + 2) * kHW;          // tile pixels with halo
constexpr int kWPerThread = kWChunks / kConvThreads;                           // 18
static_assert(kWChunks % kConvThreads == 0, "weight chunks split evenly");
static_assert((kWSlots + 2 * kTileChunks) * 16 <= 160 * 1024, "weights and two tiles fit the LDS");
static_assert(kTH * kTW * 8 % kConvThreads == 0, "result chunks split evenly");
static_assert(kTH * kTW * 8 <= kTileChunks, "the results fit in a tile buffer");
constexpr int kTPerThread = (kTileChunks + kConvThreads - 1) / kConvThreads;  // 11

// The chunks are held as a native vector type: copies of the uint4 struct
// became memory copies through a stack array once the results were staged
// in LDS (192 bytes of scratch per lane).
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void tile_fetch(u32x4 (&r)[kTPerThread], const uint4* __restrict__ in4,
                                           int N, int tile, int tid) {
  const u32x4* in = reinterpret_cast<const u32x4*>(in4);
  const int tiles_x = N / kTW;
  const int row0 = (tile / tiles_x) * kTH, col0 = (tile % tiles_x) * kTW;
#pragma unroll
  for (int k = 0; k < kTPerThread; ++k) {
    // Chunk q is 16-byte chunk q % 8 of tile pixel q / 8 (a pixel's 128
    // bytes by eight consecutive lanes); threads past the tile's last chunk
    // re-read that chunk (not stored).
    const int q = min(k * kConvThreads + tid, kTileChunks - 1);
    const int c = q & 7, p = q >> 3;
    int gy = row0 - 1 + p / kHW, gx = col0 - 1 + p % kHW;
    gy = gy < 0 ? gy + N : (gy >= N ? gy - N : gy);
    gx = gx < 0 ? gx + N : (gx >= N ? gx - N : gx);
    r[k] = in[((size_t)gy * N + gx) * 8 + c];
  }
}

// Chunk q of tile_fetch to its chunk-major LDS slot.  The eight lanes of a
// pixel write slots kTPix = 340 apart (64 mod 256 bytes): with the pixel
// offsets each 16-byte bank group serves four lanes of a wavefront, no
// conflict.
__device__ __forceinline__ int tile_slot(int q) { return (q & 7) * kTPix + (q >> 3); }

__device__ __forceinline__ void tile_store(uint4* buf4, int tid, const u32x4 (&r)[kTPerThread]) {
  u32x4* buf = reinterpret_cast<u32x4*>(buf4);
#pragma unroll
  for (int k = 0; k < kTPerThread - 1; ++k) buf[tile_slot(k * kConvThreads + tid)] = r[k];
  const int q = (kTPerThread - 1) * kConvThreads + tid;
  if (q < kTileChunks) buf[tile_slot(q)] = r[kTPerThread - 1];
}

template <int MODE>
__global__ void __launch_bounds__(kConvThreads)
    k_cnn_conv(int N, const unsigned short* __restrict__ in, const unsigned short* __restrict__ w,
               unsigned short* out, const unsigned short* skip) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  uint4* wl = reinterpret_cast<uint4*>(lds);                         // kWSlots
  uint4* ib = reinterpret_cast<uint4*>(lds) + kWSlots;               // 2 x kTileChunks
  const int tid = threadIdx.x;
  const int tiles_x = N / kTW, tiles = tiles_x * (N / kTH);
  const uint4* in4 = reinterpret_cast<const uint4*>(in);
  int tile = blockIdx.x;
  if (tile >= tiles) return;  // uniform per workgroup
  {
    const uint4* wg = reinterpret_cast<const uint4*>(w) + (size_t)(MODE == 2 ? blockIdx.y : 0) * kWChunks;
    uint4 r[kWPerThread];
#pragma unroll
    for (int k = 0; k < kWPerThread; ++k) {
      const int q = k * kConvThreads + tid;
      r[k] = wg[q];  // chunk q & 7 of weight row q >> 3
    }
#pragma unroll
    for (int k = 0; k < kWPerThread; ++k) {
      const int q = k * kConvThreads + tid;
      wl[(q & 7) * kWStride + (q >> 3)] = r[k];
    }
  }
  {
    u32x4 first[kTPerThread];
    tile_fetch(first, in4, N, tile, tid);
    tile_store(ib, tid, first);
  }
  __syncthreads();

  const int lane = tid & 63, wave = tid >> 6;
  const int m = lane & 31, kh = lane >> 5;
  int cur = 0;
  for (; tile < tiles; tile += gridDim.x) {
    const int next = tile + gridDim.x;
    u32x4 pre[kTPerThread];
    tile_fetch(pre, in4, N, next < tiles ? next : tile, tid);  // last pass: a re-read
    const uint4* il = ib + cur * kTileChunks;
    // The skip values (MODE 1) at this lane's outputs (pixel column m of
    // rows 2 wave + i), loaded before the product loop so that their
    // latency hides behind it (out may alias skip: each value is read here,
    // before the barriers after which this workgroup writes it).
    const int row0 = (tile / tiles_x) * kTH, col0 = (tile % tiles_x) * kTW;
    uint2 skv[2][2][4];
    if (MODE == 1) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const size_t ob = ((size_t)(row0 + 2 * wave + i) * N + (col0 + m)) * kC;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int g = 0; g < 4; ++g)
            skv[i][j][g] = *reinterpret_cast<const uint2*>(skip + ob + 32 * j + 8 * g + 4 * kh);
      }
    }

    f32x16 acc[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[j][i][v] = 0.f;
    // K loop of 36 steps (9 taps x 4 chunks of 16 input channels), fully
    // unrolled, with the four operand fragments of step s + kAheadK read
    // from LDS while the four products of step s run (LDS latency under
    // this load is several steps of products; at most 15 LDS reads may be
    // outstanding, so 3 steps of 4: measured 5 % faster than 2, and 4
    // steps, which make the compiler wait on the counter, slower).
    const uint4* wb = wl + kh * kWStride + m;               // chunk kh, row m
    const uint4* ibase = il + kh * kTPix + 2 * wave * kHW + m;  // chunk kh, pixel (2 wave, m)
    auto fetch = [&](int st, bf16x8 (&fr)[4]) {
      const int tap = st >> 2, kc = st & 3;
      const int poff = 2 * kc * kTPix + (tap / 3) * kHW + tap % 3;
      fr[0] = __builtin_bit_cast(bf16x8, wb[2 * kc * kWStride + tap * kC]);
      fr[1] = __builtin_bit_cast(bf16x8, wb[2 * kc * kWStride + tap * kC + 32]);
      fr[2] = __builtin_bit_cast(bf16x8, ibase[poff]);
      fr[3] = __builtin_bit_cast(bf16x8, ibase[poff + kHW]);
    };
    bf16x8 fr[kAheadK + 1][4];
#pragma unroll
    for (int st = 0; st < kAheadK; ++st) fetch(st, fr[st]);
#pragma unroll
    for (int st = 0; st < 36; ++st) {
      if (st + kAheadK < 36) fetch(st + kAheadK, fr[(st + kAheadK) % (kAheadK + 1)]);
      const bf16x8(&f)[4] = fr[st % (kAheadK + 1)];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f[0], f[2], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f[0], f[3], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f[1], f[2], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f[1], f[3], acc[1][1], 0, 0, 0);
      // Nothing moves across step boundaries: the reads of step
      // st + kAheadK stay in step st, ahead of their use by that many steps
      // of products, so the LDS latency hides behind the matrix pipe.
      __builtin_amdgcn_sched_barrier(0);
    }

    // Lane holds pixel column m and output channels 32j + 8g + 4kh + (0..3)
    // of output rows 2 wave + i.  The bf16 results go to this tile's LDS
    // buffer (read by every wavefront's products until the barrier) as
    // pixel records (pixel p = 32 row + column, 16-byte chunk 4j + g, half
    // kh; chunks placed by swz), then out a whole chunk per lane.  The next
    // tile goes to the other buffer first (free since the last pass's final
    // barrier), so that its registers are not held through the results.
    __syncthreads();
    if (next < tiles) tile_store(ib + (cur ^ 1) * kTileChunks, tid, pre);
    uint4* rl = ib + cur * kTileChunks;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          float v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = acc[j][i][4 * g + r];
          if (MODE == 1) {
            const uint2 sk = skv[i][j][g];
            v[0] += from_bf16(sk.x & 0xffff);
            v[1] += from_bf16(sk.x >> 16);
            v[2] += from_bf16(sk.y & 0xffff);
            v[3] += from_bf16(sk.y >> 16);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r], 0.f);
          }
          uint2 pk;
          pk.x = to_bf16(v[0]) | ((unsigned)to_bf16(v[1]) << 16);
          pk.y = to_bf16(v[2]) | ((unsigned)to_bf16(v[3]) << 16);
          reinterpret_cast<uint2*>(rl + swz(32 * (2 * wave + i) + m, 4 * j + g))[kh] = pk;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTH * kTW * 8 / kConvThreads; ++k) {
      const int q = k * kConvThreads + tid;
      const int p = q >> 3, c = q & 7;
      const int y = row0 + (p >> 5), x = col0 + (p & 31);
      size_t base;
      if (MODE == 2) {
        const int a = blockIdx.y >> 1, b = blockIdx.y & 1;
        base = ((size_t)(2 * y + a) * (2 * N) + (2 * x + b)) * kC;
      } else {
        base = ((size_t)y * N + x) * kC;
      }
      *reinterpret_cast<uint4*>(out + base + 8 * c) = rl[swz(p, c)];
    }
    __syncthreads();
    cur ^= 1;
  }
}

// ---------------------------------------------------------------- 64-channel conv, tall tiles
// The same convolution (MODE as k_cnn_conv) on tiles of 16 x 32 pixels by
// eight wavefronts: wavefront w computes output rows 4 (w >> 1) .. + 3 for
// the 32 output channels of half w & 1 (four 32 x 32 accumulator tiles).
// The K loop runs over (column tap dx, 16-channel chunk kc): the six input
// rows that four output rows see are read once and serve all three row taps
// dy, so a step of 12 products reads 3 weight and 6 pixel fragments from
// LDS (0.75 per product, against 1 in k_cnn_conv, whose products wait on
// LDS), the next step's reads issued before the current step's products.
// LDS: the weight set and one input tile (16 + 2) x (32 + 2) pixels; the
// next tile is fetched into registers during the products and stored after
// them.  Both sides of HBM are read and written a whole 16-byte chunk per
// lane, consecutive lanes on consecutive chunks: a tile is fetched eight
// lanes to a pixel (all of its 128 bytes), and the results go through the
// input tile's LDS (free once the products are done) so that they leave as
// whole pixels too.  Reading a chunk per lane across pixels (lanes 128
// bytes apart) or storing from the accumulator layout (8 bytes per lane)
// touches a line per lane and ran the kernel at 0.75x the speed.
constexpr int kTH4 = 16;
constexpr int kConv4Threads = 512;
constexpr int kTPix4 = (kTH4 + 2) * kHW;
constexpr int kTileChunks4 = kTPix4 * 8;
constexpr int kTPerThread4 = (kTileChunks4 + kConv4Threads - 1) / kConv4Threads;  // 10
constexpr int kWPerThread4 = kWChunks / kConv4Threads;                            // 9
static_assert(kWChunks % kConv4Threads == 0, "weight chunks split evenly");
static_assert((kWSlots + kTileChunks4) * 16 <= 160 * 1024, "weights and tile fit the LDS");
static_assert(kTH4 * kTW * 8 % kConv4Threads == 0, "result chunks split evenly");
static_assert(kTH4 * kTW * 8 <= kTileChunks4, "the results fit in the input tile's LDS");

template <int MODE>
__global__ void __launch_bounds__(kConv4Threads)
    k_cnn_conv4(int N, const unsigned short* __restrict__ in, const unsigned short* __restrict__ w,
                unsigned short* out, const unsigned short* skip) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  uint4* wl = reinterpret_cast<uint4*>(lds);             // kWSlots
  uint4* ib = reinterpret_cast<uint4*>(lds) + kWSlots;   // kTileChunks4
  const int tid = threadIdx.x;
  const int tiles_x = N / kTW, tiles = tiles_x * (N / kTH4);
  const uint4* in4 = reinterpret_cast<const uint4*>(in);
  int tile = blockIdx.x;
  if (tile >= tiles) return;  // uniform per workgroup
  // Chunk q of a tile's input (q < kTileChunks4): 16-byte chunk q % 8 of
  // tile pixel q / 8, with periodic wrap; it goes to LDS slot lds_slot(q) of
  // the chunk-major layout.  (The eight lanes of a pixel write slots
  // kTPix4 = 612 apart, 64 mod 256 bytes: with the pixel offsets each
  // 16-byte bank group serves four lanes of a wavefront, no conflict.)
  auto lds_slot = [](int q) { return (q & 7) * kTPix4 + (q >> 3); };
  auto chunk_of = [&](int t, int q) {
    const int row0 = (t / tiles_x) * kTH4, col0 = (t % tiles_x) * kTW;
    const int c = q & 7, p = q >> 3;
    int gy = row0 - 1 + p / kHW, gx = col0 - 1 + p % kHW;
    gy = gy < 0 ? gy + N : (gy >= N ? gy - N : gy);
    gx = gx < 0 ? gx + N : (gx >= N ? gx - N : gx);
    return in4[((size_t)gy * N + gx) * 8 + c];
  };
  {
    const uint4* wg = reinterpret_cast<const uint4*>(w) + (size_t)(MODE == 2 ? blockIdx.y : 0) * kWChunks;
    uint4 r[kWPerThread4];
#pragma unroll
    for (int k = 0; k < kWPerThread4; ++k) {
      const int q = k * kConv4Threads + tid;
      r[k] = wg[q];  // chunk q & 7 of weight row q >> 3
    }
#pragma unroll
    for (int k = 0; k < kWPerThread4; ++k) {
      const int q = k * kConv4Threads + tid;
      wl[(q & 7) * kWStride + (q >> 3)] = r[k];
    }
    uint4 t[kTPerThread4];
#pragma unroll
    for (int k = 0; k < kTPerThread4; ++k) t[k] = chunk_of(tile, min(k * kConv4Threads + tid, kTileChunks4 - 1));
#pragma unroll
    for (int k = 0; k < kTPerThread4; ++k)
      if (k * kConv4Threads + tid < kTileChunks4) ib[lds_slot(k * kConv4Threads + tid)] = t[k];
  }
  __syncthreads();

  const int lane = tid & 63, wave = tid >> 6;
  const int rg = wave >> 1, hf = wave & 1;
  const int m = lane & 31, kh = lane >> 5;
  const uint4* wb = wl + kh * kWStride + 32 * hf + m;         // chunk kh, weight row 32 hf + m
  const uint4* ibase = ib + kh * kTPix4 + 4 * rg * kHW + m;   // chunk kh, pixel (4 rg, m)
  for (; tile < tiles; tile += gridDim.x) {
    const int next = tile + gridDim.x;
    // The next tile's input, in registers until this tile's products are
    // done (the last pass re-reads this tile; nothing is stored then).
    uint4 pre[kTPerThread4];
#pragma unroll
    for (int k = 0; k < kTPerThread4; ++k)
      pre[k] = chunk_of(next < tiles ? next : tile, min(k * kConv4Threads + tid, kTileChunks4 - 1));
    const int row0 = (tile / tiles_x) * kTH4, col0 = (tile % tiles_x) * kTW;

    f32x16 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;
    // Step st = (dx, kc): fragments A[dy] (weights of tap (dy, dx), output
    // channel 32 hf + m) and B[r] (input row 4 rg + r, column m + dx), all
    // of input-channel chunk 2 kc + kh.
    auto fetch = [&](int st, bf16x8 (&fa)[3], bf16x8 (&fb)[6]) {
      const int dx = st >> 2, kc = st & 3;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
        fa[dy] = __builtin_bit_cast(bf16x8, wb[2 * kc * kWStride + (dy * 3 + dx) * kC]);
#pragma unroll
      for (int r = 0; r < 6; ++r)
        fb[r] = __builtin_bit_cast(bf16x8, ibase[2 * kc * kTPix4 + r * kHW + dx]);
    };
    // The skip values (MODE 1), read before the products so that their
    // latency hides behind them (out may alias skip: each value is read
    // here, before the barrier after which this workgroup writes it).
    uint2 skv[4][4];
    if (MODE == 1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const size_t ob = ((size_t)(row0 + 4 * rg + i) * N + (col0 + m)) * kC;
#pragma unroll
        for (int g = 0; g < 4; ++g)
          skv[i][g] = *reinterpret_cast<const uint2*>(skip + ob + 32 * hf + 8 * g + 4 * kh);
      }
    }
    bf16x8 fa[2][3], fb[2][6];
    fetch(0, fa[0], fb[0]);
#pragma unroll
    for (int st = 0; st < 12; ++st) {
      if (st + 1 < 12) fetch(st + 1, fa[(st + 1) & 1], fb[(st + 1) & 1]);
      // The next step's reads go out before any of this step's products, a
      // whole step ahead of their use; without the barrier the compiler
      // reuses this step's operand registers for them and issues each read
      // just before it is needed.
      __builtin_amdgcn_sched_barrier(0);
      const bf16x8(&a)[3] = fa[st & 1];
      const bf16x8(&b)[6] = fb[st & 1];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[dy], b[i + dy], acc[i], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }

    // Lane holds pixel column m and output channels 32 hf + 8 g + 4 kh +
    // (0..3) of output rows 4 rg + i.  The bf16 results go to LDS as pixel
    // records (pixel p = 32 row + column, 16-byte chunk 4 hf + g, half kh;
    // chunks placed by swz), then out a chunk per lane.
    __syncthreads();  // every wavefront is done reading this tile's input
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float v[4];
        for (int r = 0; r < 4; ++r) v[r] = acc[i][4 * g + r];
        if (MODE == 1) {
          const uint2 sk = skv[i][g];
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
        reinterpret_cast<uint2*>(ib + swz(32 * (4 * rg + i) + m, 4 * hf + g))[kh] = pk;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTH4 * kTW * 8 / kConv4Threads; ++k) {
      const int q = k * kConv4Threads + tid;
      const int p = q >> 3, c = q & 7;
      const int y = row0 + (p >> 5), x = col0 + (p & 31);
      size_t base;
      if (MODE == 2) {
        const int a = blockIdx.y >> 1, b = blockIdx.y & 1;
        base = ((size_t)(2 * y + a) * (2 * N) + (2 * x + b)) * kC;
      } else {
        base = ((size_t)y * N + x) * kC;
      }
      *reinterpret_cast<uint4*>(out + base + 8 * c) = ib[swz(p, c)];
    }
    if (next < tiles) {
      __syncthreads();  // every wavefront is done with the results
#pragma unroll
      for (int k = 0; k < kTPerThread4; ++k)
        if (k * kConv4Threads + tid < kTileChunks4) ib[lds_slot(k * kConv4Threads + tid)] = pre[k];
      __syncthreads();
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
  __shared__ __attribute__((aligned(16))) uint4 tl[kFHW * kFHW * 8];  // chunk-major: [c][pixel]
  __shared__ __attribute__((aligned(16))) unsigned wf[9 * kC / 2];    // bf16 pairs [tap][ch/2]
  const int tiles_x = M / kFT;
  const int y0 = (blockIdx.x / tiles_x) * kFT, x0 = (blockIdx.x % tiles_x) * kFT;
  const int ty = threadIdx.x / kFT, tx = threadIdx.x % kFT;
  const int y = y0 + ty, x = x0 + tx;
  // The tile's reads, the weights' and this node's uin value go out
  // together (no latency waits on another before the products).
  const T base = uin ? uin[(size_t)y * pui + x] : T(0);
  {
    constexpr int kChunks = kFHW * kFHW * 8, kPer = (kChunks + 255) / 256;
    uint4 r[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int q = min((int)threadIdx.x + k * 256, kChunks - 1);
      const int p = q >> 3, c = q & 7;
      int gy = y0 - 1 + p / kFHW, gx = x0 - 1 + p % kFHW;
      gy = gy < 0 ? gy + M : (gy >= M ? gy - M : gy);
      gx = gx < 0 ? gx + M : (gx >= M ? gx - M : gx);
      r[k] = reinterpret_cast<const uint4*>(z)[((size_t)gy * M + gx) * 8 + c];
    }
    // The weights are bf16 values (rounded at setup), so packing is exact.
    for (int q = threadIdx.x; q < 9 * kC / 2; q += 256)
      wf[q] = to_bf16(fin_w[2 * q]) | ((unsigned)to_bf16(fin_w[2 * q + 1]) << 16);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int q = threadIdx.x + k * 256;
      if (q < kChunks) tl[(q & 7) * (kFHW * kFHW) + (q >> 3)] = r[k];
    }
  }
  __syncthreads();
  // Products of two bf16 values are exact in FP32; v_dot2 adds a pair of
  // them to the FP32 accumulator.
  float acc = 0.f;
#pragma unroll 1
  for (int tap = 0; tap < 9; ++tap) {
    const int p = (ty + tap / 3) * kFHW + tx + tap % 3;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const uint4 v = tl[c * (kFHW * kFHW) + p];
      const uint4 wv = *reinterpret_cast<const uint4*>(wf + tap * (kC / 2) + c * 4);
      acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, v.x),
                                            __builtin_bit_cast(bf16x2, wv.x), acc, false);
      acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, v.y),
                                            __builtin_bit_cast(bf16x2, wv.y), acc, false);
      acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, v.z),
                                            __builtin_bit_cast(bf16x2, wv.z), acc, false);
      acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, v.w),
                                            __builtin_bit_cast(bf16x2, wv.w), acc, false);
    }
  }
  const T d = (T)(scale[0] * acc);
  auto put = [&](int yy, int xx) {
    const T b = uin ? uin[(size_t)yy * pui + xx] : T(0);
    uout[(size_t)yy * puo + xx] = b + d;
  };
  uout[(size_t)y * puo + x] = base + d;
  if (y == 0) put(M, x);
  if (x == 0) put(y, M);
  if (x == 0 && y == 0) put(M, M);
}

int g_cus = 256;  // compute units of the device (set by cnn_init)

}  // namespace

size_t cnn_conv_lds() { return (size_t)(kWSlots + 2 * kTileChunks) * 16; }
size_t cnn_conv4_lds() { return (size_t)(kWSlots + kTileChunks4) * 16; }

hipError_t cnn_init() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&g_cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_cnn_conv<0>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)cnn_conv_lds());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_cnn_conv<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)cnn_conv_lds());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_cnn_conv<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)cnn_conv_lds());
  const void* tall[] = {(const void*)k_cnn_conv4<0>, (const void*)k_cnn_conv4<1>,
                        (const void*)k_cnn_conv4<2>};
  for (const void* fn : tall)
    if (e == hipSuccess)
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)cnn_conv4_lds());
  return e;
}

int cnn_partials() { return kPartials; }

template <typename T>
hipError_t launch_cnn_head(hipStream_t s, int N, const T* e, int pe, float* partials,
                           const float* stem_w, unsigned short* h, float* scale) {
  hipLaunchKernelGGL(k_cnn_absmax<T>, dim3(kPartials), dim3(256), 0, s, N, e, pe, partials);
  hipLaunchKernelGGL(k_cnn_scale, dim3(1), dim3(256), 0, s, partials, scale);
  const long threads = (long)N * N * 8;
  hipLaunchKernelGGL(k_cnn_stem<T>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, N, e,
                     pe, scale, stem_w, h);
  return hipGetLastError();
}

hipError_t launch_cnn_conv(hipStream_t s, int mode, int N, const unsigned short* in,
                           const unsigned short* w, unsigned short* out, const unsigned short* skip) {
  // At most one workgroup per compute unit (its LDS holds a whole weight
  // set).  Tall tiles (16 rows) where they still give every compute unit a
  // tile; else 8-row tiles, one per workgroup up to a workgroup per compute
  // unit (a 256^2 layer: 12.9 us on 256 workgroups against 15.8 us on 128
  // taking two tiles each, measured with 8-byte result stores: the weight
  // set's load is then shared by fewer products but spread over twice the
  // compute units).
  const int sets = mode == 2 ? 4 : 1;
  const int tall = (N / kTW) * (N / kTH4);
  if (tall * sets >= g_cus) {
    int g = std::max(1, g_cus / sets);
    g = std::min(g, tall);
    const dim3 grid((unsigned)g, (unsigned)sets);
    const size_t lds = cnn_conv4_lds();
    if (mode == 0)
      hipLaunchKernelGGL(k_cnn_conv4<0>, grid, dim3(kConv4Threads), lds, s, N, in, w, out, skip);
    else if (mode == 1)
      hipLaunchKernelGGL(k_cnn_conv4<1>, grid, dim3(kConv4Threads), lds, s, N, in, w, out, skip);
    else
      hipLaunchKernelGGL(k_cnn_conv4<2>, grid, dim3(kConv4Threads), lds, s, N, in, w, out, skip);
    return hipGetLastError();
  }
  const int tiles = (N / kTW) * (N / kTH);
  int g = std::max(1, g_cus / sets);
  g = std::min(g, tiles);
  const dim3 grid((unsigned)g, (unsigned)sets);
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
