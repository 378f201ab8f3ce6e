// Kernels of the learned SART initialiser: a small convolutional
// encoder-decoder trained to map an early split-SART image to a later one.
//
// Activations are NHWC BF16 (gradients FP32 where they accumulate), weights
// FP32 masters with BF16 copies laid out [out][tap][in] (in padded to a
// multiple of 8 with zeros).  The 3x3 convolution is an implicit GEMM on
// the gfx950 BF16 matrix cores (v_mfma_f32_16x16x32_bf16): M = pixels, N =
// output channels, K = 9 taps x input channels, FP32 accumulation.  The
// gradient with respect to the input is the same kernel run on the output
// gradient with the weights flipped and transposed; the weight gradient is
// a GEMM over pixels.

#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>

#include "device.h"
#include "internal.h"

namespace ss {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ inline float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }
__device__ inline uint16_t f2bf(float f) { return static_cast<uint16_t>(bf16_bits_rne(f)); }

__device__ inline bf16x8 as_bf16x8(u16x8 u) {
  bf16x8 r;
  __builtin_memcpy(&r, &u, sizeof r);
  return r;
}

// Operand layouts of v_mfma_f32_16x16x32_bf16 for lane l (g = l / 16):
//   A[m][k]: m = l % 16, k = 8 g .. 8 g + 7   (8 values per lane)
//   B[k][n]: n = l % 16, k = 8 g .. 8 g + 7
//   D[m][n]: m = 4 g + r (r = 0..3), n = l % 16
__device__ inline f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int kConvWaves = 4;

// y[n,i,j,o] = act(bias[o] + sum_{tap,c} w[o][tap][c] x[n, i+ky-1, j+kx-1, c]).
// A wave computes 16 consecutive pixels of one image row for NT tiles of 16
// output channels.  VEC: C is a multiple of 8 (one 16-byte load per lane).
template <int NT, bool VEC>
__global__ __launch_bounds__(kWave* kConvWaves) void k_conv3x3(const uint16_t* __restrict__ x, int H, int W,
                                                                int C, int Cp, const uint16_t* __restrict__ w,
                                                                const float* __restrict__ bias, int O, int relu,
                                                                void* __restrict__ y, int y_f32) {
  const int lane = lane_id(), g = lane / 16, m = lane % 16;
  const int row = blockIdx.y;  // n * H + i
  const int i = row % H;
  const int x0 = (blockIdx.x * kConvWaves + wave_id()) * 16;
  const int o0 = blockIdx.z * 16 * NT;
  if (x0 >= W) return;
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int K = 9 * Cp;
  const int64_t img0 = static_cast<int64_t>(row - i) * W;  // first pixel of image n
  for (int kc = 0; kc < K; kc += 32) {
    const int k = kc + 8 * g;
    const int tap = k / Cp, c0 = k % Cp;
    u16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
    if (tap < 9) {
      const int yy = i + tap / 3 - 1, xx = x0 + m + tap % 3 - 1;
      if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
        const uint16_t* src = x + (img0 + static_cast<int64_t>(yy) * W + xx) * C + c0;
        if constexpr (VEC) {
          a = *gl(reinterpret_cast<const u16x8*>(src));
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) a[q] = c0 + q < C ? gl(src)[q] : uint16_t{0};
        }
      }
    }
    const bf16x8 av = as_bf16x8(a);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int o = o0 + 16 * t + m;
      u16x8 b = {0, 0, 0, 0, 0, 0, 0, 0};
      if (tap < 9 && o < O) b = *gl(reinterpret_cast<const u16x8*>(w + (static_cast<int64_t>(o) * 9 + tap) * Cp + c0));
      acc[t] = mma(av, as_bf16x8(b), acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int o = o0 + 16 * t + m;
    if (o >= O) continue;
    const float bo = bias ? gl(bias)[o] : 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int px = x0 + 4 * g + r;
      if (px >= W) continue;
      float v = acc[t][r] + bo;
      if (relu) v = fmaxf(v, 0.0f);
      const int64_t idx = (static_cast<int64_t>(row) * W + px) * O + o;
      if (y_f32) glw(static_cast<float*>(y))[idx] = v;
      else glw(static_cast<uint16_t*>(y))[idx] = f2bf(v);
    }
  }
}

// The same convolution with the operands staged in shared memory, for
// input channels (padded) a multiple of 16: a block computes 64
// consecutive pixels of one image row (16 per wavefront) for NT tiles of 16
// output channels.  Per chunk of CC input channels it copies the three input
// rows the tile reads (66 pixels with the borders, zeros outside the image)
// and the chunk of the tile's weights into shared memory with 16-byte loads,
// then every wavefront runs the chunk's nine taps on the matrix cores from
// there: each input value is read from memory once per block instead of
// once per tap, and each weight once per block instead of once per
// wavefront.  K order within a chunk: with CC = 32 one tap per product (its
// four groups of 8 channels), with CC = 16 two taps per product (taps 2s and
// 2s + 1, the ninth paired with zeros).  The weights' rows are padded by one
// vector in shared memory, so the 16 output channels of a read fall on
// different banks.
constexpr int kConvPx = 16 * kConvWaves;  // pixels per block
template <int NT, int CC>
__global__ __launch_bounds__(kWave* kConvWaves) void k_conv3x3_t(const uint16_t* __restrict__ x, int H, int W,
                                                                  int C, int Cp, const uint16_t* __restrict__ w,
                                                                  const float* __restrict__ bias, int O, int relu,
                                                                  void* __restrict__ y, int y_f32) {
  constexpr int V = CC / 8;               // 16-byte vectors per pixel and chunk
  constexpr int XV = 3 * (kConvPx + 2) * V;
  constexpr int WS = 9 * V + 1;           // vectors per output channel (padded)
  constexpr int WV = NT * 16 * 9 * V;
  __shared__ u16x8 xs[XV];
  __shared__ u16x8 wsm[NT * 16 * WS];
  const int lane = lane_id(), g = lane / 16, m = lane % 16, wv = wave_id();
  const int row = blockIdx.y;  // n * H + i
  const int i = row % H;
  const int xb = blockIdx.x * kConvPx;
  const int o0 = blockIdx.z * 16 * NT;
  const int64_t img0 = static_cast<int64_t>(row - i) * W;  // first pixel of image n
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int p = 16 * wv + m;  // this lane's pixel in the block (A rows)
  for (int c0 = 0; c0 < Cp; c0 += CC) {
    for (int v = threadIdx.x; v < XV; v += kWave * kConvWaves) {
      const int q = v % V, px = (v / V) % (kConvPx + 2), r = v / V / (kConvPx + 2);
      const int yy = i + r - 1, xx = xb + px - 1;
      u16x8 val = {0, 0, 0, 0, 0, 0, 0, 0};
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        val = *gl(reinterpret_cast<const u16x8*>(x + (img0 + static_cast<int64_t>(yy) * W + xx) * C + c0 + 8 * q));
      xs[v] = val;
    }
    for (int v = threadIdx.x; v < WV; v += kWave * kConvWaves) {
      const int q = v % V, tap = (v / V) % 9, oo = v / V / 9;
      const int o = o0 + oo;
      u16x8 val = {0, 0, 0, 0, 0, 0, 0, 0};
      if (o < O) val = *gl(reinterpret_cast<const u16x8*>(w + (static_cast<int64_t>(o) * 9 + tap) * Cp + c0 + 8 * q));
      wsm[oo * WS + tap * V + q] = val;
    }
    __syncthreads();
    if constexpr (CC == 32) {
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const bf16x8 a = as_bf16x8(xs[((tap / 3) * (kConvPx + 2) + p + tap % 3) * V + g]);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mma(a, as_bf16x8(wsm[(16 * t + m) * WS + tap * V + g]), acc[t]);
      }
    } else {
#pragma unroll
      for (int s2 = 0; s2 < 5; ++s2) {
        const int tap = 2 * s2 + (g >> 1), q = g & 1;
        const bool in = tap < 9;
        const int tt = in ? tap : 0;
        u16x8 av = xs[((tt / 3) * (kConvPx + 2) + p + tt % 3) * V + q];
        if (!in) av = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        const bf16x8 a = as_bf16x8(av);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mma(a, as_bf16x8(wsm[(16 * t + m) * WS + tt * V + q]), acc[t]);
      }
    }
    __syncthreads();
  }
  const int x0 = xb + 16 * wv;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int o = o0 + 16 * t + m;
    if (o >= O) continue;
    const float bo = bias ? gl(bias)[o] : 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int px = x0 + 4 * g + r;
      if (px >= W) continue;
      float v = acc[t][r] + bo;
      if (relu) v = fmaxf(v, 0.0f);
      const int64_t idx = (static_cast<int64_t>(row) * W + px) * O + o;
      if (y_f32) glw(static_cast<float*>(y))[idx] = v;
      else glw(static_cast<uint16_t*>(y))[idx] = f2bf(v);
    }
  }
}

// Partial weight gradients: part[z][o][tap][c] = sum over the pixels of row
// group z of gy[p][o] x[p + shift(tap)][c] (laid out like the FP32 master
// weights, [O][9][C], per group).  GEMM M = o, N = (tap, c) flattened as
// tap * Cp + c, K = pixels.  A wave owns one 16 x 16 tile and one group of
// kWgradRows image rows; k_wgrad_reduce then adds the groups in index
// order, so the gradient is the same on every run.
constexpr int kWgradRows = 8;
__global__ __launch_bounds__(kWave* kConvWaves) void k_conv3x3_wgrad(const uint16_t* __restrict__ x,
                                                                      const uint16_t* __restrict__ gy, int NH,
                                                                      int H, int W, int C, int Cp, int O,
                                                                      float* __restrict__ part) {
  const int lane = lane_id(), g = lane / 16, m = lane % 16;
  const int o0 = blockIdx.x * 16;
  const int n0 = blockIdx.y * 16;
  const int row0 = (blockIdx.z * kConvWaves + wave_id()) * kWgradRows;
  if (row0 >= NH) return;
  const int o = o0 + m;             // A row
  const int nb = n0 + m;            // B column
  const int tap = nb / Cp, c = nb % Cp;
  const bool bvalid = tap < 9 && c < C;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const int row1 = row0 + kWgradRows < NH ? row0 + kWgradRows : NH;
  for (int row = row0; row < row1; ++row) {
    const int i = row % H;
    const int64_t img0 = static_cast<int64_t>(row - i) * W;
    const int yy = i + dy;
    for (int xb = 0; xb < W; xb += 32) {
      u16x8 a, b;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int px = xb + 8 * g + q;
        a[q] = (o < O && px < W) ? gl(gy)[(static_cast<int64_t>(row) * W + px) * O + o] : uint16_t{0};
        const int xx = px + dx;
        b[q] = (bvalid && px < W && yy >= 0 && yy < H && xx >= 0 && xx < W)
                   ? gl(x)[(img0 + static_cast<int64_t>(yy) * W + xx) * C + c]
                   : uint16_t{0};
      }
      acc = mma(as_bf16x8(a), as_bf16x8(b), acc);
    }
  }
  if (bvalid) {
    float* out = part + static_cast<int64_t>(row0 / kWgradRows) * O * 9 * C;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int oo = o0 + 4 * g + r;
      if (oo < O) glw(out)[(static_cast<int64_t>(oo) * 9 + tap) * C + c] = acc[r];
    }
  }
}

// Weight gradient, staged: a wavefront owns one 16 x 16 tile of (o, c) and
// all nine taps, and works through units of 32 pixels of one image row (the
// units of its block's range, in turn).  Per unit it copies the output
// gradient's 32 x 16 tile and the input's three rows of 34 x 16 (the 32
// pixels and one on each side, zero outside the image) into LDS with
// 16-byte loads, then reads the matrix-core operands from there: A[o][p] =
// gy[p][o], B_tap[p][c] = x[p + shift(tap)][c], nine products per unit
// sharing A.  The rows are stored 20 values apart, so the four 16-lane groups
// of an operand read fall in different banks.  The block's four wavefronts
// then add their tiles in order into the block's partial, [O][9][C] per
// block row; k_wgrad_reduce adds those in order.  Needs W a multiple of 32;
// VX (VG): C (O) a multiple of 8, the input's (output gradient's) values
// in 16-byte loads, else value by value.
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

// Eight 16-bit values to LDS at an 8-byte aligned place.
__device__ inline void store_lds8(uint16_t* d, const u16x8& v) {
  reinterpret_cast<u16x4*>(d)[0] = u16x4{v[0], v[1], v[2], v[3]};
  reinterpret_cast<u16x4*>(d)[1] = u16x4{v[4], v[5], v[6], v[7]};
}

// Values k0 .. k0+7 of one pixel's n channels (zero past n); VEC: n is a
// multiple of 8, one 16-byte load.
template <bool VEC>
__device__ inline u16x8 load8(const uint16_t* px, int k0, int n) {
  u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
  if constexpr (VEC) {
    if (k0 < n) v = *gl(reinterpret_cast<const u16x8*>(px + k0));
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = k0 + q < n ? gl(px)[k0 + q] : uint16_t{0};
  }
  return v;
}

constexpr int kWgTile = 32;        // pixels per unit
constexpr int kWgStride = 20;      // LDS row stride in 16-bit values
constexpr int kWgWaves = 4;
constexpr int kWgLdsPerWave = (kWgTile + 3 * (kWgTile + 2)) * kWgStride;  // 16-bit values
template <bool VX, bool VG>
__global__ __launch_bounds__(kWave* kWgWaves) void k_wgrad_tiles(const uint16_t* __restrict__ x,
                                                                  const uint16_t* __restrict__ gy, int H, int W,
                                                                  int C, int O, int64_t units, int groups,
                                                                  float* __restrict__ part) {
  __shared__ uint16_t lds[kWgWaves * kWgLdsPerWave];
  __shared__ float red[kWgWaves - 1][9][4][kWave];
  const int lane = lane_id(), g = lane / 16, m = lane % 16;
  const int ct = (C + 15) / 16;
  const int o0 = (blockIdx.x / ct) * 16, c0 = (blockIdx.x % ct) * 16;
  const int z = blockIdx.y;
  uint16_t* gs = lds + wave_id() * kWgLdsPerWave;  // [32][stride] output gradient
  uint16_t* xs = gs + kWgTile * kWgStride;         // [3][34][stride] input rows
  const int upr = W / kWgTile;                     // units per image row
  const int64_t u0 = units * z / groups, u1 = units * (z + 1) / groups;
  f32x4 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t u = u0 + wave_id(); u < u1; u += kWgWaves) {
    const int64_t row = u / upr;               // n * H + i
    const int i = static_cast<int>(row % H);
    const int x0 = static_cast<int>(u % upr) * kWgTile;
    // the output gradient's tile: lane = (pixel, half of the 16 channels)
    {
      const int px = lane >> 1, h8 = (lane & 1) * 8;
      store_lds8(gs + px * kWgStride + h8, load8<VG>(gy + (row * W + x0 + px) * O, o0 + h8, O));
    }
    // the input's three rows, pixels x0 - 1 .. x0 + 32
    for (int it = lane; it < 3 * (kWgTile + 2) * 2; it += kWave) {
      const int dy = it / ((kWgTile + 2) * 2), r = it % ((kWgTile + 2) * 2);
      const int pq = r >> 1, h8 = (r & 1) * 8;
      const int yy = i + dy - 1, xx = x0 + pq - 1;
      u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
      if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = load8<VX>(x + ((row - i + yy) * W + xx) * C, c0 + h8, C);
      store_lds8(xs + (dy * (kWgTile + 2) + pq) * kWgStride + h8, v);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    u16x8 a;
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = gs[(8 * g + q) * kWgStride + m];
    const bf16x8 av = as_bf16x8(a);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3, dx = t % 3;
      u16x8 b;
#pragma unroll
      for (int q = 0; q < 8; ++q) b[q] = xs[(dy * (kWgTile + 2) + 8 * g + q + dx) * kWgStride + m];
      acc[t] = mma(av, as_bf16x8(b), acc[t]);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the next unit overwrites the tiles
  }
  // the block's four tiles, added in wavefront order
  if (wave_id() > 0) {
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave_id() - 1][t][r][lane] = acc[t][r];
  }
  __syncthreads();
  if (wave_id() == 0) {
    const int c = c0 + m;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float s = acc[t][r];
        for (int w = 0; w < kWgWaves - 1; ++w) s += red[w][t][r][lane];
        const int o = o0 + 4 * g + r;
        if (o < O && c < C) glw(part)[((static_cast<int64_t>(z) * O + o) * 9 + t) * C + c] = s;
      }
    }
  }
}

// dst[e] += sum over groups z (in index order) of part[z][e], e < count.
__global__ void k_wgrad_reduce(const float* __restrict__ part, int groups, int64_t count, float* __restrict__ dst) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  float s = 0.0f;
  for (int z = 0; z < groups; ++z) s += gl(part)[static_cast<int64_t>(z) * count + e];
  dst[e] += s;
}

// The same sum with many groups and few elements: one block per element,
// thread t adding groups t, t + 256, ... in order, then the block's threads
// in a fixed tree.
constexpr int kReduceThreads = 256;
__global__ __launch_bounds__(kReduceThreads) void k_wgrad_reduce_wide(const float* __restrict__ part, int groups,
                                                                      int64_t count, float* __restrict__ dst) {
  __shared__ float red[kReduceThreads / kWave];
  const int64_t e = blockIdx.x;
  float s = 0.0f;
  for (int z = threadIdx.x; z < groups; z += kReduceThreads) s += gl(part)[static_cast<int64_t>(z) * count + e];
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < kReduceThreads / kWave; ++w) t += red[w];
    dst[e] += t;
  }
}

// dst[e] += the groups' partials of element e, by the kernel that suits the
// shape (both add in a fixed order).
void reduce_partials(const float* part, int groups, int64_t count, float* dst, hipStream_t st) {
  if (groups > 64 && count <= 65536)
    k_wgrad_reduce_wide<<<static_cast<unsigned>(count), kReduceThreads, 0, st>>>(part, groups, count, dst);
  else
    k_wgrad_reduce<<<static_cast<unsigned>((count + 255) / 256), 256, 0, st>>>(part, groups, count, dst);
}

// Partial bias gradients: part[blk][o] = sum over the block's `per`
// pixels of gy[p][o].  The block's threads cover floor(256 / O) pixels x O
// channels at a time (adjacent threads, adjacent values: coalesced); each
// thread sums its pixels in order, then the pixel lanes are added in order;
// k_wgrad_reduce adds the blocks in order.  O <= 256.
constexpr int kBiasThreads = 256;

// Pixels per bias block: about 512 blocks, between 64 and 4096 pixels.
inline int64_t bias_pix(int64_t P) { return std::min<int64_t>(4096, std::max<int64_t>(64, (P + 511) / 512)); }

__global__ __launch_bounds__(kBiasThreads) void k_bias_grad(const uint16_t* __restrict__ gy, int64_t P, int O,
                                                            int64_t per, float* __restrict__ part) {
  __shared__ float sums[kBiasThreads];
  const int lanes = kBiasThreads / O;  // pixels at a time
  const int t = threadIdx.x;
  const int o = t % O, j = t / O;
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t p1 = p0 + per < P ? p0 + per : P;
  float s = 0.0f;
  if (j < lanes)
    for (int64_t p = p0 + j; p < p1; p += lanes) s += bf2f(gl(gy)[p * O + o]);
  sums[t] = s;
  __syncthreads();
  if (t < O) {
    float r = 0.0f;
    for (int q = 0; q < lanes; ++q) r += sums[q * O + t];
    part[static_cast<int64_t>(blockIdx.x) * O + t] = r;
  }
}

// BF16 forward copy [O][9][Cp] and the flipped, transposed copy [C][9][Op]
// (w_bwd[c][tap][o] = w[o][8 - tap][c]) that turns the input gradient into a
// forward convolution.
__global__ void k_prep_weights(const float* __restrict__ w, int O, int C, int Op, int Cp, uint16_t* wf,
                               uint16_t* wb) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nf = static_cast<int64_t>(O) * 9 * Cp, nb = static_cast<int64_t>(C) * 9 * Op;
  if (t < nf) {
    const int c = static_cast<int>(t % Cp), tap = static_cast<int>((t / Cp) % 9), o = static_cast<int>(t / (9 * Cp));
    wf[t] = c < C ? f2bf(w[(static_cast<int64_t>(o) * 9 + tap) * C + c]) : uint16_t{0};
  }
  if (t < nb) {
    const int o = static_cast<int>(t % Op), tap = static_cast<int>((t / Op) % 9), c = static_cast<int>(t / (9 * Op));
    wb[t] = o < O ? f2bf(w[(static_cast<int64_t>(o) * 9 + (8 - tap)) * C + c]) : uint16_t{0};
  }
}

// out = bf16(g * [y > 0]) (y: the ReLU output), or bf16(g) when y is null.
__global__ void k_relu_mask(const float* __restrict__ g, const uint16_t* __restrict__ y, int64_t n,
                            uint16_t* __restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  float v = g[t];
  if (y && !(bf2f(y[t]) > 0.0f)) v = 0.0f;
  out[t] = f2bf(v);
}

// 2x2 average pool of an (H, W) map.
__global__ void k_pool2(const uint16_t* __restrict__ x, int64_t NHo, int H, int W, int C, uint16_t* __restrict__ y) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int Wo = W / 2, Ho = H / 2;
  if (t >= NHo * Wo * C) return;
  const int c = static_cast<int>(t % C);
  const int64_t pix = t / C;
  const int j = static_cast<int>(pix % Wo);
  const int64_t r = pix / Wo;  // n * Ho + i
  const int i = static_cast<int>(r % Ho);
  const int64_t n = r / Ho;
  const int64_t base = ((n * H + 2 * i) * W + 2 * j) * C + c;
  const float s = bf2f(x[base]) + bf2f(x[base + C]) + bf2f(x[base + static_cast<int64_t>(W) * C]) +
                  bf2f(x[base + static_cast<int64_t>(W) * C + C]);
  y[t] = f2bf(0.25f * s);
}

// gx (H, W map) (+)= gy[n, i/2, j/2, c] / 4
__global__ void k_pool2_grad(const float* __restrict__ gy, int64_t NH, int H, int W, int C, float* __restrict__ gx,
                             int accumulate) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= NH * W * C) return;
  const int c = static_cast<int>(t % C);
  const int64_t pix = t / C;
  const int j = static_cast<int>(pix % W);
  const int64_t r = pix / W;
  const int i = static_cast<int>(r % H);
  const int64_t n = r / H;
  const float v = 0.25f * gy[((n * (H / 2) + i / 2) * (W / 2) + j / 2) * C + c];
  gx[t] = accumulate ? gx[t] + v : v;
}

// y[n, i, j, coff + c] = x[n, i/2, j/2, c] for the (2H, 2W) map y of Ctot
// channels; with up = 0 the copy is at the same resolution.
__global__ void k_to_slice(const uint16_t* __restrict__ x, int64_t NHy, int Hy, int Wy, int C, int up,
                           uint16_t* __restrict__ y, int Ctot, int coff) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= NHy * Wy * C) return;
  const int c = static_cast<int>(t % C);
  const int64_t pix = t / C;
  const int j = static_cast<int>(pix % Wy);
  const int64_t r = pix / Wy;
  const int i = static_cast<int>(r % Hy);
  const int64_t n = r / Hy;
  int64_t src;
  if (up) src = ((n * (Hy / 2) + i / 2) * (Wy / 2) + j / 2) * C + c;
  else src = pix * C + c;
  y[pix * Ctot + coff + c] = x[src];
}

// gx (+)= the gradient of the slice [coff, coff + C) of gy (map Hy x Wy),
// summed over 2x2 blocks when the slice was upsampled.
__global__ void k_from_slice(const float* __restrict__ gy, int64_t NHx, int Hx, int Wx, int C, int up, int Ctot,
                             int coff, float* __restrict__ gx, int accumulate) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= NHx * Wx * C) return;
  const int c = static_cast<int>(t % C);
  const int64_t pix = t / C;
  float v;
  if (up) {
    const int j = static_cast<int>(pix % Wx);
    const int64_t r = pix / Wx;
    const int i = static_cast<int>(r % Hx);
    const int64_t n = r / Hx;
    const int Wy = 2 * Wx;
    const int64_t b = (n * 2 * Hx + 2 * i) * Wy + 2 * j;
    v = gy[b * Ctot + coff + c] + gy[(b + 1) * Ctot + coff + c] + gy[(b + Wy) * Ctot + coff + c] +
        gy[(b + Wy + 1) * Ctot + coff + c];
  } else {
    v = gy[pix * Ctot + coff + c];
  }
  gx[t] = accumulate ? gx[t] + v : v;
}

// out = x + r; g = 2 (out - target) / count; part[block] = the block's sum
// of (out - target)^2 (FP64), which k_loss_reduce adds to the loss in block
// order.
__global__ void k_residual_mse(const float* __restrict__ r, const float* __restrict__ x,
                               const float* __restrict__ target, int64_t n, float* __restrict__ out,
                               float* __restrict__ g, double* part) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double e2 = 0.0;
  if (t < n) {
    const float o = x[t] + r[t];
    out[t] = o;
    if (target) {
      const float d = o - target[t];
      if (g) g[t] = 2.0f * d / static_cast<float>(n);
      e2 = static_cast<double>(d) * d;
    }
  }
  if (target && part) {
    __shared__ double red[4];
    e2 = block_sum<4>(e2, red);
    if (threadIdx.x == 0) part[blockIdx.x] = e2;
  }
}

// loss += (sum of the blocks' partials, in block order) / n: one block.
__global__ void k_loss_reduce(const double* __restrict__ part, int64_t nblocks, int64_t n, double* loss) {
  __shared__ double red[4];
  double s = 0.0;
  const int64_t per = (nblocks + 255) / 256;
  const int64_t b0 = threadIdx.x * per, b1 = b0 + per < nblocks ? b0 + per : nblocks;
  for (int64_t b = b0; b < b1; ++b) s += part[b];
  s = block_sum<4>(s, red);
  if (threadIdx.x == 0) *loss += s / static_cast<double>(n);
}

__global__ void k_to_bf16(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ y) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) y[t] = f2bf(x[t]);
}

// Adam (Kingma & Ba) with bias correction, FP32 master weights.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.0f - b1) * gt;
  const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  w[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

// Vertical-snake vector (per image, nx*nz values) <-> image NHWC (1 channel).
__global__ void k_snake_image(const float* __restrict__ src, int64_t nimg, int nx, int nz, int to_image,
                              float* __restrict__ dst32, uint16_t* __restrict__ dst16) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t N = static_cast<int64_t>(nx) * nz;
  if (t >= nimg * N) return;
  const int64_t b = t / N, q = t % N;  // q = r * nx + c (image index)
  const int64_t r = q / nx, c = q % nx;
  const int64_t j = c * nz + ((c & 1) == 0 ? r : nz - 1 - r);
  if (to_image) {
    const float v = src[b * N + j];
    if (dst32) dst32[t] = v;
    if (dst16) dst16[t] = f2bf(v);
  } else {
    dst32[b * N + j] = src[t];
  }
}

inline unsigned blocks256(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace
}  // namespace ss

using namespace ss;

#define SS_NN_CHECK(cond, fn)                                                   \
  do {                                                                          \
    if (!(cond)) return fail(SS_E_ARG, "%s: bad argument (%s)", fn, #cond);     \
  } while (0)

extern "C" ss_status ss_nn_conv3x3(const void* x, int32_t N, int32_t H, int32_t W, int32_t C, const void* w,
                                   const float* bias, int32_t O, int32_t relu, void* y, int32_t y_f32,
                                   void* stream) {
  clear_error();
  SS_NN_CHECK(x && w && y && N > 0 && H > 0 && W > 0 && C > 0 && O > 0, "ss_nn_conv3x3");
  SS_NN_CHECK(static_cast<int64_t>(N) * H <= 65535, "ss_nn_conv3x3");
  const int Cp = (C + 7) / 8 * 8;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 block(kWave * kConvWaves);
  const unsigned gx = static_cast<unsigned>((W + 16 * kConvWaves - 1) / (16 * kConvWaves));
  const unsigned gy = static_cast<unsigned>(N) * H;
  const auto* xi = static_cast<const uint16_t*>(x);
  const auto* wi = static_cast<const uint16_t*>(w);
  if (C % 8 == 0 && Cp % 16 == 0) {  // operands staged in shared memory
    const int nt = O >= 64 ? 4 : (O > 16 ? 2 : 1);
    const dim3 grid(gx, gy, (O + 16 * nt - 1) / (16 * nt));
#define SS_CONV_T(NT, CC) k_conv3x3_t<NT, CC><<<grid, block, 0, st>>>(xi, H, W, C, Cp, wi, bias, O, relu, y, y_f32)
    // chunks of 32 channels where they divide the input and the tile is
    // narrow; 16 for 64-channel tiles, whose 32-channel chunk (50 KB of
    // shared memory) would leave room for 3 blocks per compute unit (with 16:
    // d3a 0.072 -> 0.058 ms, the 128-channel layers 0.042 -> 0.035 ms)
    if (Cp % 32 == 0 && nt != 4) {
      if (nt == 2) SS_CONV_T(2, 32);
      else SS_CONV_T(1, 32);
    } else {
      if (nt == 4) SS_CONV_T(4, 16);
      else if (nt == 2) SS_CONV_T(2, 16);
      else SS_CONV_T(1, 16);
    }
#undef SS_CONV_T
  } else if (O >= 64) {
    const dim3 grid(gx, gy, (O + 63) / 64);
    if (C % 8 == 0) k_conv3x3<4, true><<<grid, block, 0, st>>>(xi, H, W, C, Cp, wi, bias, O, relu, y, y_f32);
    else k_conv3x3<4, false><<<grid, block, 0, st>>>(xi, H, W, C, Cp, wi, bias, O, relu, y, y_f32);
  } else {
    const dim3 grid(gx, gy, (O + 15) / 16);
    if (C % 8 == 0) k_conv3x3<1, true><<<grid, block, 0, st>>>(xi, H, W, C, Cp, wi, bias, O, relu, y, y_f32);
    else k_conv3x3<1, false><<<grid, block, 0, st>>>(xi, H, W, C, Cp, wi, bias, O, relu, y, y_f32);
  }
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

// The weight gradient's partial groups: with the staged kernel (W a
// multiple of 32) enough block rows that the grid holds about 2048
// blocks, partials at most 4 MiB and each block at least 4 units; else one
// group per kWgradRows image rows.
bool wgrad_staged(int C, int O, int W) { return W % kWgTile == 0; }

int64_t wgrad_groups(int N, int H, int W, int C, int O) {
  if (!wgrad_staged(C, O, W)) return (static_cast<int64_t>(N) * H + kWgradRows - 1) / kWgradRows;
  const int64_t units = static_cast<int64_t>(N) * H * (W / kWgTile);
  const int64_t tiles = static_cast<int64_t>((O + 15) / 16) * ((C + 15) / 16);
  const int64_t by_blocks = (2048 + tiles - 1) / tiles;
  const int64_t by_bytes = std::max<int64_t>(1, (int64_t{4} << 20) / (static_cast<int64_t>(O) * 9 * C * 4));
  const int64_t by_units = std::max<int64_t>(1, units / (4 * kWgWaves));
  return std::max<int64_t>(1, std::min({by_blocks, by_bytes, by_units, int64_t{65535}}));
}

extern "C" ss_status ss_nn_wgrad_workspace_bytes(int32_t N, int32_t H, int32_t W, int32_t C, int32_t O,
                                                 size_t* bytes) {
  clear_error();
  SS_NN_CHECK(bytes && N > 0 && H > 0 && W > 0 && C > 0 && O > 0, "ss_nn_wgrad_workspace_bytes");
  const int64_t groups = wgrad_groups(N, H, W, C, O);
  const int64_t P = static_cast<int64_t>(N) * H * W;
  const int64_t pblocks = (P + bias_pix(P) - 1) / bias_pix(P);
  *bytes = sizeof(float) * static_cast<size_t>(std::max(groups * O * 9 * C, pblocks * O));
  return SS_OK;
}

extern "C" ss_status ss_nn_conv3x3_wgrad(const void* x, const void* gy, int32_t N, int32_t H, int32_t W, int32_t C,
                                         int32_t O, float* gw, float* gb, void* workspace, size_t workspace_bytes,
                                         void* stream) {
  clear_error();
  SS_NN_CHECK(x && gy && gw && workspace && N > 0 && H > 0 && W > 0 && C > 0 && O > 0 && (!gb || O <= 256),
              "ss_nn_conv3x3_wgrad");
  size_t need = 0;
  ss_nn_wgrad_workspace_bytes(N, H, W, C, O, &need);
  if (workspace_bytes < need) return fail(SS_E_WORKSPACE, "ss_nn_conv3x3_wgrad: workspace needs %zu bytes", need);
  const int Cp = (C + 7) / 8 * 8;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int NH = N * H;
  float* part = static_cast<float*>(workspace);
  const int groups = static_cast<int>(wgrad_groups(N, H, W, C, O));
  if (wgrad_staged(C, O, W)) {
    const int64_t units = static_cast<int64_t>(NH) * (W / kWgTile);
    const dim3 grid(((O + 15) / 16) * ((C + 15) / 16), groups);
    const auto* xi = static_cast<const uint16_t*>(x);
    const auto* gi = static_cast<const uint16_t*>(gy);
    const dim3 blk(kWave * kWgWaves);
    if (C % 8 == 0 && O % 8 == 0) k_wgrad_tiles<true, true><<<grid, blk, 0, st>>>(xi, gi, H, W, C, O, units, groups, part);
    else if (C % 8 == 0) k_wgrad_tiles<true, false><<<grid, blk, 0, st>>>(xi, gi, H, W, C, O, units, groups, part);
    else if (O % 8 == 0) k_wgrad_tiles<false, true><<<grid, blk, 0, st>>>(xi, gi, H, W, C, O, units, groups, part);
    else k_wgrad_tiles<false, false><<<grid, blk, 0, st>>>(xi, gi, H, W, C, O, units, groups, part);
  } else {
    const dim3 grid((O + 15) / 16, (9 * Cp + 15) / 16,
                    (NH + kWgradRows * kConvWaves - 1) / (kWgradRows * kConvWaves));
    k_conv3x3_wgrad<<<grid, kWave * kConvWaves, 0, st>>>(static_cast<const uint16_t*>(x),
                                                         static_cast<const uint16_t*>(gy), NH, H, W, C, Cp, O, part);
  }
  const int64_t nw = static_cast<int64_t>(O) * 9 * C;
  reduce_partials(part, groups, nw, gw, st);
  if (gb) {
    const int64_t P = static_cast<int64_t>(NH) * W;
    const int64_t per = bias_pix(P);
    const unsigned pb = static_cast<unsigned>((P + per - 1) / per);
    k_bias_grad<<<pb, kBiasThreads, 0, st>>>(static_cast<const uint16_t*>(gy), P, O, per, part);
    reduce_partials(part, static_cast<int>(pb), O, gb, st);
  }
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_nn_prep_weights(const float* w, int32_t O, int32_t C, void* w_fwd, void* w_bwd,
                                        void* stream) {
  clear_error();
  SS_NN_CHECK(w && w_fwd && w_bwd && O > 0 && C > 0, "ss_nn_prep_weights");
  const int Cp = (C + 7) / 8 * 8, Op = (O + 7) / 8 * 8;
  const int64_t n = std::max(static_cast<int64_t>(O) * 9 * Cp, static_cast<int64_t>(C) * 9 * Op);
  k_prep_weights<<<blocks256(n), 256, 0, static_cast<hipStream_t>(stream)>>>(
      w, O, C, Op, Cp, static_cast<uint16_t*>(w_fwd), static_cast<uint16_t*>(w_bwd));
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_nn_relu_mask(const float* g, const void* y, int64_t n, void* out, void* stream) {
  clear_error();
  SS_NN_CHECK(g && out && n > 0, "ss_nn_relu_mask");
  k_relu_mask<<<blocks256(n), 256, 0, static_cast<hipStream_t>(stream)>>>(g, static_cast<const uint16_t*>(y), n,
                                                                         static_cast<uint16_t*>(out));
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_nn_pool2(const void* x, int32_t N, int32_t H, int32_t W, int32_t C, void* y, void* stream) {
  clear_error();
  SS_NN_CHECK(x && y && N > 0 && H > 1 && W > 1 && C > 0 && H % 2 == 0 && W % 2 == 0, "ss_nn_pool2");
  const int64_t NHo = static_cast<int64_t>(N) * (H / 2);
  k_pool2<<<blocks256(NHo * (W / 2) * C), 256, 0, static_cast<hipStream_t>(stream)>>>(
      static_cast<const uint16_t*>(x), NHo, H, W, C, static_cast<uint16_t*>(y));
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_nn_pool2_grad(const float* gy, int32_t N, int32_t H, int32_t W, int32_t C, float* gx,
                                      int32_t accumulate, void* stream) {
  clear_error();
  SS_NN_CHECK(gy && gx && N > 0 && H % 2 == 0 && W % 2 == 0 && C > 0, "ss_nn_pool2_grad");
  const int64_t NH = static_cast<int64_t>(N) * H;
  k_pool2_grad<<<blocks256(NH * W * C), 256, 0, static_cast<hipStream_t>(stream)>>>(gy, NH, H, W, C, gx, accumulate);
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_nn_to_slice(const void* x, int32_t N, int32_t Hy, int32_t Wy, int32_t C, int32_t up,
                                    void* y, int32_t Ctot, int32_t coff, void* stream) {
  clear_error();
  SS_NN_CHECK(x && y && N > 0 && Hy > 0 && Wy > 0 && C > 0 && coff >= 0 && coff + C <= Ctot, "ss_nn_to_slice");
  SS_NN_CHECK(!up || (Hy % 2 == 0 && Wy % 2 == 0), "ss_nn_to_slice");
  const int64_t NHy = static_cast<int64_t>(N) * Hy;
  k_to_slice<<<blocks256(NHy * Wy * C), 256, 0, static_cast<hipStream_t>(stream)>>>(
      static_cast<const uint16_t*>(x), NHy, Hy, Wy, C, up, static_cast<uint16_t*>(y), Ctot, coff);
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_nn_from_slice(const float* gy, int32_t N, int32_t Hx, int32_t Wx, int32_t C, int32_t up,
                                      int32_t Ctot, int32_t coff, float* gx, int32_t accumulate, void* stream) {
  clear_error();
  SS_NN_CHECK(gy && gx && N > 0 && Hx > 0 && Wx > 0 && C > 0 && coff >= 0 && coff + C <= Ctot, "ss_nn_from_slice");
  const int64_t NHx = static_cast<int64_t>(N) * Hx;
  k_from_slice<<<blocks256(NHx * Wx * C), 256, 0, static_cast<hipStream_t>(stream)>>>(gy, NHx, Hx, Wx, C, up, Ctot,
                                                                                    coff, gx, accumulate);
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_nn_mse_workspace_bytes(int64_t n, size_t* bytes) {
  clear_error();
  SS_NN_CHECK(bytes && n > 0, "ss_nn_mse_workspace_bytes");
  *bytes = sizeof(double) * static_cast<size_t>(blocks256(n));
  return SS_OK;
}

extern "C" ss_status ss_nn_residual_mse(const float* r, const float* x, const float* target, int64_t n, float* out,
                                        float* g, double* loss, void* workspace, size_t workspace_bytes,
                                        void* stream) {
  clear_error();
  SS_NN_CHECK(r && x && out && n > 0, "ss_nn_residual_mse");
  const bool with_loss = target && loss;
  if (with_loss && (!workspace || workspace_bytes < sizeof(double) * blocks256(n)))
    return fail(SS_E_WORKSPACE, "ss_nn_residual_mse: workspace needs %zu bytes", sizeof(double) * blocks256(n));
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* part = with_loss ? static_cast<double*>(workspace) : nullptr;
  k_residual_mse<<<blocks256(n), 256, 0, st>>>(r, x, target, n, out, g, part);
  if (with_loss) k_loss_reduce<<<1, 256, 0, st>>>(part, blocks256(n), n, loss);
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_nn_to_bf16(const float* x, int64_t n, void* y, void* stream) {
  clear_error();
  SS_NN_CHECK(x && y && n > 0, "ss_nn_to_bf16");
  k_to_bf16<<<blocks256(n), 256, 0, static_cast<hipStream_t>(stream)>>>(x, n, static_cast<uint16_t*>(y));
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_nn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                                float b2, float eps, int32_t step, void* stream) {
  clear_error();
  SS_NN_CHECK(w && g && m && v && n > 0 && step > 0, "ss_nn_adam");
  const float c1 = 1.0f - powf(b1, static_cast<float>(step));
  const float c2 = 1.0f - powf(b2, static_cast<float>(step));
  k_adam<<<blocks256(n), 256, 0, static_cast<hipStream_t>(stream)>>>(w, g, m, v, n, lr, b1, b2, eps, c1, c2);
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}

extern "C" ss_status ss_nn_snake_image(const float* src, int64_t nimg, int32_t nx, int32_t nz, int32_t to_image,
                                       float* dst32, void* dst16, void* stream) {
  clear_error();
  SS_NN_CHECK(src && nimg > 0 && nx > 0 && nz > 0 && (dst32 || (to_image && dst16)), "ss_nn_snake_image");
  const int64_t n = nimg * nx * nz;
  k_snake_image<<<blocks256(n), 256, 0, static_cast<hipStream_t>(stream)>>>(src, nimg, nx, nz, to_image, dst32,
                                                                           static_cast<uint16_t*>(dst16));
  SS_HIP_TRY(hipGetLastError());
  return SS_OK;
}
