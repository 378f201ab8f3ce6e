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

// dst[e] += sum over groups z (in index order) of part[z][e], e < count.
__global__ void k_wgrad_reduce(const float* __restrict__ part, int groups, int64_t count, float* __restrict__ dst) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  float s = 0.0f;
  for (int z = 0; z < groups; ++z) s += gl(part)[static_cast<int64_t>(z) * count + e];
  dst[e] += s;
}

// Partial bias gradients: part[blk][o] = sum over the block's 256 pixels of
// gy[p][o] (in pixel order); k_wgrad_reduce adds the blocks in order.
constexpr int kBiasPix = 256;
__global__ void k_bias_grad(const uint16_t* __restrict__ gy, int64_t P, int O, float* __restrict__ part) {
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * kBiasPix;
  const int64_t p1 = p0 + kBiasPix < P ? p0 + kBiasPix : P;
  for (int o = threadIdx.x; o < O; o += blockDim.x) {
    float s = 0.0f;
    for (int64_t p = p0; p < p1; ++p) s += bf2f(gl(gy)[p * O + o]);
    part[static_cast<int64_t>(blockIdx.x) * O + o] = s;
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
  if (O >= 64) {
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

extern "C" ss_status ss_nn_wgrad_workspace_bytes(int32_t N, int32_t H, int32_t W, int32_t C, int32_t O,
                                                 size_t* bytes) {
  clear_error();
  SS_NN_CHECK(bytes && N > 0 && H > 0 && W > 0 && C > 0 && O > 0, "ss_nn_wgrad_workspace_bytes");
  const int64_t groups = (static_cast<int64_t>(N) * H + kWgradRows - 1) / kWgradRows;
  const int64_t pblocks = (static_cast<int64_t>(N) * H * W + kBiasPix - 1) / kBiasPix;
  *bytes = sizeof(float) * static_cast<size_t>(std::max(groups * O * 9 * C, pblocks * O));
  return SS_OK;
}

extern "C" ss_status ss_nn_conv3x3_wgrad(const void* x, const void* gy, int32_t N, int32_t H, int32_t W, int32_t C,
                                         int32_t O, float* gw, float* gb, void* workspace, size_t workspace_bytes,
                                         void* stream) {
  clear_error();
  SS_NN_CHECK(x && gy && gw && workspace && N > 0 && H > 0 && W > 0 && C > 0 && O > 0, "ss_nn_conv3x3_wgrad");
  size_t need = 0;
  ss_nn_wgrad_workspace_bytes(N, H, W, C, O, &need);
  if (workspace_bytes < need) return fail(SS_E_WORKSPACE, "ss_nn_conv3x3_wgrad: workspace needs %zu bytes", need);
  const int Cp = (C + 7) / 8 * 8;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int NH = N * H;
  float* part = static_cast<float*>(workspace);
  const int groups = (NH + kWgradRows - 1) / kWgradRows;
  const dim3 grid((O + 15) / 16, (9 * Cp + 15) / 16, (NH + kWgradRows * kConvWaves - 1) / (kWgradRows * kConvWaves));
  k_conv3x3_wgrad<<<grid, kWave * kConvWaves, 0, st>>>(static_cast<const uint16_t*>(x),
                                                       static_cast<const uint16_t*>(gy), NH, H, W, C, Cp, O, part);
  const int64_t nw = static_cast<int64_t>(O) * 9 * C;
  k_wgrad_reduce<<<blocks256(nw), 256, 0, st>>>(part, groups, nw, gw);
  if (gb) {
    const int64_t P = static_cast<int64_t>(NH) * W;
    const unsigned pb = static_cast<unsigned>((P + kBiasPix - 1) / kBiasPix);
    k_bias_grad<<<pb, 128, 0, st>>>(static_cast<const uint16_t*>(gy), P, O, part);
    k_wgrad_reduce<<<blocks256(O), 256, 0, st>>>(part, static_cast<int>(pb), O, gb);
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
