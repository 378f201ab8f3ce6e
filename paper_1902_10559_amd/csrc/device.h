// Device-side helpers for gfx950 (CDNA4, 64-lane wavefronts).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ssart.h"

namespace ss {

constexpr int kWave = 64;

// Pointers that reach kernels through descriptor tables (or structs) are
// generic to the compiler, which then emits flat loads: those count against
// the same wait counter as scalar loads, so every wait for a descriptor
// field also drains all data loads in flight.  Casting to the global
// address space gives global loads and stores.
#define SS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ inline const SS_GLOBAL T* gl(const T* p) {
  return (const SS_GLOBAL T*)p;
}
template <typename T>
__device__ inline SS_GLOBAL T* glw(T* p) {
  return (SS_GLOBAL T*)p;
}

// FP32 pairs move as one 64-bit word (the vector class has no
// address-space-qualified copy operators).
__device__ inline uint64_t pack2(float a, float b) {
  return static_cast<uint64_t>(__float_as_uint(a)) | (static_cast<uint64_t>(__float_as_uint(b)) << 32);
}
__device__ inline float lo_f(uint64_t u) { return __uint_as_float(static_cast<uint32_t>(u)); }
__device__ inline float hi_f(uint64_t u) { return __uint_as_float(static_cast<uint32_t>(u >> 32)); }

__device__ inline int lane_id() { return static_cast<int>(threadIdx.x) & (kWave - 1); }
__device__ inline int wave_id() { return static_cast<int>(threadIdx.x) / kWave; }
__device__ inline uint64_t lanemask_lt() { return (uint64_t{1} << lane_id()) - 1; }

// Sum over groups of G adjacent lanes (G a power of two <= 64); every lane of
// a group ends with the group's sum.  Fixed butterfly order: deterministic.
template <int G>
__device__ inline float group_sum(float v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <int G>
__device__ inline double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Block-wide FP64 sum in a fixed order (wave butterflies, then waves in
// index order); the result is valid in thread 0.  `red` holds one double
// per wave.
template <int WPB>
__device__ inline double block_sum(double v, double* red) {
  v = group_sum<kWave>(v);
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < WPB; ++w) t += red[w];
  }
  return t;
}

// Round to nearest-even FP32 -> BF16 bits (NaN kept quiet).
__device__ inline uint32_t bf16_bits_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ inline uint32_t f16_bits_rne(float x) {
  return static_cast<uint32_t>(__half_as_ushort(__float2half_rn(x)));
}

// Round a value pair to storage type WT and store it at element k.
template <int WT>
__device__ inline void store_pair(void* base, int64_t k, float a, float b) {
  if constexpr (WT == SS_F32) {
    glw(reinterpret_cast<uint64_t*>(base))[k] = pack2(a, b);
  } else if constexpr (WT == SS_BF16) {
    glw(reinterpret_cast<uint32_t*>(base))[k] = bf16_bits_rne(a) | (bf16_bits_rne(b) << 16);
  } else {
    glw(reinterpret_cast<uint32_t*>(base))[k] = f16_bits_rne(a) | (f16_bits_rne(b) << 16);
  }
}

template <int WT>
__device__ inline void store_one(void* base, int64_t k, float a) {
  if constexpr (WT == SS_F32) {
    glw(reinterpret_cast<float*>(base))[k] = a;
  } else if constexpr (WT == SS_BF16) {
    glw(reinterpret_cast<uint16_t*>(base))[k] = static_cast<uint16_t>(bf16_bits_rne(a));
  } else {
    glw(reinterpret_cast<uint16_t*>(base))[k] = static_cast<uint16_t>(f16_bits_rne(a));
  }
}

// NV FP32 numbers: the two halves of the folded pair (NV = 2) or one system.
template <int NV>
struct Vec {
  float v[NV];
};

template <int NV>
__device__ inline Vec<NV> load_vec(const float* p, int64_t i) {
  Vec<NV> r;
  if constexpr (NV == 2) {
    const uint64_t u = gl(reinterpret_cast<const uint64_t*>(p))[i];
    r.v[0] = lo_f(u);
    r.v[1] = hi_f(u);
  } else {
    r.v[0] = gl(p)[i];
  }
  return r;
}

template <int NV>
__device__ inline void store_vec(float* p, int64_t i, const Vec<NV>& x) {
  if constexpr (NV == 2) {
    glw(reinterpret_cast<uint64_t*>(p))[i] = pack2(x.v[0], x.v[1]);
  } else {
    glw(p)[i] = x.v[0];
  }
}

// Matrix values of entry k widened to FP32.
template <int NV, int WT>
__device__ inline Vec<NV> load_vals(const void* base, int64_t k) {
  Vec<NV> r;
  if constexpr (NV == 2) {
    if constexpr (WT == SS_F32) {
      const uint64_t u = gl(reinterpret_cast<const uint64_t*>(base))[k];
      r.v[0] = lo_f(u);
      r.v[1] = hi_f(u);
    } else if constexpr (WT == SS_BF16) {
      const uint32_t u = gl(reinterpret_cast<const uint32_t*>(base))[k];
      r.v[0] = __uint_as_float(u << 16);
      r.v[1] = __uint_as_float(u & 0xffff0000u);
    } else {
      const uint32_t u = gl(reinterpret_cast<const uint32_t*>(base))[k];
      r.v[0] = __half2float(__ushort_as_half(static_cast<unsigned short>(u & 0xffffu)));
      r.v[1] = __half2float(__ushort_as_half(static_cast<unsigned short>(u >> 16)));
    }
  } else {
    if constexpr (WT == SS_F32) {
      r.v[0] = gl(reinterpret_cast<const float*>(base))[k];
    } else if constexpr (WT == SS_BF16) {
      r.v[0] = __uint_as_float(static_cast<uint32_t>(gl(reinterpret_cast<const uint16_t*>(base))[k]) << 16);
    } else {
      r.v[0] = __half2float(__ushort_as_half(gl(reinterpret_cast<const unsigned short*>(base))[k]));
    }
  }
  return r;
}

// Entries are streamed in aligned chunks of SS_CHUNK = 4 (one 16-byte load of
// indices, one or two of values): a quarter of the load instructions that
// entry-wise loads need, which is what bounds the solver kernels.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int WT>
__device__ inline float widen16(uint32_t bits) {
  if constexpr (WT == SS_BF16) return __uint_as_float(bits << 16);
  else return __half2float(__ushort_as_half(static_cast<unsigned short>(bits)));
}

// Indices of entries k0 .. k0+3 (k0 a multiple of 4).
__device__ inline u32x4 load_idx_chunk(const int32_t* idx, int64_t k0) {
  return gl(reinterpret_cast<const u32x4*>(idx))[k0 >> 2];
}

// Values of entries k0 .. k0+3 (k0 a multiple of 4) widened to FP32.
template <int NV, int WT>
__device__ inline void load_val_chunk(const void* base, int64_t k0, Vec<NV>* v) {
  if constexpr (NV == 2 && WT == SS_F32) {  // 8 bytes per entry: two loads
    const SS_GLOBAL u32x4* p = gl(reinterpret_cast<const u32x4*>(base)) + (k0 >> 1);
    const u32x4 a = p[0], b = p[1];
    v[0].v[0] = __uint_as_float(a.x);
    v[0].v[1] = __uint_as_float(a.y);
    v[1].v[0] = __uint_as_float(a.z);
    v[1].v[1] = __uint_as_float(a.w);
    v[2].v[0] = __uint_as_float(b.x);
    v[2].v[1] = __uint_as_float(b.y);
    v[3].v[0] = __uint_as_float(b.z);
    v[3].v[1] = __uint_as_float(b.w);
  } else if constexpr (NV == 2) {  // a 16-bit pair per entry
    const u32x4 a = gl(reinterpret_cast<const u32x4*>(base))[k0 >> 2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j].v[0] = widen16<WT>(a[j] & 0xffffu);
      v[j].v[1] = widen16<WT>(a[j] >> 16);
    }
  } else if constexpr (WT == SS_F32) {
    const u32x4 a = gl(reinterpret_cast<const u32x4*>(base))[k0 >> 2];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j].v[0] = __uint_as_float(a[j]);
  } else {  // one 16-bit value per entry: 8 bytes per chunk
    const u32x2 a = gl(reinterpret_cast<const u32x2*>(base))[k0 >> 2];
    v[0].v[0] = widen16<WT>(a.x & 0xffffu);
    v[1].v[0] = widen16<WT>(a.x >> 16);
    v[2].v[0] = widen16<WT>(a.y & 0xffffu);
    v[3].v[0] = widen16<WT>(a.y >> 16);
  }
}

// Loads of SS_CHUNK consecutive entries starting at any entry k (the
// interleaved stream form): 4-byte alignment is all the vector loads need.
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u32x4_a8 __attribute__((ext_vector_type(4), aligned(8)));

// (the address-space cast is written out: template deduction would drop the
// typedef's alignment)
__device__ inline u32x4 load_idx_at(const int32_t* idx, int64_t k) {
  return *(const SS_GLOBAL u32x4_a4*)(idx + k);
}

// Values of entries k .. k+3 widened to FP32; entries of at least 4 bytes
// (a pair, or one FP32 value).
template <int NV, int WT>
__device__ inline void load_val_at(const void* base, int64_t k, Vec<NV>* v) {
  static_assert(NV == 2 || WT == SS_F32, "entries of at least 4 bytes");
  if constexpr (NV == 2 && WT == SS_F32) {
    const SS_GLOBAL u32x4_a8* p = (const SS_GLOBAL u32x4_a8*)(reinterpret_cast<const uint64_t*>(base) + k);
    const u32x4 a = p[0], b = p[1];
    v[0].v[0] = __uint_as_float(a.x);
    v[0].v[1] = __uint_as_float(a.y);
    v[1].v[0] = __uint_as_float(a.z);
    v[1].v[1] = __uint_as_float(a.w);
    v[2].v[0] = __uint_as_float(b.x);
    v[2].v[1] = __uint_as_float(b.y);
    v[3].v[0] = __uint_as_float(b.z);
    v[3].v[1] = __uint_as_float(b.w);
  } else {
    const u32x4 a = *(const SS_GLOBAL u32x4_a4*)(reinterpret_cast<const uint32_t*>(base) + k);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (NV == 2) {
        v[j].v[0] = widen16<WT>(a[j] & 0xffffu);
        v[j].v[1] = widen16<WT>(a[j] >> 16);
      } else {
        v[j].v[0] = __uint_as_float(a[j]);
      }
    }
  }
}

}  // namespace ss

#define SS_HIP_TRY(expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ss::fail(SS_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)
