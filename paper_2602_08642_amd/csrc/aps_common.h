// Internal device helpers shared by the gfx950 kernels of libaps (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/aps.h"

#define APS_HIP_TRY(expr)                                   \
  do {                                                      \
    if ((expr) != hipSuccess) return APS_ERR_HIP;           \
  } while (0)

#define APS_LAUNCH_CHECK()                                  \
  do {                                                      \
    if (hipGetLastError() != hipSuccess) return APS_ERR_HIP; \
  } while (0)

namespace aps {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct LevelPtrs {
  float4* p[APS_MAX_LEVELS];
};

static inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ---- bfloat16 <-> float (round to nearest even, NaN kept quiet) ------------------------
__device__ __host__ inline uint16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __host__ inline float bf2f(uint16_t h) {
  return __builtin_bit_cast(float, ((uint32_t)h) << 16);
}
// four floats -> four bf16 with the hardware packed conversion (round to nearest even)
__device__ inline u16x4 f2bf4(float a, float b, float c, float d) {
  typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
  return __builtin_bit_cast(u16x4, __builtin_convertvector(f32x4{a, b, c, d}, bf16x4_t));
}
template <typename T>
__device__ inline T f2t(float v);
template <>
__device__ inline float f2t<float>(float v) { return v; }
template <>
__device__ inline uint16_t f2t<uint16_t>(float v) { return f2bf(v); }

// ---- Philox4x32-10 (Salmon et al., SC'11) --------------------------------------------
__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    // one 32 x 32 -> 64-bit multiply (v_mad_u64_u32) gives both halves of a product
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                   (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// u in [0, 1 - 2^-24]: top 24 bits of word (pixel mod 4) of the block with counter
// (pixel div 4, frame, stream 0, 0); one block serves four consecutive pixels.
__device__ inline float u24(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }
__device__ inline uint4 uniform_block(uint64_t seed, uint32_t quad, uint32_t frame) {
  return philox4x32_10(make_uint4(quad, frame, 0u, 0u), (uint32_t)seed, (uint32_t)(seed >> 32));
}
__device__ inline float uniform24(uint64_t seed, uint32_t pixel, uint32_t frame) {
  const uint4 r = uniform_block(seed, pixel >> 2, frame);
  const uint32_t k = pixel & 3u;
  return u24(k == 0 ? r.x : k == 1 ? r.y : k == 2 ? r.z : r.w);
}

// u of the sampling step: Philox per pixel (tex == nullptr), or a T x T threshold texture
// tiled over each image with a toroidal offset (ox, oy) = (word0, word1) mod T of Philox with
// counter (image, frame, stream 2, 0): u = tex[(y + oy) mod T][(x + ox) mod T].
struct USource {
  const float* tex;
  uint32_t T, H, W;
};
__device__ inline float draw_u(const USource& us, uint64_t seed, uint32_t pixel, uint32_t frame) {
  if (!us.tex) return uniform24(seed, pixel, frame);
  const uint32_t hw = us.H * us.W;
  const uint32_t n = pixel / hw, r = pixel - n * hw;
  const uint32_t y = r / us.W, x = r - y * us.W;
  const uint4 w = philox4x32_10(make_uint4(n, frame, 2u, 0u), (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint32_t ox = w.x % us.T, oy = w.y % us.T;
  return us.tex[((y + oy) % us.T) * us.T + (x + ox) % us.T];
}

// ---- wave / block reductions (wave64) -------------------------------------------------
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_isum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// inclusive prefix sum within a wave64
__device__ inline int wave_iscan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ inline void status_or(uint32_t* st, uint32_t bits) {
  if (st) atomicOr(st, bits);
}

template <typename T> struct Ld;
template <> struct Ld<float> {
  static __device__ inline float get(const float* p, size_t i) { return p[i]; }
};
template <> struct Ld<uint16_t> {
  static __device__ inline float get(const uint16_t* p, size_t i) { return bf2f(p[i]); }
};

// Fused sampler CNN (conv.hip): x [N,H,W,C] (dtype), three 3x3 layers Cin->16 (ReLU) ->16 (ReLU)
// ->1 with packed weights w0..w2 and biases b0..b2, z [N,H,W] float32.  Returns an aps_status;
// APS_ERR_UNSUPPORTED when the shapes are not covered (the caller then runs the layers one by one).
int sampler_cnn(const void* x, int N, int H, int W, int C, int Cin, const void* w0, const float* b0,
                const void* w1, const float* b1, const void* w2, const float* b2, int dtype, float* z,
                hipStream_t st);

}  // namespace aps
