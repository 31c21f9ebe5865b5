// MFMA operand fragments and 8-element copies shared by the convolution kernels (conv.hip) and
// the fused sampler CNN (sampler_cnn.hip).  A fragment is one lane's 8 consecutive K elements of
// a 16x16 MFMA operand: bf16 feeds one v_mfma_f32_16x16x32_bf16, fp32 feeds eight
// v_mfma_f32_16x16x4f32 (element e of the four lane groups is one K = 4 step).
#pragma once
#include "aps_common.h"

namespace aps {

// raw copy (no conversion) for the direct / concat paths
__device__ inline void copy8(float* d, const float* s) {
  *reinterpret_cast<float4*>(d) = *reinterpret_cast<const float4*>(s);
  *reinterpret_cast<float4*>(d + 4) = *reinterpret_cast<const float4*>(s + 4);
}
__device__ inline void copy8(uint16_t* d, const uint16_t* s) {
  *reinterpret_cast<u16x8*>(d) = *reinterpret_cast<const u16x8*>(s);
}
__device__ inline void zero8(float* d) {
  *reinterpret_cast<float4*>(d) = make_float4(0.f, 0.f, 0.f, 0.f);
  *reinterpret_cast<float4*>(d + 4) = make_float4(0.f, 0.f, 0.f, 0.f);
}
__device__ inline void zero8(uint16_t* d) { *reinterpret_cast<u16x8*>(d) = u16x8{0, 0, 0, 0, 0, 0, 0, 0}; }

template <typename T>
struct Frag;
template <>
struct Frag<float> {
  float v[8];
};
template <>
struct Frag<uint16_t> {
  u16x8 v;
};

__device__ inline void frag_load(Frag<float>& f, const float* p) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  f.v[0] = a.x; f.v[1] = a.y; f.v[2] = a.z; f.v[3] = a.w;
  f.v[4] = b.x; f.v[5] = b.y; f.v[6] = b.z; f.v[7] = b.w;
}
__device__ inline void frag_load(Frag<uint16_t>& f, const uint16_t* p) {
  f.v = *reinterpret_cast<const u16x8*>(p);
}

__device__ inline f32x4 mma(const Frag<float>& a, const Frag<float>& b, f32x4 c) {
#pragma unroll
  for (int e = 0; e < 8; ++e) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[e], b.v[e], c, 0, 0, 0);
  return c;
}
__device__ inline f32x4 mma(const Frag<uint16_t>& a, const Frag<uint16_t>& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a.v),
                                                 __builtin_bit_cast(bf16x8, b.v), c, 0, 0, 0);
}

}  // namespace aps
