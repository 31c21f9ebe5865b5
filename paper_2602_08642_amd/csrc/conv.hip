// NHWC convolution (k = 1 or 3, zero padding) as an implicit GEMM on gfx950 MFMA:
//   M = output channels (16 per MFMA tile), N = pixels (a 16-pixel row segment per tile),
//   K = taps x input channels, walked in chunks of 32 channels.
// The input tile of a chunk, with its 1-pixel halo, is staged once in LDS and read by all
// taps; weights are pre-packed in MFMA fragment order and read straight into registers.
// bf16: v_mfma_f32_16x16x32_bf16 (fp32 accumulate).  f32: v_mfma_f32_16x16x4f32.
// Input transforms fused into the staging: 2x2 average pool of a finer tensor, or nearest
// 2x upsampling of a coarser tensor concatenated with a skip tensor (U-Net decoder).
// Epilogue: bias, optional ReLU, store (f32 or bf16).
#include "aps_common.h"

using namespace aps;

namespace {

constexpr int kChunk = 32;
constexpr int kMaxTM = 4;

struct ConvArgs {
  const void* x;
  const void* x2;
  int N, H, W;   // output (= conv input after the transform) size
  int Cx, C2, mode;
  const void* wp;
  const float* bias;
  int Cout, nchunk, ntx;
  void* y;
  int ldy, relu;
};

// ---- 8-element vectors of the storage type ---------------------------------------------
struct V8f {
  float v[8];
};

__device__ inline V8f load8(const float* p) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  return V8f{{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w}};
}
__device__ inline V8f load8(const uint16_t* p) {
  const u16x8 h = *reinterpret_cast<const u16x8*>(p);
  V8f r;
#pragma unroll
  for (int e = 0; e < 8; ++e) r.v[e] = bf2f(h[e]);
  return r;
}
__device__ inline void store8(float* p, const V8f& r) {
  *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
  *reinterpret_cast<float4*>(p + 4) = make_float4(r.v[4], r.v[5], r.v[6], r.v[7]);
}
__device__ inline void store8(uint16_t* p, const V8f& r) {
  u16x8 h;
#pragma unroll
  for (int e = 0; e < 8; ++e) h[e] = f2bf(r.v[e]);
  *reinterpret_cast<u16x8*>(p) = h;
}
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

// Stage channels [ci, ci+8) of input pixel (iy, ix) into LDS.
template <typename T>
__device__ inline void stage8(const ConvArgs& a, int n, int iy, int ix, int ci, T* dst) {
  const int Cin = a.Cx + a.C2;
  if (iy < 0 || iy >= a.H || ix < 0 || ix >= a.W || ci >= Cin) {
    zero8(dst);
    return;
  }
  const T* x = static_cast<const T*>(a.x);
  if (a.mode == APS_CONV_DIRECT) {
    copy8(dst, x + (((size_t)n * a.H + iy) * a.W + ix) * a.Cx + ci);
  } else if (a.mode == APS_CONV_POOL2) {
    const int W2 = 2 * a.W;
    const T* p = x + (((size_t)n * 2 * a.H + 2 * iy) * W2 + 2 * ix) * a.Cx + ci;
    const V8f q0 = load8(p), q1 = load8(p + a.Cx), q2 = load8(p + (size_t)W2 * a.Cx),
              q3 = load8(p + (size_t)W2 * a.Cx + a.Cx);
    V8f r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r.v[e] = ((q0.v[e] + q1.v[e]) + (q2.v[e] + q3.v[e])) * 0.25f;
    store8(dst, r);
  } else {  // APS_CONV_UP2_CAT
    if (ci < a.Cx) {
      const int Hh = a.H / 2, Wh = a.W / 2;
      copy8(dst, x + (((size_t)n * Hh + iy / 2) * Wh + ix / 2) * a.Cx + ci);
    } else {
      const T* x2 = static_cast<const T*>(a.x2);
      copy8(dst, x2 + (((size_t)n * a.H + iy) * a.W + ix) * a.C2 + (ci - a.Cx));
    }
  }
}

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

template <typename TO>
__device__ inline void store_out(TO* p, int ldy, int co0, int Cout, const float* v);
template <>
__device__ inline void store_out<float>(float* p, int ldy, int co0, int Cout, const float* v) {
  if ((ldy & 3) == 0 && co0 + 4 <= ldy) {
    *reinterpret_cast<float4*>(p + co0) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (co0 + q < Cout) p[co0 + q] = v[q];
  }
}
template <>
__device__ inline void store_out<uint16_t>(uint16_t* p, int ldy, int co0, int Cout, const float* v) {
  if ((ldy & 3) == 0 && co0 + 4 <= ldy) {
    *reinterpret_cast<u16x4*>(p + co0) = u16x4{f2bf(v[0]), f2bf(v[1]), f2bf(v[2]), f2bf(v[3])};
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (co0 + q < Cout) p[co0 + q] = f2bf(v[q]);
  }
}

template <typename T, typename TO, int KS, int TM, int TN>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
  constexpr int R = KS / 2;
  constexpr int TH = 4 * TN, TWp = 16;
  constexpr int SW = TWp + 2 * R, SH = TH + 2 * R;
  constexpr int PS = sizeof(T) == 2 ? 40 : 36;  // padded LDS pixel stride (elements)
  __shared__ __attribute__((aligned(16))) T Xs[SH * SW * PS];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tx0 = (blockIdx.x % a.ntx) * TWp, ty0 = (blockIdx.x / a.ntx) * TH;
  const int cob = blockIdx.y, n = blockIdx.z;
  const T* wp = static_cast<const T*>(a.wp);

  f32x4 acc[TM][TN];
#pragma unroll
  for (int m = 0; m < TM; ++m)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int c = 0; c < a.nchunk; ++c) {
    for (int it = tid; it < SH * SW * 4; it += 256) {
      const int g = it & 3, p = it >> 2;
      const int r = p / SW, col = p % SW;
      stage8<T>(a, n, ty0 - R + r, tx0 - R + col, c * kChunk + g * 8, Xs + p * PS + g * 8);
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < KS * KS; ++tap) {
      const int dy = tap / KS - R, dx = tap % KS - R;
      Frag<T> wf[TM];
#pragma unroll
      for (int m = 0; m < TM; ++m) {
        const size_t idx = ((((size_t)(cob * TM + m) * KS * KS + tap) * a.nchunk + c) * 64 + lane) * 8;
        frag_load(wf[m], wp + idx);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int row = wave * TN + j + R + dy, col = (lane & 15) + R + dx;
        Frag<T> bf;
        frag_load(bf, Xs + (row * SW + col) * PS + (lane >> 4) * 8);
#pragma unroll
        for (int m = 0; m < TM; ++m) acc[m][j] = mma(wf[m], bf, acc[m][j]);
      }
    }
    __syncthreads();
  }

  TO* y = static_cast<TO*>(a.y);
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int row = ty0 + wave * TN + j, col = tx0 + (lane & 15);
    if (row >= a.H || col >= a.W) continue;
    TO* py = y + (((size_t)n * a.H + row) * a.W + col) * a.ldy;
#pragma unroll
    for (int m = 0; m < TM; ++m) {
      const int co0 = (cob * TM + m) * 16 + 4 * (lane >> 4);
      if (co0 >= a.Cout) continue;
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float t = acc[m][j][q] + (co0 + q < a.Cout ? a.bias[co0 + q] : 0.f);
        v[q] = a.relu ? fmaxf(t, 0.f) : t;
      }
      store_out<TO>(py, a.ldy, co0, a.Cout, v);
    }
  }
}

// ---- weight packing: OHWI fp32 -> fragment order --------------------------------------
// packed[(((ct * KS*KS + tap) * nchunk + c) * 64 + lane) * 8 + e] =
//     w[co = 16 ct + lane % 16][tap][ci = 32 c + 8 (lane / 16) + e]   (0 outside)
template <typename T>
__global__ void k_pack(const float* __restrict__ w, int Cout, int KS, int Cin, int nchunk,
                       size_t total, T* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
  size_t r = i >> 9;
  const int c = (int)(r % nchunk);
  r /= nchunk;
  const int tap = (int)(r % (KS * KS));
  const int ct = (int)(r / (KS * KS));
  const int co = ct * 16 + (lane & 15), ci = c * kChunk + (lane >> 4) * 8 + e;
  float v = 0.f;
  if (co < Cout && ci < Cin) v = w[((size_t)co * KS * KS + tap) * Cin + ci];
  if constexpr (sizeof(T) == 2) out[i] = f2bf(v);
  else out[i] = v;
}

size_t packed_elems(int Cout, int KS, int Cin) {
  const size_t nct = (size_t)((Cout + 16 * kMaxTM - 1) / (16 * kMaxTM)) * kMaxTM;
  const size_t nchunk = (size_t)(Cin + kChunk - 1) / kChunk;
  return nct * KS * KS * nchunk * 512;
}

template <typename T, typename TO, int KS, int TM, int TN>
void launch_conv(const ConvArgs& a, hipStream_t st) {
  const int TH = 4 * TN;
  const int ntx = (a.W + 15) / 16, nty = (a.H + TH - 1) / TH;
  ConvArgs b = a;
  b.ntx = ntx;
  const int nco = (a.Cout + 16 * TM - 1) / (16 * TM);
  dim3 grid(ntx * nty, nco, a.N);
  k_conv<T, TO, KS, TM, TN><<<grid, 256, 0, st>>>(b);
}

template <typename T, typename TO, int KS>
void dispatch_tiles(const ConvArgs& a, hipStream_t st) {
  const bool big = (size_t)a.H * a.W >= 64 * 64;
  if (a.Cout <= 16) {
    if (big) launch_conv<T, TO, KS, 1, 4>(a, st); else launch_conv<T, TO, KS, 1, 2>(a, st);
  } else if (a.Cout <= 32) {
    if (big) launch_conv<T, TO, KS, 2, 4>(a, st); else launch_conv<T, TO, KS, 2, 2>(a, st);
  } else {
    if (big) launch_conv<T, TO, KS, 4, 4>(a, st); else launch_conv<T, TO, KS, 4, 2>(a, st);
  }
}

template <typename T, typename TO>
void dispatch_ks(const ConvArgs& a, int KS, hipStream_t st) {
  if (KS == 3) dispatch_tiles<T, TO, 3>(a, st);
  else dispatch_tiles<T, TO, 1>(a, st);
}

}  // namespace

extern "C" {

size_t aps_conv_packed_elems(int Cout, int ksize, int Cin) {
  if (Cout <= 0 || Cin <= 0 || (ksize != 1 && ksize != 3)) return 0;
  return packed_elems(Cout, ksize, Cin);
}

int aps_conv_pack_weights(const float* w, int Cout, int ksize, int Cin, int dtype, void* packed,
                          void* stream) {
  if (!w || !packed) return APS_ERR_NULL;
  if (Cout <= 0 || Cin <= 0) return APS_ERR_SHAPE;
  if (ksize != 1 && ksize != 3) return APS_ERR_UNSUPPORTED;
  const size_t total = packed_elems(Cout, ksize, Cin);
  const int nchunk = (Cin + kChunk - 1) / kChunk;
  const int blocks = (int)((total + 255) / 256);
  hipStream_t st = as_stream(stream);
  if (dtype == APS_F32)
    k_pack<float><<<blocks, 256, 0, st>>>(w, Cout, ksize, Cin, nchunk, total, static_cast<float*>(packed));
  else if (dtype == APS_BF16)
    k_pack<uint16_t><<<blocks, 256, 0, st>>>(w, Cout, ksize, Cin, nchunk, total,
                                             static_cast<uint16_t*>(packed));
  else
    return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_conv2d_fwd(const void* x, const void* x2, int N, int H, int W, int Cx, int C2, int mode,
                   const void* packed_w, const float* bias, int Cout, int ksize, int relu,
                   int dtype, void* y, int ldy, int y_dtype, void* stream) {
  if (N < 0 || H < 0 || W < 0 || Cx <= 0 || C2 < 0 || Cout <= 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!x || !packed_w || !bias || !y) return APS_ERR_NULL;
  if (ksize != 1 && ksize != 3) return APS_ERR_UNSUPPORTED;
  if (Cx % 8 || C2 % 8) return APS_ERR_UNSUPPORTED;
  if (ldy < Cout) return APS_ERR_SHAPE;
  if (mode == APS_CONV_UP2_CAT) {
    if (!x2 || C2 <= 0) return APS_ERR_NULL;
    if (H % 2 || W % 2) return APS_ERR_SHAPE;
  } else if (mode == APS_CONV_DIRECT || mode == APS_CONV_POOL2) {
    if (C2 != 0) return APS_ERR_SHAPE;
  } else {
    return APS_ERR_ARG;
  }
  if ((size_t)N * H * W == 0) return APS_OK;
  ConvArgs a{};
  a.x = x;
  a.x2 = x2;
  a.N = N;
  a.H = H;
  a.W = W;
  a.Cx = Cx;
  a.C2 = C2;
  a.mode = mode;
  a.wp = packed_w;
  a.bias = bias;
  a.Cout = Cout;
  a.nchunk = (Cx + C2 + kChunk - 1) / kChunk;
  a.y = y;
  a.ldy = ldy;
  a.relu = relu;
  hipStream_t st = as_stream(stream);
  if (dtype == APS_F32 && y_dtype == APS_F32) dispatch_ks<float, float>(a, ksize, st);
  else if (dtype == APS_BF16 && y_dtype == APS_BF16) dispatch_ks<uint16_t, uint16_t>(a, ksize, st);
  else if (dtype == APS_BF16 && y_dtype == APS_F32) dispatch_ks<uint16_t, float>(a, ksize, st);
  else return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

}  // extern "C"
