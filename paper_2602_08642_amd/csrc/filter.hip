// Gathering pyramidal filter on gfx950 (App. A): per pixel and level, one FP32 softmax
// over the concatenated kernel logits [kd | ku | kt] (eqs. app-softmax-mid/full), then
//   G: kd gather of L^l                     (eq. app-gather)
//   U: ku gather of the reconstructed coarser level around the parent (eq. app-upsample)
//   T: kt gather of the warped previous output, level 0 only (eq. app-recon-full)
// Neighbourhoods are staged in LDS with their halos (edge-clamped); each thread owns one
// output pixel and holds its logits in registers.
#include "filter_common.h"

using namespace aps;
using namespace aps::flt;

namespace {

__device__ inline float logit_value(float v) { return v; }
__device__ inline float logit_value(uint16_t v) { return bf2f(v); }
// the demodulation map d = exp(clamp(z, -8, 8)) (the same as aps_remodulate)
__device__ inline float demod_scale(float z) { return expf(fminf(fmaxf(z, -8.f), 8.f)); }

// DM: learned demodulation at this level (a.hist set); its kernels are separate instances so
// that the registers holding the map do not lower the occupancy of the others.
template <int KD, int KU, int KT, bool HU, bool HT, typename LT, bool DM>
__global__ __launch_bounds__(256) void k_level(LevelArgs a) {
  using G = Geo<KD, KU, KT, HU, HT>;
  constexpr int NK = G::NK;
  constexpr int VW = LogitVec<LT>::kW;
  constexpr int NKP = (NK + VW - 1) / VW * VW;
  __shared__ float4 Ls[G::LS];
  __shared__ float4 Cs[G::CS];
  __shared__ float4 Ts[G::PS];

  const int H = a.H, W = a.W;
  const int tid = threadIdx.x, tx = tid % TW, ty = tid / TW;
  const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH, n = blockIdx.z;
  const int x = x0 + tx, y = y0 + ty;
  const bool in = x < W && y < H;

  float z[NKP];
  // with learned demodulation, the map's three channels (and the four latents) of the same
  // logit row, loaded here so that the epilogue issues no load after its first store; bf16
  // values are kept packed two to a register until the end
  constexpr int DW = sizeof(LT) == 2 ? 2 : 4;  // registers for the map and for the latents
  uint32_t dz[DW] = {}, lz[DW] = {};
  if (in) {
    const LT* lp = static_cast<const LT*>(a.logits) + (((size_t)n * H + y) * W + x) * a.kstride;
    LogitVec<LT>::template load<NKP>(lp, z);
    if constexpr (DM) {
      auto grab = [&](int off, int cnt, uint32_t* r) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (c >= cnt) break;
          if constexpr (sizeof(LT) == 2) r[c / 2] |= (uint32_t)lp[off + c] << (16 * (c & 1));
          else r[c] = __builtin_bit_cast(uint32_t, lp[off + c]);
        }
      };
      grab(a.remod, 3, dz);
      if (a.lat) grab(a.lat_off, 4, lz);
    }
  }
  auto unpack = [](const uint32_t* r, int c) {
    if constexpr (sizeof(LT) == 2) return bf2f((uint16_t)(r[c / 2] >> (16 * (c & 1))));
    else return __builtin_bit_cast(float, r[c]);
  };
  stage_tiles<G>(a, Ls, Cs, Ts, x0, y0, n, HU, HT);
  __syncthreads();
  if (!in) return;

  float m = z[0];
#pragma unroll
  for (int k = 1; k < NK; ++k) m = fmaxf(m, z[k]);
  float sum = 0.f;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    z[k] = softmax_exp(z[k] - m);
    sum += z[k];
  }
  float ax = 0.f, ay = 0.f, az = 0.f;
  for_each_tap<KD, KU, KT, HU, HT>(a, Ls, Cs, Ts, tx, ty, x, y, x0, y0, [&](int k, float4 v) {
    ax += z[k] * v.x;
    ay += z[k] * v.y;
    az += z[k] * v.z;
  });
  const float inv = 1.f / sum;
  float4 o = make_float4(ax * inv, ay * inv, az * inv, 0.f);
  const size_t pix = ((size_t)n * H + y) * W + x;
  float4* dst = a.out + pix;
  if (a.accumulate) {
    const float4 p = *dst;
    o.x += p.x;
    o.y += p.y;
    o.z += p.z;
  }
  if constexpr (DM) {  // remodulation with the map loaded at the start
    a.hist[pix] = o;
    o.x *= demod_scale(unpack(dz, 0));
    o.y *= demod_scale(unpack(dz, 1));
    o.z *= demod_scale(unpack(dz, 2));
    if (a.lat) a.lat[pix] = make_float4(unpack(lz, 0), unpack(lz, 1), unpack(lz, 2), unpack(lz, 3));
  }
  *dst = o;
}

template <int KD, int KU, int KT, typename LT>
int launch_level_t(const LevelArgs& a, bool hu, bool ht, int N, hipStream_t st) {
  dim3 grid((a.W + TW - 1) / TW, (a.H + TH - 1) / TH, N);
  if (a.hist) {
    if (hu && ht) k_level<KD, KU, KT, true, true, LT, true><<<grid, 256, 0, st>>>(a);
    else if (hu) k_level<KD, KU, KT, true, false, LT, true><<<grid, 256, 0, st>>>(a);
    else if (ht) k_level<KD, KU, KT, false, true, LT, true><<<grid, 256, 0, st>>>(a);
    else k_level<KD, KU, KT, false, false, LT, true><<<grid, 256, 0, st>>>(a);
  } else {
    if (hu && ht) k_level<KD, KU, KT, true, true, LT, false><<<grid, 256, 0, st>>>(a);
    else if (hu) k_level<KD, KU, KT, true, false, LT, false><<<grid, 256, 0, st>>>(a);
    else if (ht) k_level<KD, KU, KT, false, true, LT, false><<<grid, 256, 0, st>>>(a);
    else k_level<KD, KU, KT, false, false, LT, false><<<grid, 256, 0, st>>>(a);
  }
  APS_LAUNCH_CHECK();
  return APS_OK;
}

template <typename LT>
int launch_level_d(const LevelArgs& a, int KD, int KU, int KT, bool hu, bool ht, int N,
                   hipStream_t st) {
  if (KD == 5 && KU == 3 && KT == 3) return launch_level_t<5, 3, 3, LT>(a, hu, ht, N, st);
  if (KD == 7 && KU == 3 && KT == 3) return launch_level_t<7, 3, 3, LT>(a, hu, ht, N, st);
  if (KD == 5 && KU == 2 && KT == 5) return launch_level_t<5, 2, 5, LT>(a, hu, ht, N, st);
  if (KD == 3 && KU == 3 && KT == 3) return launch_level_t<3, 3, 3, LT>(a, hu, ht, N, st);
  return APS_ERR_UNSUPPORTED;
}

}  // namespace

namespace aps {
namespace flt {
int launch_level(const LevelArgs& a, int dtype, int KD, int KU, int KT, bool hu, bool ht, int N,
                 hipStream_t st) {
  if (dtype == APS_F32) return launch_level_d<float>(a, KD, KU, KT, hu, ht, N, st);
  if (dtype == APS_BF16) return launch_level_d<uint16_t>(a, KD, KU, KT, hu, ht, N, st);
  return APS_ERR_UNSUPPORTED;
}
}  // namespace flt
}  // namespace aps

extern "C" {

size_t aps_denoise_pyramid_workspace_size(int N, int H, int W, int levels) {
  size_t b = 256;
  for (int l = 1; l < levels; ++l) b += (size_t)N * (H >> l) * (W >> l) * sizeof(float4);
  return b;
}

int aps_denoise_pyramid(const float* const* L, const void* const* logits, int logit_dtype,
                        const int* kstride, int levels, int KD, int KU, int KT,
                        const float* prev, const float* mv, int N, int H, int W, float* out,
                        void* ws, size_t ws_bytes, void* stream) {
  return aps_denoise_pyramid_ex(L, logits, logit_dtype, kstride, levels, KD, KU, KT, prev, mv, N, H,
                                W, -1, -1, out, nullptr, nullptr, ws, ws_bytes, stream);
}

int aps_denoise_pyramid_ex(const float* const* L, const void* const* logits, int logit_dtype,
                           const int* kstride, int levels, int KD, int KU, int KT,
                           const float* prev, const float* mv, int N, int H, int W,
                           int demod_offset, int lat_offset, float* out, float* out_demod,
                           float* lat_out, void* ws, size_t ws_bytes, void* stream) {
  if (levels < 1 || levels > APS_MAX_LEVELS) return APS_ERR_UNSUPPORTED;
  if (demod_offset >= 0 && (!out_demod || kstride == nullptr)) return APS_ERR_NULL;
  if (lat_out && (demod_offset < 0 || lat_offset < 0)) return APS_ERR_ARG;
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  const int div = 1 << (levels - 1);
  if (H % div || W % div) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!L || !logits || !kstride || !out) return APS_ERR_NULL;
  if (prev && !mv) return APS_ERR_NULL;
  if (levels > 1 && (!ws || ws_bytes < aps_denoise_pyramid_workspace_size(N, H, W, levels)))
    return APS_ERR_WORKSPACE;
  const bool temporal = prev != nullptr;
  for (int l = 0; l < levels; ++l) {
    if (!L[l] || !logits[l]) return APS_ERR_NULL;
    if (!kstride_ok(kstride[l], level_k(l, levels, KD, KU, KT, temporal), logit_dtype))
      return APS_ERR_SHAPE;
  }
  if (demod_offset >= 0 && kstride[0] < demod_offset + 3) return APS_ERR_SHAPE;
  if (lat_out && kstride[0] < lat_offset + 4) return APS_ERR_SHAPE;
  float4* tmp[APS_MAX_LEVELS] = {};
  char* wp = static_cast<char*>(ws);
  for (int l = 1; l < levels; ++l) {
    tmp[l] = reinterpret_cast<float4*>(wp);
    wp += (size_t)N * (H >> l) * (W >> l) * sizeof(float4);
  }
  hipStream_t st = as_stream(stream);
  for (int l = levels - 1; l >= 0; --l) {
    LevelArgs a{};
    a.L = reinterpret_cast<const float4*>(L[l]);
    a.logits = logits[l];
    a.kstride = kstride[l];
    a.coarse = l < levels - 1 ? tmp[l + 1] : nullptr;
    a.prev = reinterpret_cast<const float4*>(prev);
    a.mv = reinterpret_cast<const float2*>(mv);
    a.out = l == 0 ? reinterpret_cast<float4*>(out) : tmp[l];
    a.H = H >> l;
    a.W = W >> l;
    a.eval_g = 1;
    a.eval_u = l < levels - 1;
    a.eval_t = l == 0 && temporal;
    a.accumulate = 0;
    if (l == 0 && demod_offset >= 0) {
      a.hist = reinterpret_cast<float4*>(out_demod);
      a.remod = demod_offset;
      a.lat = reinterpret_cast<float4*>(lat_out);
      a.lat_off = lat_offset;
    }
    const int r = launch_level(a, logit_dtype, KD, KU, KT, l < levels - 1, l == 0 && temporal,
                               N, st);
    if (r != APS_OK) return r;
  }
  return APS_OK;
}

int aps_reproject(const float* prev, const float* mv, const void* logits0, int logit_dtype,
                  int kstride, int KD, int KU, int KT, int has_upsample, int N, int H, int W,
                  float* accum_out, void* stream) {
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!prev || !mv || !logits0 || !accum_out) return APS_ERR_NULL;
  if (has_upsample && (H % 2 || W % 2)) return APS_ERR_SHAPE;
  if (!kstride_ok(kstride, KD * KD + (has_upsample ? KU * KU : 0) + KT * KT, logit_dtype))
    return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  LevelArgs a{};
  a.logits = logits0;
  a.kstride = kstride;
  a.prev = reinterpret_cast<const float4*>(prev);
  a.mv = reinterpret_cast<const float2*>(mv);
  a.out = reinterpret_cast<float4*>(accum_out);
  a.H = H;
  a.W = W;
  a.eval_t = 1;
  a.accumulate = 1;
  return launch_level(a, logit_dtype, KD, KU, KT, has_upsample != 0, true, N, as_stream(stream));
}

int aps_upsample(const float* coarse, const void* logits, int logit_dtype, int kstride, int KD,
                 int KU, int KT, int has_temporal, int N, int H, int W, float* accum_out,
                 void* stream) {
  if (N < 0 || H < 0 || W < 0 || H % 2 || W % 2) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!coarse || !logits || !accum_out) return APS_ERR_NULL;
  if (!kstride_ok(kstride, KD * KD + KU * KU + (has_temporal ? KT * KT : 0), logit_dtype))
    return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  LevelArgs a{};
  a.logits = logits;
  a.kstride = kstride;
  a.coarse = reinterpret_cast<const float4*>(coarse);
  a.out = reinterpret_cast<float4*>(accum_out);
  a.H = H;
  a.W = W;
  a.eval_u = 1;
  a.accumulate = 1;
  return launch_level(a, logit_dtype, KD, KU, KT, true, has_temporal != 0, N, as_stream(stream));
}

}  // extern "C"
