// Gathering pyramidal filter on gfx950 (App. A): per pixel and level, one FP32 softmax
// over the concatenated kernel logits [kd | ku | kt] (eqs. app-softmax-mid/full), then
//   G: kd gather of L^l                     (eq. app-gather)
//   U: ku gather of the reconstructed coarser level around the parent (eq. app-upsample)
//   T: kt gather of the warped previous output, level 0 only (eq. app-recon-full)
// Neighbourhoods are staged in LDS with their halos (edge-clamped); each thread owns one
// output pixel and holds its logits in registers.
#include "aps_common.h"

using namespace aps;

namespace {

constexpr int TW = 32, TH = 8;  // output tile (256 threads, one pixel each)

struct LevelArgs {
  const float4* L;      // level input [N, H, W]
  const void* logits;   // [N, H, W, kstride]
  int kstride;
  const float4* coarse; // reconstructed level l+1 [N, H/2, W/2]
  const float4* prev;   // previous output at level-0 resolution
  const float2* mv;
  float4* out;          // [N, H, W]
  int H, W;
  int eval_g, eval_u, eval_t, accumulate;
};

// Logits are read as whole 16-byte vectors: NKP = K rounded up to 4 (f32) or 8 (bf16)
// values, all inside the pixel's kstride (a multiple of the vector width).
template <typename LT>
struct LogitVec;
template <>
struct LogitVec<float> {
  static constexpr int kW = 4;
  template <int NKP>
  static __device__ inline void load(const float* p, float* z) {
#pragma unroll
    for (int k = 0; k < NKP; k += 4) {
      const float4 v = *reinterpret_cast<const float4*>(p + k);
      z[k] = v.x;
      z[k + 1] = v.y;
      z[k + 2] = v.z;
      z[k + 3] = v.w;
    }
  }
};
template <>
struct LogitVec<uint16_t> {
  static constexpr int kW = 8;
  template <int NKP>
  static __device__ inline void load(const uint16_t* p, float* z) {
#pragma unroll
    for (int k = 0; k < NKP; k += 8) {
      const u16x8 v = *reinterpret_cast<const u16x8*>(p + k);
#pragma unroll
      for (int e = 0; e < 8; ++e) z[k + e] = bf2f(v[e]);
    }
  }
};

__device__ inline float4 warp_at(const float4* __restrict__ prev, const float2* __restrict__ mv,
                                 int H, int W, int n, int x, int y) {
  const float2 m = mv[((size_t)n * H + y) * W + x];
  const float fxf = floorf(m.x), fyf = floorf(m.y);
  const float fx = m.x - fxf, fy = m.y - fyf;
  const int x0 = x + (int)fxf, y0 = y + (int)fyf;
  const int xa = min(max(x0, 0), W - 1), xb = min(max(x0 + 1, 0), W - 1);
  const int ya = min(max(y0, 0), H - 1), yb = min(max(y0 + 1, 0), H - 1);
  const float4* P = prev + (size_t)n * H * W;
  const float4 a = P[(size_t)ya * W + xa], b = P[(size_t)ya * W + xb];
  const float4 c = P[(size_t)yb * W + xa], d = P[(size_t)yb * W + xb];
  const float gx = 1.f - fx, gy = 1.f - fy;
  return make_float4(gy * (gx * a.x + fx * b.x) + fy * (gx * c.x + fx * d.x),
                     gy * (gx * a.y + fx * b.y) + fy * (gx * c.y + fx * d.y),
                     gy * (gx * a.z + fx * b.z) + fy * (gx * c.z + fx * d.z), 0.f);
}

template <int KD, int KU, int KT, bool HU, bool HT, typename LT>
__global__ __launch_bounds__(256) void k_level(LevelArgs a) {
  constexpr int RD = KD / 2, RT = KT / 2;
  constexpr int ND = KD * KD, NU = HU ? KU * KU : 0, NT = HT ? KT * KT : 0;
  constexpr int NK = ND + NU + NT;
  constexpr int VW = LogitVec<LT>::kW;
  constexpr int NKP = (NK + VW - 1) / VW * VW;
  constexpr int LW = TW + 2 * RD, LH = TH + 2 * RD;
  constexpr int CW = TW / 2 + 2, CH = TH / 2 + 2;
  constexpr int PW = TW + 2 * RT, PH = TH + 2 * RT;
  __shared__ float4 Ls[LH * LW];
  __shared__ float4 Cs[HU ? CH * CW : 1];
  __shared__ float4 Ts[HT ? PH * PW : 1];

  const int H = a.H, W = a.W;
  const int tid = threadIdx.x, tx = tid % TW, ty = tid / TW;
  const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH, n = blockIdx.z;
  const int x = x0 + tx, y = y0 + ty;
  const bool in = x < W && y < H;

  float z[NKP];
  if (in) {
    const LT* lp = static_cast<const LT*>(a.logits) + (((size_t)n * H + y) * W + x) * a.kstride;
    LogitVec<LT>::template load<NKP>(lp, z);
  }
  if (a.eval_g) {
    const float4* Ln = a.L + (size_t)n * H * W;
    for (int k = tid; k < LH * LW; k += 256) {
      const int r = k / LW, c = k % LW;
      const int yy = min(max(y0 - RD + r, 0), H - 1), xx = min(max(x0 - RD + c, 0), W - 1);
      Ls[k] = Ln[(size_t)yy * W + xx];
    }
  }
  const int cy0 = y0 / 2 - 1, cx0 = x0 / 2 - 1;
  if (HU && a.eval_u) {
    const int Hc = H / 2, Wc = W / 2;
    const float4* Cn = a.coarse + (size_t)n * Hc * Wc;
    for (int k = tid; k < CH * CW; k += 256) {
      const int r = k / CW, c = k % CW;
      const int yy = min(max(cy0 + r, 0), Hc - 1), xx = min(max(cx0 + c, 0), Wc - 1);
      Cs[k] = Cn[(size_t)yy * Wc + xx];
    }
  }
  if (HT && a.eval_t) {
    for (int k = tid; k < PH * PW; k += 256) {
      const int r = k / PW, c = k % PW;
      const int yy = min(max(y0 - RT + r, 0), H - 1), xx = min(max(x0 - RT + c, 0), W - 1);
      Ts[k] = warp_at(a.prev, a.mv, H, W, n, xx, yy);
    }
  }
  __syncthreads();
  if (!in) return;

  float m = z[0];
#pragma unroll
  for (int k = 1; k < NK; ++k) m = fmaxf(m, z[k]);
  float sum = 0.f;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    z[k] = expf(z[k] - m);
    sum += z[k];
  }
  float ax = 0.f, ay = 0.f, az = 0.f;
  if (a.eval_g) {
#pragma unroll
    for (int dy = -RD; dy <= RD; ++dy)
#pragma unroll
      for (int dx = -RD; dx <= RD; ++dx) {
        const float w = z[(dy + RD) * KD + (dx + RD)];
        const float4 v = Ls[(ty + RD + dy) * LW + (tx + RD + dx)];
        ax += w * v.x;
        ay += w * v.y;
        az += w * v.z;
      }
  }
  if (HU && a.eval_u) {
    if (KU == 2) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const float w = z[ND + j * 2 + i];
          const float4 v = Cs[((y + j) / 2 - cy0) * CW + ((x + i) / 2 - cx0)];
          ax += w * v.x;
          ay += w * v.y;
          az += w * v.z;
        }
    } else {
      constexpr int RU = KU / 2;
      const int py = y / 2 - cy0, px = x / 2 - cx0;
#pragma unroll
      for (int dy = -RU; dy <= RU; ++dy)
#pragma unroll
        for (int dx = -RU; dx <= RU; ++dx) {
          const float w = z[ND + (dy + RU) * KU + (dx + RU)];
          const float4 v = Cs[(py + dy) * CW + (px + dx)];
          ax += w * v.x;
          ay += w * v.y;
          az += w * v.z;
        }
    }
  }
  if (HT && a.eval_t) {
#pragma unroll
    for (int dy = -RT; dy <= RT; ++dy)
#pragma unroll
      for (int dx = -RT; dx <= RT; ++dx) {
        const float w = z[ND + NU + (dy + RT) * KT + (dx + RT)];
        const float4 v = Ts[(ty + RT + dy) * PW + (tx + RT + dx)];
        ax += w * v.x;
        ay += w * v.y;
        az += w * v.z;
      }
  }
  const float inv = 1.f / sum;
  float4 o = make_float4(ax * inv, ay * inv, az * inv, 0.f);
  float4* dst = a.out + ((size_t)n * H + y) * W + x;
  if (a.accumulate) {
    const float4 p = *dst;
    o.x += p.x;
    o.y += p.y;
    o.z += p.z;
  }
  *dst = o;
}

template <int KD, int KU, int KT, typename LT>
int launch_level_t(const LevelArgs& a, bool hu, bool ht, int N, hipStream_t st) {
  dim3 grid((a.W + TW - 1) / TW, (a.H + TH - 1) / TH, N);
  if (hu && ht) k_level<KD, KU, KT, true, true, LT><<<grid, 256, 0, st>>>(a);
  else if (hu) k_level<KD, KU, KT, true, false, LT><<<grid, 256, 0, st>>>(a);
  else if (ht) k_level<KD, KU, KT, false, true, LT><<<grid, 256, 0, st>>>(a);
  else k_level<KD, KU, KT, false, false, LT><<<grid, 256, 0, st>>>(a);
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

int launch_level(const LevelArgs& a, int dtype, int KD, int KU, int KT, bool hu, bool ht, int N,
                 hipStream_t st) {
  if (dtype == APS_F32) return launch_level_d<float>(a, KD, KU, KT, hu, ht, N, st);
  if (dtype == APS_BF16) return launch_level_d<uint16_t>(a, KD, KU, KT, hu, ht, N, st);
  return APS_ERR_UNSUPPORTED;
}

bool kstride_ok(int kstride, int K, int dtype) {
  const int vw = dtype == APS_BF16 ? 8 : 4;
  return kstride >= K && kstride % vw == 0;
}

int level_k(int l, int levels, int KD, int KU, int KT, bool temporal) {
  return KD * KD + (l < levels - 1 ? KU * KU : 0) + (l == 0 && temporal ? KT * KT : 0);
}

}  // namespace

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
  if (levels < 1 || levels > APS_MAX_LEVELS) return APS_ERR_UNSUPPORTED;
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
