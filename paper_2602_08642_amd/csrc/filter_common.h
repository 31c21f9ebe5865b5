// Shared pieces of the gathering-pyramid kernels (forward and backward): tile geometry,
// logit loads, the edge-clamped bilinear warp, LDS staging of one output tile's
// neighbourhoods and the iteration over the kernel taps of one output pixel.
#pragma once
#include "aps_common.h"

namespace aps {
namespace flt {

constexpr int TW = 32, TH = 8;  // output tile (256 threads, one pixel each)

struct LevelArgs {
  const float4* L;       // level input [N, H, W]
  const void* logits;    // [N, H, W, kstride]
  int kstride;
  const float4* coarse;  // reconstructed level l+1 [N, H/2, W/2]
  const float4* prev;    // previous output at level-0 resolution
  const float2* mv;
  float4* out;           // [N, H, W]
  int H, W;
  int eval_g, eval_u, eval_t, accumulate;
  // learned demodulation (level 0): with hist set, the reconstruction o (of the demodulated
  // pyramid) is also written to hist and out = o * exp(clamp(z[remod .. remod + 2], -8, 8));
  // with lat set, the four latent channels z[lat_off .. lat_off + 3] are copied to lat
  float4* hist;
  int remod;
  float4* lat;
  int lat_off;
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

// Bilinear sample of prev at (x + mv.x, y + mv.y), both taps clamped to the edge; the integer
// cell comes from floor(mv), so the fractional weights are exact in binary32.
struct WarpTaps {
  int ya, yb, xa, xb;
  float gy, fy, gx, fx;  // weights (1 - fy), fy, (1 - fx), fx
};
__device__ inline WarpTaps warp_taps(float2 m, int H, int W, int x, int y) {
  const float fxf = floorf(m.x), fyf = floorf(m.y);
  WarpTaps t;
  t.fx = m.x - fxf;
  t.fy = m.y - fyf;
  t.gx = 1.f - t.fx;
  t.gy = 1.f - t.fy;
  const int x0 = x + (int)fxf, y0 = y + (int)fyf;
  t.xa = min(max(x0, 0), W - 1);
  t.xb = min(max(x0 + 1, 0), W - 1);
  t.ya = min(max(y0, 0), H - 1);
  t.yb = min(max(y0 + 1, 0), H - 1);
  return t;
}

__device__ inline float4 warp_at(const float4* __restrict__ prev, const float2* __restrict__ mv,
                                 int H, int W, int n, int x, int y) {
  const WarpTaps t = warp_taps(mv[((size_t)n * H + y) * W + x], H, W, x, y);
  const float4* P = prev + (size_t)n * H * W;
  const float4 a = P[(size_t)t.ya * W + t.xa], b = P[(size_t)t.ya * W + t.xb];
  const float4 c = P[(size_t)t.yb * W + t.xa], d = P[(size_t)t.yb * W + t.xb];
  return make_float4(t.gy * (t.gx * a.x + t.fx * b.x) + t.fy * (t.gx * c.x + t.fx * d.x),
                     t.gy * (t.gx * a.y + t.fx * b.y) + t.fy * (t.gx * c.y + t.fx * d.y),
                     t.gy * (t.gx * a.z + t.fx * b.z) + t.fy * (t.gx * c.z + t.fx * d.z), 0.f);
}

// e^x for x <= 0 (softmax numerators after the max subtraction) as one hardware exp2: the
// relative error is about (|x| + 1) 2^-23, below 1e-5 for the logit spreads that carry weight.
__device__ inline float softmax_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }

// Tile geometry of one level kernel instantiation.
template <int KD, int KU, int KT, bool HU, bool HT>
struct Geo {
  static constexpr int RD = KD / 2, RT = KT / 2, RU = KU / 2;
  static constexpr int ND = KD * KD, NU = HU ? KU * KU : 0, NT = HT ? KT * KT : 0;
  static constexpr int NK = ND + NU + NT;
  static constexpr int LW = TW + 2 * RD, LH = TH + 2 * RD;
  static constexpr int CW = TW / 2 + 2, CH = TH / 2 + 2;
  static constexpr int PW = TW + 2 * RT, PH = TH + 2 * RT;
  static constexpr int LS = LH * LW, CS = HU ? CH * CW : 1, PS = HT ? PH * PW : 1;
};

// Stage the tile's L^l (+ halo), coarse parents and warped history into LDS (edge-clamped).
template <class G>
__device__ inline void stage_tiles(const LevelArgs& a, float4* Ls, float4* Cs, float4* Ts, int x0,
                                   int y0, int n, bool hu, bool ht) {
  const int H = a.H, W = a.W, tid = threadIdx.x;
  if (a.eval_g) {
    const float4* Ln = a.L + (size_t)n * H * W;
    for (int k = tid; k < G::LS; k += 256) {
      const int r = k / G::LW, c = k % G::LW;
      const int yy = min(max(y0 - G::RD + r, 0), H - 1), xx = min(max(x0 - G::RD + c, 0), W - 1);
      Ls[k] = Ln[(size_t)yy * W + xx];
    }
  }
  if (hu && a.eval_u) {
    const int cy0 = y0 / 2 - 1, cx0 = x0 / 2 - 1;
    const int Hc = H / 2, Wc = W / 2;
    const float4* Cn = a.coarse + (size_t)n * Hc * Wc;
    for (int k = tid; k < G::CS; k += 256) {
      const int r = k / G::CW, c = k % G::CW;
      const int yy = min(max(cy0 + r, 0), Hc - 1), xx = min(max(cx0 + c, 0), Wc - 1);
      Cs[k] = Cn[(size_t)yy * Wc + xx];
    }
  }
  if (ht && a.eval_t) {
    for (int k = tid; k < G::PS; k += 256) {
      const int r = k / G::PW, c = k % G::PW;
      const int yy = min(max(y0 - G::RT + r, 0), H - 1), xx = min(max(x0 - G::RT + c, 0), W - 1);
      Ts[k] = warp_at(a.prev, a.mv, H, W, n, xx, yy);
    }
  }
}

// Call f(channel, value) for every evaluated tap of output pixel (x, y) (tile coords tx, ty).
template <int KD, int KU, int KT, bool HU, bool HT, class F>
__device__ inline void for_each_tap(const LevelArgs& a, const float4* Ls, const float4* Cs,
                                    const float4* Ts, int tx, int ty, int x, int y, int x0, int y0,
                                    F&& f) {
  using G = Geo<KD, KU, KT, HU, HT>;
  if (a.eval_g) {
#pragma unroll
    for (int dy = -G::RD; dy <= G::RD; ++dy)
#pragma unroll
      for (int dx = -G::RD; dx <= G::RD; ++dx)
        f((dy + G::RD) * KD + (dx + G::RD), Ls[(ty + G::RD + dy) * G::LW + (tx + G::RD + dx)]);
  }
  if (HU && a.eval_u) {
    const int cy0 = y0 / 2 - 1, cx0 = x0 / 2 - 1;
    if (KU == 2) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
          f(G::ND + j * 2 + i, Cs[((y + j) / 2 - cy0) * G::CW + ((x + i) / 2 - cx0)]);
    } else {
      const int py = y / 2 - cy0, px = x / 2 - cx0;
#pragma unroll
      for (int dy = -G::RU; dy <= G::RU; ++dy)
#pragma unroll
        for (int dx = -G::RU; dx <= G::RU; ++dx)
          f(G::ND + (dy + G::RU) * KU + (dx + G::RU), Cs[(py + dy) * G::CW + (px + dx)]);
    }
  }
  if (HT && a.eval_t) {
#pragma unroll
    for (int dy = -G::RT; dy <= G::RT; ++dy)
#pragma unroll
      for (int dx = -G::RT; dx <= G::RT; ++dx)
        f(G::ND + G::NU + (dy + G::RT) * KT + (dx + G::RT),
          Ts[(ty + G::RT + dy) * G::PW + (tx + G::RT + dx)]);
  }
}

inline bool kstride_ok(int kstride, int K, int dtype) {
  const int vw = dtype == APS_BF16 ? 8 : 4;
  return kstride >= K && kstride % vw == 0;
}

inline int level_k(int l, int levels, int KD, int KU, int KT, bool temporal) {
  return KD * KD + (l < levels - 1 ? KU * KU : 0) + (l == 0 && temporal ? KT * KT : 0);
}

// forward level launch (filter.hip); used by the backward's level recomputation
int launch_level(const LevelArgs& a, int dtype, int KD, int KU, int KT, bool hu, bool ht, int N,
                 hipStream_t st);

}  // namespace flt
}  // namespace aps
