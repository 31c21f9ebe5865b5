// Backward of the gathering pyramidal filter (App. A), hand-written for gfx950.
//
// Forward per output pixel q of level l:  y_q = sum_k w_qk v_qk,  w_q = softmax(z_q) over the
// joint [kd | ku | kt] block (eqs. app-softmax-mid/full), v_qk the gathered value of tap k.
//   dLoss/dz_qk  = w_qk (<g_q, v_qk> - <g_q, y_q>)           (softmax Jacobian)
//   dLoss/dv_qk  = w_qk g_q, routed back to the pixel tap k read:
//     kd taps -> L^l            (eq. app-gather, edge-clamped)
//     ku taps -> Lhat^{l+1}     (eq. app-upsample), which is the output of level l+1
//     kt taps -> W(prev)        (eq. app-recon-full) and through the bilinear warp to prev.
// The coarser reconstructed levels are recomputed with the forward kernel, not stored; the
// pass then runs fine-to-coarse, level l handing dLoss/dLhat^{l+1} to level l+1.
// The transposes are gathers over the clamped preimages of each input pixel (deterministic);
// only the warp's bilinear splat into prev uses atomics.
#include "filter_common.h"

using namespace aps;
using namespace aps::flt;

namespace {

struct BwdArgs {
  LevelArgs f;          // forward inputs of the level (f.out unused)
  const float4* gout;   // dLoss/dLhat^l [N, H, W]
  void* glogits;        // [N, H, W, gstride] in the gradient dtype
  int gstride;
  float* wbuf;          // [N, H, W, NK] normalised weights for the transposes
};

__device__ inline void gstore(float* p, float v) { *p = v; }
__device__ inline void gstore(uint16_t* p, float v) { *p = f2bf(v); }

template <int KD, int KU, int KT, bool HU, bool HT, typename LT, typename GT>
__global__ __launch_bounds__(256) void k_level_bwd(BwdArgs b) {
  const LevelArgs& a = b.f;
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
  const size_t pix = ((size_t)n * H + y) * W + x;

  float z[NKP];
  if (in) LogitVec<LT>::template load<NKP>(static_cast<const LT*>(a.logits) + pix * a.kstride, z);
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
  const float inv = 1.f / sum;
#pragma unroll
  for (int k = 0; k < NK; ++k) z[k] *= inv;
  float yx = 0.f, yy = 0.f, yz = 0.f;
  for_each_tap<KD, KU, KT, HU, HT>(a, Ls, Cs, Ts, tx, ty, x, y, x0, y0, [&](int k, float4 v) {
    yx += z[k] * v.x;
    yy += z[k] * v.y;
    yz += z[k] * v.z;
  });
  const float4 g = b.gout[pix];
  const float gy = g.x * yx + g.y * yy + g.z * yz;
  GT* gl = static_cast<GT*>(b.glogits) + pix * b.gstride;
  for_each_tap<KD, KU, KT, HU, HT>(a, Ls, Cs, Ts, tx, ty, x, y, x0, y0, [&](int k, float4 v) {
    gstore(gl + k, z[k] * (g.x * v.x + g.y * v.y + g.z * v.z - gy));
  });
  // blocks of the joint softmax whose term is not part of this output (the standalone
  // reproject and upsample terms): only their share of the normalisation, -w_k <g, y>
  if (!a.eval_g) {
#pragma unroll
    for (int k = 0; k < G::ND; ++k) gstore(gl + k, -z[k] * gy);
  }
  if (HU && !a.eval_u) {
#pragma unroll
    for (int k = G::ND; k < G::ND + G::NU; ++k) gstore(gl + k, -z[k] * gy);
  }
  if (HT && !a.eval_t) {
#pragma unroll
    for (int k = G::ND + G::NU; k < NK; ++k) gstore(gl + k, -z[k] * gy);
  }
  for (int k = NK; k < b.gstride; ++k) gstore(gl + k, 0.f);
  float* wb = b.wbuf + pix * NK;
#pragma unroll
  for (int k = 0; k < NK; ++k) wb[k] = z[k];
}

// Sum over the edge-clamped K x K same-resolution preimages of pixel (x, y):
// acc = sum_{tap (dy,dx), q : clamp(q + d) == (x, y)} wbuf[q][koff + tap] * g[q]
template <int K>
__device__ inline float4 gather_same_T(const float* __restrict__ wbuf, int nk, int koff,
                                       const float4* __restrict__ g, int H, int W, int n, int x,
                                       int y) {
  constexpr int R = K / 2;
  float ax = 0.f, ay = 0.f, az = 0.f;
  for (int dy = -R; dy <= R; ++dy) {
    for (int qy = y - R; qy <= y + R; ++qy) {
      if (qy < 0 || qy >= H || min(max(qy + dy, 0), H - 1) != y) continue;
      for (int dx = -R; dx <= R; ++dx) {
        for (int qx = x - R; qx <= x + R; ++qx) {
          if (qx < 0 || qx >= W || min(max(qx + dx, 0), W - 1) != x) continue;
          const size_t q = ((size_t)n * H + qy) * W + qx;
          const float w = wbuf[q * nk + koff + (dy + R) * K + (dx + R)];
          const float4 gq = g[q];
          ax += w * gq.x;
          ay += w * gq.y;
          az += w * gq.z;
        }
      }
    }
  }
  return make_float4(ax, ay, az, 0.f);
}

template <int K>
__global__ __launch_bounds__(256) void k_gatherT_same(const float* __restrict__ wbuf, int nk,
                                                      int koff, const float4* __restrict__ g,
                                                      int N, int H, int W, float4* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)N * H * W) return;
  const int x = (int)(i % W), y = (int)((i / W) % H), n = (int)(i / ((size_t)W * H));
  out[i] = gather_same_T<K>(wbuf, nk, koff, g, H, W, n, x, y);
}

// Coarse source index of fine pixel q for upsampling tap t (0 .. KU-1) on one axis.
template <int KU>
__device__ inline int up_src(int q, int t, int nc) {
  if (KU == 2) return min((q + t) / 2, nc - 1);
  return min(max(q / 2 + t - KU / 2, 0), nc - 1);
}

// dLoss/dLhat^{l+1}[P] = sum over fine q and ku taps reading P of w[q][koff+tap] * g[q]
template <int KU>
__global__ __launch_bounds__(256) void k_gatherT_up(const float* __restrict__ wbuf, int nk,
                                                    int koff, const float4* __restrict__ g, int N,
                                                    int Hf, int Wf, float4* __restrict__ outc) {
  const int Hc = Hf / 2, Wc = Wf / 2;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)N * Hc * Wc) return;
  const int X = (int)(i % Wc), Y = (int)((i / Wc) % Hc), n = (int)(i / ((size_t)Wc * Hc));
  float ax = 0.f, ay = 0.f, az = 0.f;
  for (int ty = 0; ty < KU; ++ty) {
    for (int qy = 2 * Y - 2; qy <= 2 * Y + 3; ++qy) {
      if (qy < 0 || qy >= Hf || up_src<KU>(qy, ty, Hc) != Y) continue;
      for (int tx = 0; tx < KU; ++tx) {
        for (int qx = 2 * X - 2; qx <= 2 * X + 3; ++qx) {
          if (qx < 0 || qx >= Wf || up_src<KU>(qx, tx, Wc) != X) continue;
          const size_t q = ((size_t)n * Hf + qy) * Wf + qx;
          const float w = wbuf[q * nk + koff + ty * KU + tx];
          const float4 gq = g[q];
          ax += w * gq.x;
          ay += w * gq.y;
          az += w * gq.z;
        }
      }
    }
  }
  outc[i] = make_float4(ax, ay, az, 0.f);
}

// kt taps: dLoss/dW(prev) by the same-resolution transpose, then the bilinear warp's
// transpose splatted into grad_prev (float atomics; summation order is not fixed).
template <int KT>
__global__ __launch_bounds__(256) void k_gatherT_warp(const float* __restrict__ wbuf, int nk,
                                                      int koff, const float4* __restrict__ g,
                                                      const float2* __restrict__ mv, int N, int H,
                                                      int W, float* __restrict__ grad_prev) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)N * H * W) return;
  const int x = (int)(i % W), y = (int)((i / W) % H), n = (int)(i / ((size_t)W * H));
  const float4 gw = gather_same_T<KT>(wbuf, nk, koff, g, H, W, n, x, y);
  const WarpTaps t = warp_taps(mv[i], H, W, x, y);
  float* P = grad_prev + (size_t)n * H * W * 4;
  const int idx[4] = {t.ya * W + t.xa, t.ya * W + t.xb, t.yb * W + t.xa, t.yb * W + t.xb};
  const float wt[4] = {t.gy * t.gx, t.gy * t.fx, t.fy * t.gx, t.fy * t.fx};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (wt[k] == 0.f) continue;
    float* d = P + (size_t)idx[k] * 4;
    atomicAdd(d + 0, wt[k] * gw.x);
    atomicAdd(d + 1, wt[k] * gw.y);
    atomicAdd(d + 2, wt[k] * gw.z);
  }
}

template <int KD, int KU, int KT, typename LT, typename GT>
int launch_bwd_t(const BwdArgs& b, bool hu, bool ht, int N, hipStream_t st) {
  dim3 grid((b.f.W + TW - 1) / TW, (b.f.H + TH - 1) / TH, N);
  if (hu && ht) k_level_bwd<KD, KU, KT, true, true, LT, GT><<<grid, 256, 0, st>>>(b);
  else if (hu) k_level_bwd<KD, KU, KT, true, false, LT, GT><<<grid, 256, 0, st>>>(b);
  else if (ht) k_level_bwd<KD, KU, KT, false, true, LT, GT><<<grid, 256, 0, st>>>(b);
  else k_level_bwd<KD, KU, KT, false, false, LT, GT><<<grid, 256, 0, st>>>(b);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

template <int KD, int KU, int KT>
int launch_bwd_k(const BwdArgs& b, int ldt, int gdt, bool hu, bool ht, int N, hipStream_t st) {
  if (ldt == APS_F32 && gdt == APS_F32) return launch_bwd_t<KD, KU, KT, float, float>(b, hu, ht, N, st);
  if (ldt == APS_BF16 && gdt == APS_BF16)
    return launch_bwd_t<KD, KU, KT, uint16_t, uint16_t>(b, hu, ht, N, st);
  if (ldt == APS_BF16 && gdt == APS_F32)
    return launch_bwd_t<KD, KU, KT, uint16_t, float>(b, hu, ht, N, st);
  return APS_ERR_UNSUPPORTED;
}

int launch_bwd(const BwdArgs& b, int ldt, int gdt, int KD, int KU, int KT, bool hu, bool ht, int N,
               hipStream_t st) {
  if (KD == 5 && KU == 3 && KT == 3) return launch_bwd_k<5, 3, 3>(b, ldt, gdt, hu, ht, N, st);
  if (KD == 7 && KU == 3 && KT == 3) return launch_bwd_k<7, 3, 3>(b, ldt, gdt, hu, ht, N, st);
  if (KD == 5 && KU == 2 && KT == 5) return launch_bwd_k<5, 2, 5>(b, ldt, gdt, hu, ht, N, st);
  if (KD == 3 && KU == 3 && KT == 3) return launch_bwd_k<3, 3, 3>(b, ldt, gdt, hu, ht, N, st);
  return APS_ERR_UNSUPPORTED;
}

template <int K>
void launch_same_T(const float* wbuf, int nk, int koff, const float4* g, int N, int H, int W,
                   float4* out, hipStream_t st) {
  const size_t n = (size_t)N * H * W;
  k_gatherT_same<K><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(wbuf, nk, koff, g, N, H, W, out);
}

int launch_same_T_k(int K, const float* wbuf, int nk, int koff, const float4* g, int N, int H,
                    int W, float4* out, hipStream_t st) {
  if (K == 3) launch_same_T<3>(wbuf, nk, koff, g, N, H, W, out, st);
  else if (K == 5) launch_same_T<5>(wbuf, nk, koff, g, N, H, W, out, st);
  else if (K == 7) launch_same_T<7>(wbuf, nk, koff, g, N, H, W, out, st);
  else return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int launch_up_T(int KU, const float* wbuf, int nk, int koff, const float4* g, int N, int Hf, int Wf,
                float4* outc, hipStream_t st) {
  const size_t n = (size_t)N * (Hf / 2) * (Wf / 2);
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (KU == 3) k_gatherT_up<3><<<blocks, 256, 0, st>>>(wbuf, nk, koff, g, N, Hf, Wf, outc);
  else if (KU == 2) k_gatherT_up<2><<<blocks, 256, 0, st>>>(wbuf, nk, koff, g, N, Hf, Wf, outc);
  else return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int launch_warp_T(int KT, const float* wbuf, int nk, int koff, const float4* g, const float2* mv,
                  int N, int H, int W, float* gprev, hipStream_t st) {
  const size_t n = (size_t)N * H * W;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (KT == 3) k_gatherT_warp<3><<<blocks, 256, 0, st>>>(wbuf, nk, koff, g, mv, N, H, W, gprev);
  else if (KT == 5) k_gatherT_warp<5><<<blocks, 256, 0, st>>>(wbuf, nk, koff, g, mv, N, H, W, gprev);
  else return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

size_t aps_denoise_pyramid_bwd_workspace_size(int N, int H, int W, int levels, int KD, int KU,
                                              int KT, int temporal) {
  size_t b = 256;
  for (int l = 1; l < levels; ++l) b += 2 * align256((size_t)N * (H >> l) * (W >> l) * sizeof(float4));
  const int nk0 = level_k(0, levels, KD, KU, KT, temporal != 0);
  b += align256((size_t)N * H * W * nk0 * sizeof(float));
  return b;
}

int aps_denoise_pyramid_bwd(const float* const* L, const void* const* logits, int logit_dtype,
                            const int* kstride, int levels, int KD, int KU, int KT,
                            const float* prev, const float* mv, int N, int H, int W,
                            const float* grad_out, void* const* grad_logits, int grad_dtype,
                            const int* gstride, float* const* grad_L, float* grad_prev, void* ws,
                            size_t ws_bytes, void* stream) {
  if (levels < 1 || levels > APS_MAX_LEVELS) return APS_ERR_UNSUPPORTED;
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  const int div = 1 << (levels - 1);
  if (H % div || W % div) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!L || !logits || !kstride || !grad_out || !grad_logits || !gstride || !grad_L)
    return APS_ERR_NULL;
  if (prev && !mv) return APS_ERR_NULL;
  if (grad_dtype != APS_F32 && grad_dtype != APS_BF16) return APS_ERR_UNSUPPORTED;
  const bool temporal = prev != nullptr;
  for (int l = 0; l < levels; ++l) {
    if (!L[l] || !logits[l] || !grad_logits[l] || !grad_L[l]) return APS_ERR_NULL;
    const int K = level_k(l, levels, KD, KU, KT, temporal);
    if (!kstride_ok(kstride[l], K, logit_dtype) || gstride[l] < K) return APS_ERR_SHAPE;
  }
  if (!ws || ws_bytes < aps_denoise_pyramid_bwd_workspace_size(N, H, W, levels, KD, KU, KT, temporal))
    return APS_ERR_WORKSPACE;
  char* wp = static_cast<char*>(ws);
  float4* rec[APS_MAX_LEVELS] = {};
  float4* gC[APS_MAX_LEVELS] = {};
  for (int l = 1; l < levels; ++l) {
    const size_t bytes = align256((size_t)N * (H >> l) * (W >> l) * sizeof(float4));
    rec[l] = reinterpret_cast<float4*>(wp);
    wp += bytes;
    gC[l] = reinterpret_cast<float4*>(wp);
    wp += bytes;
  }
  float* wbuf = reinterpret_cast<float*>(wp);
  hipStream_t st = as_stream(stream);

  // 1. recompute Lhat^{L-1} .. Lhat^1 (coarse to fine) with the forward kernel
  for (int l = levels - 1; l >= 1; --l) {
    LevelArgs a{};
    a.L = reinterpret_cast<const float4*>(L[l]);
    a.logits = logits[l];
    a.kstride = kstride[l];
    a.coarse = l < levels - 1 ? rec[l + 1] : nullptr;
    a.out = rec[l];
    a.H = H >> l;
    a.W = W >> l;
    a.eval_g = 1;
    a.eval_u = l < levels - 1;
    const int r = launch_level(a, logit_dtype, KD, KU, KT, l < levels - 1, false, N, st);
    if (r != APS_OK) return r;
  }
  // 2. fine to coarse
  for (int l = 0; l < levels; ++l) {
    const bool hu = l < levels - 1, ht = l == 0 && temporal;
    const int Hl = H >> l, Wl = W >> l;
    const int nk = level_k(l, levels, KD, KU, KT, temporal);
    BwdArgs b{};
    b.f.L = reinterpret_cast<const float4*>(L[l]);
    b.f.logits = logits[l];
    b.f.kstride = kstride[l];
    b.f.coarse = hu ? rec[l + 1] : nullptr;
    b.f.prev = reinterpret_cast<const float4*>(prev);
    b.f.mv = reinterpret_cast<const float2*>(mv);
    b.f.H = Hl;
    b.f.W = Wl;
    b.f.eval_g = 1;
    b.f.eval_u = hu;
    b.f.eval_t = ht;
    b.gout = l == 0 ? reinterpret_cast<const float4*>(grad_out) : gC[l];
    b.glogits = grad_logits[l];
    b.gstride = gstride[l];
    b.wbuf = wbuf;
    int r = launch_bwd(b, logit_dtype, grad_dtype, KD, KU, KT, hu, ht, N, st);
    if (r != APS_OK) return r;
    r = launch_same_T_k(KD, wbuf, nk, 0, b.gout, N, Hl, Wl, reinterpret_cast<float4*>(grad_L[l]), st);
    if (r != APS_OK) return r;
    if (hu) {
      r = launch_up_T(KU, wbuf, nk, KD * KD, b.gout, N, Hl, Wl, gC[l + 1], st);
      if (r != APS_OK) return r;
    }
    if (ht && grad_prev) {
      r = launch_warp_T(KT, wbuf, nk, KD * KD + (hu ? KU * KU : 0), b.gout, b.f.mv, N, Hl, Wl,
                        grad_prev, st);
      if (r != APS_OK) return r;
    }
  }
  return APS_OK;
}

// ---- standalone terms: reproject (kt block) and upsample (ku block) ------------------------

size_t aps_reproject_bwd_workspace_size(int N, int H, int W, int KD, int KU, int KT,
                                        int has_upsample) {
  const int nk = KD * KD + (has_upsample ? KU * KU : 0) + KT * KT;
  return align256((size_t)N * H * W * nk * sizeof(float)) + 256;
}

int aps_reproject_bwd(const float* prev, const float* mv, const void* logits0, int logit_dtype,
                      int kstride, int KD, int KU, int KT, int has_upsample, int N, int H, int W,
                      const float* grad_accum, void* grad_logits0, int grad_dtype, int gstride,
                      float* grad_prev, void* ws, size_t ws_bytes, void* stream) {
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if (has_upsample && (H % 2 || W % 2)) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!prev || !mv || !logits0 || !grad_accum || !grad_logits0) return APS_ERR_NULL;
  if (grad_dtype != APS_F32 && grad_dtype != APS_BF16) return APS_ERR_UNSUPPORTED;
  const int nk = KD * KD + (has_upsample ? KU * KU : 0) + KT * KT;
  if (!kstride_ok(kstride, nk, logit_dtype) || gstride < nk) return APS_ERR_SHAPE;
  if (!ws || ws_bytes < aps_reproject_bwd_workspace_size(N, H, W, KD, KU, KT, has_upsample))
    return APS_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  BwdArgs b{};
  b.f.logits = logits0;
  b.f.kstride = kstride;
  b.f.prev = reinterpret_cast<const float4*>(prev);
  b.f.mv = reinterpret_cast<const float2*>(mv);
  b.f.H = H;
  b.f.W = W;
  b.f.eval_t = 1;
  b.gout = reinterpret_cast<const float4*>(grad_accum);
  b.glogits = grad_logits0;
  b.gstride = gstride;
  b.wbuf = static_cast<float*>(ws);
  int r = launch_bwd(b, logit_dtype, grad_dtype, KD, KU, KT, has_upsample != 0, true, N, st);
  if (r != APS_OK) return r;
  if (grad_prev)
    r = launch_warp_T(KT, b.wbuf, nk, KD * KD + (has_upsample ? KU * KU : 0), b.gout, b.f.mv, N, H,
                      W, grad_prev, st);
  return r;
}

size_t aps_upsample_bwd_workspace_size(int N, int H, int W, int KD, int KU, int KT,
                                       int has_temporal) {
  const int nk = KD * KD + KU * KU + (has_temporal ? KT * KT : 0);
  return align256((size_t)N * H * W * nk * sizeof(float)) + 256;
}

int aps_upsample_bwd(const float* coarse, const void* logits, int logit_dtype, int kstride, int KD,
                     int KU, int KT, int has_temporal, int N, int H, int W,
                     const float* grad_accum, void* grad_logits, int grad_dtype, int gstride,
                     float* grad_coarse, void* ws, size_t ws_bytes, void* stream) {
  if (N < 0 || H < 0 || W < 0 || H % 2 || W % 2) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!coarse || !logits || !grad_accum || !grad_logits || !grad_coarse) return APS_ERR_NULL;
  if (grad_dtype != APS_F32 && grad_dtype != APS_BF16) return APS_ERR_UNSUPPORTED;
  const int nk = KD * KD + KU * KU + (has_temporal ? KT * KT : 0);
  if (!kstride_ok(kstride, nk, logit_dtype) || gstride < nk) return APS_ERR_SHAPE;
  if (!ws || ws_bytes < aps_upsample_bwd_workspace_size(N, H, W, KD, KU, KT, has_temporal))
    return APS_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  BwdArgs b{};
  b.f.logits = logits;
  b.f.kstride = kstride;
  b.f.coarse = reinterpret_cast<const float4*>(coarse);
  b.f.H = H;
  b.f.W = W;
  b.f.eval_u = 1;
  b.gout = reinterpret_cast<const float4*>(grad_accum);
  b.glogits = grad_logits;
  b.gstride = gstride;
  b.wbuf = static_cast<float*>(ws);
  const int r = launch_bwd(b, logit_dtype, grad_dtype, KD, KU, KT, true, has_temporal != 0, N, st);
  if (r != APS_OK) return r;
  return launch_up_T(KU, b.wbuf, nk, KD * KD, b.gout, N, H, W,
                     reinterpret_cast<float4*>(grad_coarse), st);
}

}  // extern "C"
