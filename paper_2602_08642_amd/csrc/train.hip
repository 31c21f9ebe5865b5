// Training kernels on gfx950: the tonemapped training loss with its gradient, and AdamW.
//
// Loss (Sec. 5, differentiable filmic tonemapper; Sec. 6.3 eqs. loss_spatial, loss_temporal,
// loss_combined), per pixel and colour channel c, with m = 1:
//   I = sRGB(tau(alpha * (sat_beta(log(max(L, 0) + eps)) + k); s, h))
//   spatial  = |I - I_ref|
//   temporal = |(I - W(I_prev)) - (I_ref - W(I_ref_prev))|, 0 where the back-projection leaves
//              the frame; W = bilinear warp along the motion vectors (edge-clamped taps)
//   loss = mean over pixels and channels of max(1.25 temporal, spatial)
// The kernel writes dLoss/dL of the current output and, when the previous output is part of
// the graph, adds dLoss/dL_prev through the warp (float atomics).
#include "aps_common.h"

using namespace aps;

namespace {

constexpr float kEps = 1e-4f;

struct TmoParams {
  float k, alpha, beta, s, h;
};

__device__ inline float tau(float x, float s, float h) {
  if (x < s - 1.f) return 0.5f * s * expf((x + 1.f - s) / s);
  if (x < 1.f - h) return 0.5f * (1.f + x);
  return 1.f - 0.5f * h * expf(-(x + h - 1.f) / h);
}
__device__ inline float dtau(float x, float s, float h) {
  if (x < s - 1.f) return 0.5f * expf((x + 1.f - s) / s);
  if (x < 1.f - h) return 0.5f;
  return 0.5f * expf(-(x + h - 1.f) / h);
}
__device__ inline float srgb(float v) {
  v = fminf(fmaxf(v, 0.f), 1.f);
  return v <= 0.0031308f ? 12.92f * v : 1.055f * powf(v, 1.f / 2.4f) - 0.055f;
}
__device__ inline float dsrgb(float v) {
  if (v < 0.f || v > 1.f) return 0.f;
  return v <= 0.0031308f ? 12.92f : (1.055f / 2.4f) * powf(v, 1.f / 2.4f - 1.f);
}

// I = tm(L) and the per-pixel Jacobian J[c][d] = dI_c / dL_d.
__device__ inline void tonemap(const float4 L, const TmoParams& p, float I[3], float J[3][3]) {
  const float Lc[3] = {L.x, L.y, L.z};
  float y[3], dy[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float v = fmaxf(Lc[c], 0.f);
    y[c] = logf(v + kEps);
    dy[c] = Lc[c] > 0.f ? 1.f / (Lc[c] + kEps) : 0.f;
  }
  const float m = (y[0] + y[1] + y[2]) * (1.f / 3.f);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float sat = m + p.beta * (y[c] - m);
    const float x = p.alpha * (sat + p.k);
    const float t = tau(x, p.s, p.h);
    I[c] = srgb(t);
    const float gc = dsrgb(t) * dtau(x, p.s, p.h) * p.alpha;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      J[c][d] = gc * ((c == d ? p.beta : 0.f) + (1.f - p.beta) * (1.f / 3.f)) * dy[d];
  }
}

struct Warp {
  int idx[4];
  float wt[4];
};
__device__ inline Warp warp_taps(float2 m, int H, int W, int x, int y) {
  const float fxf = floorf(m.x), fyf = floorf(m.y);
  const float fx = m.x - fxf, fy = m.y - fyf, gx = 1.f - fx, gy = 1.f - fy;
  const int x0 = x + (int)fxf, y0 = y + (int)fyf;
  const int xa = min(max(x0, 0), W - 1), xb = min(max(x0 + 1, 0), W - 1);
  const int ya = min(max(y0, 0), H - 1), yb = min(max(y0 + 1, 0), H - 1);
  return Warp{{ya * W + xa, ya * W + xb, yb * W + xa, yb * W + xb},
              {gy * gx, gy * fx, fy * gx, fy * fx}};
}

__device__ inline float sgn(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

__global__ __launch_bounds__(256) void k_tmo_loss(const float4* __restrict__ out,
                                                  const float4* __restrict__ ref,
                                                  const float4* __restrict__ prev_out,
                                                  const float4* __restrict__ prev_ref,
                                                  const float2* __restrict__ mv,
                                                  const float* __restrict__ params, int N, int H,
                                                  int W, float inv_count,
                                                  float4* __restrict__ grad_out,
                                                  float* __restrict__ grad_prev,
                                                  float* __restrict__ part) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  float lsum = 0.f;
  if (i < (size_t)N * H * W) {
    const int x = (int)(i % W), y = (int)((i / W) % H), n = (int)(i / ((size_t)W * H));
    const TmoParams p{params[n * 5 + 0], params[n * 5 + 1], params[n * 5 + 2], params[n * 5 + 3],
                      params[n * 5 + 4]};
    float I[3], J[3][3], Ir[3], Jr[3][3];
    tonemap(out[i], p, I, J);
    tonemap(ref[i], p, Ir, Jr);
    float gI[3] = {0.f, 0.f, 0.f}, gIp[3] = {0.f, 0.f, 0.f};
    Warp w{};
    bool temporal = false;
    float Ip[3] = {0.f, 0.f, 0.f}, Ipr[3] = {0.f, 0.f, 0.f};
    float Jp[4][3][3];
    if (prev_out) {
      const float2 m = mv[i];
      const float px = (float)x + m.x, py = (float)y + m.y;
      temporal = px >= -0.5f && px <= (float)W - 0.5f && py >= -0.5f && py <= (float)H - 0.5f;
      w = warp_taps(m, H, W, x, y);
      const size_t base = (size_t)n * H * W;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float a[3], b[3], Jr_[3][3];
        tonemap(prev_out[base + w.idx[t]], p, a, Jp[t]);
        tonemap(prev_ref[base + w.idx[t]], p, b, Jr_);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          Ip[c] += w.wt[t] * a[c];
          Ipr[c] += w.wt[t] * b[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float ds = I[c] - Ir[c];
      const float ls = fabsf(ds);
      float l = ls;
      float g = sgn(ds);
      if (temporal) {
        const float dt = (I[c] - Ip[c]) - (Ir[c] - Ipr[c]);
        const float lt = 1.25f * fabsf(dt);
        if (lt > ls) {
          l = lt;
          g = 1.25f * sgn(dt);
          gIp[c] = -g;
        }
      }
      lsum += l;
      gI[c] = g * inv_count;
      gIp[c] *= inv_count;
    }
    float gl[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) gl[d] = gI[0] * J[0][d] + gI[1] * J[1][d] + gI[2] * J[2][d];
    grad_out[i] = make_float4(gl[0], gl[1], gl[2], 0.f);
    if (temporal && grad_prev) {
      float* G = grad_prev + (size_t)n * H * W * 4;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (w.wt[t] == 0.f) continue;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float v = w.wt[t] * (gIp[0] * Jp[t][0][d] + gIp[1] * Jp[t][1][d] + gIp[2] * Jp[t][2][d]);
          if (v != 0.f) atomicAdd(G + (size_t)w.idx[t] * 4 + d, v);
        }
      }
    }
  }
  __shared__ float red[4];
  lsum = wave_sum(lsum);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_sum_partials(const float* __restrict__ part, int nb,
                                                      float scale, float* __restrict__ out) {
  float acc = 0.f;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[b];
  __shared__ float red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = ((red[0] + red[1]) + (red[2] + red[3])) * scale;
}

// ------------------------------------------------------------------ AdamW
// m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
// p -= lr * ((m / bc1) / (sqrt(v / bc2) + eps) + wd * p)     (decoupled weight decay)
__global__ __launch_bounds__(256) void k_adamw(float* __restrict__ p, float* __restrict__ m,
                                               float* __restrict__ v,
                                               const float* __restrict__ g, size_t n, float lr,
                                               float b1, float b2, float eps, float wd, float bc1,
                                               float bc2, float gscale) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i] * gscale;
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i];
  p[i] = pi - lr * ((mi / bc1) / (sqrtf(vi / bc2) + eps) + wd * pi);
}

__global__ __launch_bounds__(256) void k_sumsq_partial(const float* __restrict__ g, size_t n,
                                                       size_t per, float* __restrict__ part) {
  const size_t i0 = (size_t)blockIdx.x * per, i1 = min(n, i0 + per);
  float acc = 0.f;
  for (size_t i = i0 + threadIdx.x; i < i1; i += 256) acc += g[i] * g[i];
  __shared__ float red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// dst[p][c] = src[p][c] for c < C, 0 for C <= c < dst_ld (layout and dtype conversion)
template <typename S, typename D>
__global__ __launch_bounds__(256) void k_copy_channels(const S* __restrict__ src, int src_ld,
                                                       D* __restrict__ dst, int dst_ld, size_t npix,
                                                       int C) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npix * dst_ld) return;
  const size_t p = i / dst_ld;
  const int c = (int)(i % dst_ld);
  dst[i] = f2t<D>(c < C ? Ld<S>::get(src, p * src_ld + c) : 0.f);
}

__global__ __launch_bounds__(256) void k_scale_by(float* __restrict__ x, size_t n,
                                                  const float* __restrict__ s) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] *= *s;
}

}  // namespace

extern "C" {

int aps_copy_channels(const void* src, int src_dtype, int src_ld, void* dst, int dst_dtype,
                      int dst_ld, int64_t npix, int C, void* stream) {
  if (npix < 0 || C < 0 || src_ld < C || dst_ld < C || dst_ld <= 0) return APS_ERR_SHAPE;
  if (npix == 0) return APS_OK;
  if (!src || !dst) return APS_ERR_NULL;
  const size_t n = (size_t)npix * dst_ld;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipStream_t st = as_stream(stream);
  const bool sf = src_dtype == APS_F32, df = dst_dtype == APS_F32;
  if ((src_dtype != APS_F32 && src_dtype != APS_BF16) || (dst_dtype != APS_F32 && dst_dtype != APS_BF16))
    return APS_ERR_UNSUPPORTED;
  if (sf && df)
    k_copy_channels<float, float><<<blocks, 256, 0, st>>>(static_cast<const float*>(src), src_ld,
                                                          static_cast<float*>(dst), dst_ld, npix, C);
  else if (sf)
    k_copy_channels<float, uint16_t><<<blocks, 256, 0, st>>>(static_cast<const float*>(src), src_ld,
                                                             static_cast<uint16_t*>(dst), dst_ld,
                                                             npix, C);
  else if (df)
    k_copy_channels<uint16_t, float><<<blocks, 256, 0, st>>>(static_cast<const uint16_t*>(src),
                                                             src_ld, static_cast<float*>(dst),
                                                             dst_ld, npix, C);
  else
    k_copy_channels<uint16_t, uint16_t><<<blocks, 256, 0, st>>>(
        static_cast<const uint16_t*>(src), src_ld, static_cast<uint16_t*>(dst), dst_ld, npix, C);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_scale_by(float* x, int64_t n, const float* scale, void* stream) {
  if (n < 0) return APS_ERR_SHAPE;
  if (n == 0) return APS_OK;
  if (!x || !scale) return APS_ERR_NULL;
  k_scale_by<<<(unsigned)((n + 255) / 256), 256, 0, as_stream(stream)>>>(x, (size_t)n, scale);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

size_t aps_tmo_loss_workspace_size(int N, int H, int W) {
  return ((size_t)N * H * W + 255) / 256 * sizeof(float) + 256;
}

int aps_tmo_loss(const float* out, const float* ref, const float* prev_out, const float* prev_ref,
                 const float* mv, const float* params, int N, int H, int W, float* loss,
                 float* grad_out, float* grad_prev, void* ws, size_t ws_bytes, void* stream) {
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!out || !ref || !params || !loss || !grad_out) return APS_ERR_NULL;
  if (prev_out && (!prev_ref || !mv)) return APS_ERR_NULL;
  if (!ws || ws_bytes < aps_tmo_loss_workspace_size(N, H, W)) return APS_ERR_WORKSPACE;
  const size_t npix = (size_t)N * H * W;
  const int nb = (int)((npix + 255) / 256);
  float* part = static_cast<float*>(ws);
  const float inv = 1.f / (3.f * (float)npix);
  hipStream_t st = as_stream(stream);
  k_tmo_loss<<<nb, 256, 0, st>>>(reinterpret_cast<const float4*>(out),
                                 reinterpret_cast<const float4*>(ref),
                                 reinterpret_cast<const float4*>(prev_out),
                                 reinterpret_cast<const float4*>(prev_ref),
                                 reinterpret_cast<const float2*>(mv), params, N, H, W, inv,
                                 reinterpret_cast<float4*>(grad_out), grad_prev, part);
  k_sum_partials<<<1, 256, 0, st>>>(part, nb, inv, loss);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_adamw_step(float* param, float* m, float* v, const float* grad, int64_t n, float lr,
                   float beta1, float beta2, float eps, float weight_decay, int step,
                   float grad_scale, void* stream) {
  if (n < 0 || step < 1) return APS_ERR_ARG;
  if (n == 0) return APS_OK;
  if (!param || !m || !v || !grad) return APS_ERR_NULL;
  const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
  k_adamw<<<(unsigned)((n + 255) / 256), 256, 0, as_stream(stream)>>>(
      param, m, v, grad, (size_t)n, lr, beta1, beta2, eps, weight_decay, bc1, bc2, grad_scale);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

size_t aps_sumsq_workspace_size(int64_t n) {
  return (size_t)((n + 65535) / 65536 + 1) * sizeof(float) + 256;
}

int aps_sumsq(const float* x, int64_t n, float* out, void* ws, size_t ws_bytes, void* stream) {
  if (n < 0) return APS_ERR_SHAPE;
  if (!x || !out) return APS_ERR_NULL;
  if (!ws || ws_bytes < aps_sumsq_workspace_size(n)) return APS_ERR_WORKSPACE;
  const size_t per = 65536;
  const int nb = (int)(((size_t)n + per - 1) / per);
  float* part = static_cast<float*>(ws);
  hipStream_t st = as_stream(stream);
  if (nb > 0) k_sumsq_partial<<<nb, 256, 0, st>>>(x, (size_t)n, per, part);
  k_sum_partials<<<1, 256, 0, st>>>(part, nb, 1.f, out);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

}  // extern "C"
