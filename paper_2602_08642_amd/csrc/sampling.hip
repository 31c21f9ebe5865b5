// Sampling stages of the per-frame path on gfx950:
//   budget normalisation z -> s            (Sec. 3, Overview)
//   stochastic-rounding mask s, u -> counts, offsets, compact sample list
//                                          (Sec. 4.2, eq. holdout)
//   s-normalised scatter + pyramid         (Sec. 4.2 eq. stoch_rnoisy, Sec. 4.3 eqs.
//                                           relaxed_holdout / h_factor, App. A eq. app-pyramid)
//   renderer stand-in and feature assembly (inputs of the two networks)
#include <atomic>
#include <mutex>

#include "aps_common.h"

using namespace aps;

namespace {

constexpr int kNormElems = 4096;  // pixels per block of the softmax partial reductions
constexpr int kMaskBlock = 1024;  // pixels per block of the sample mask (4 per thread)
constexpr int kMaxTexSize = 4096;  // largest blue-noise texture side accepted

// ------------------------------------------------------------------ normalisation
// Partial (max, sum exp(z - max)) over kNormElems pixels of one image; fixed partition,
// fixed reduction tree: deterministic.
__global__ __launch_bounds__(256) void k_norm_partial(const float* __restrict__ z, int npx,
                                                      int nb, float2* __restrict__ part) {
  const int n = blockIdx.y, b = blockIdx.x;
  const float* zi = z + (size_t)n * npx;
  const int base = b * kNormElems;
  float v[kNormElems / 256];
  float m = -INFINITY;
#pragma unroll
  for (int k = 0; k < kNormElems / 256; ++k) {
    const int i = base + k * 256 + threadIdx.x;
    v[k] = i < npx ? zi[i] : -INFINITY;
    m = fmaxf(m, v[k]);
  }
  __shared__ float sm[4];
  __shared__ float ss[4];
  m = wave_max(m);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sm[w] = m;
  __syncthreads();
  m = fmaxf(fmaxf(sm[0], sm[1]), fmaxf(sm[2], sm[3]));
  float e = 0.f;
#pragma unroll
  for (int k = 0; k < kNormElems / 256; ++k) e += (v[k] == -INFINITY) ? 0.f : expf(v[k] - m);
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0) ss[w] = e;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)n * nb + b] = make_float2(m, (ss[0] + ss[1]) + (ss[2] + ss[3]));
}

// Combine one image's partials into (max, sum) with a fixed order (a block of 256 threads;
// every caller gets the same result from the same partials).
__device__ inline float2 norm_combine_block(const float2* __restrict__ p, int nb, float* red) {
  float m = -INFINITY;
  for (int b = threadIdx.x; b < nb; b += 256) m = fmaxf(m, p[b].x);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  __syncthreads();
  float e = 0.f;
  for (int b = threadIdx.x; b < nb; b += 256) e += p[b].y * expf(p[b].x - m);
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  const float sum = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return make_float2(m, sum);
}

// One block per image: the combined (max, sum) for the backward pass.
__global__ __launch_bounds__(256) void k_norm_combine(const float2* __restrict__ part, int nb,
                                                      float2* __restrict__ stats) {
  __shared__ float red[4];
  const float2 ms = norm_combine_block(part + (size_t)blockIdx.x * nb, nb, red);
  if (threadIdx.x == 0) stats[blockIdx.x] = ms;
}

// s = f*B + (1-f)*B*Npx * exp(z - max) / sum over kNormApply pixels per block (8 per thread);
// each block combines the image's partials itself (a few thousand L2-resident values) instead
// of waiting for a combine launch.
constexpr int kNormPer = 8, kNormApply = 256 * kNormPer;
__global__ __launch_bounds__(256) void k_norm_apply(const float* __restrict__ z, int npx,
                                                    const float2* __restrict__ part, int nbp,
                                                    float c0, float c1, int vec,
                                                    float* __restrict__ s, uint32_t* st) {
  const int n = blockIdx.y;
  __shared__ float red[4];
  const float2 ms = norm_combine_block(part + (size_t)n * nbp, nbp, red);
  const int i0 = blockIdx.x * kNormApply + threadIdx.x * kNormPer;
  const float* zi = z + (size_t)n * npx;
  float* si = s + (size_t)n * npx;
  bool bad = false;
  if (vec && i0 + kNormPer <= npx) {
#pragma unroll
    for (int k = 0; k < kNormPer; k += 4) {
      const float4 v = *reinterpret_cast<const float4*>(zi + i0 + k);
      const float4 o = make_float4(c0 + c1 * (expf(v.x - ms.x) / ms.y), c0 + c1 * (expf(v.y - ms.x) / ms.y),
                                   c0 + c1 * (expf(v.z - ms.x) / ms.y), c0 + c1 * (expf(v.w - ms.x) / ms.y));
      bad |= !isfinite(o.x) || !isfinite(o.y) || !isfinite(o.z) || !isfinite(o.w);
      *reinterpret_cast<float4*>(si + i0 + k) = o;
    }
  } else {
    for (int k = 0; k < kNormPer; ++k) {
      if (i0 + k >= npx) break;
      const float v = c0 + c1 * (expf(zi[i0 + k] - ms.x) / ms.y);
      bad |= !isfinite(v);
      si[i0 + k] = v;
    }
  }
  if (bad) status_or(st, APS_STATUS_NONFINITE);
}

// ------------------------------------------------------------------ sample mask
// Two launches: counts with per-block sums, then offsets and the compact list, where each block
// adds up the sums of the blocks before it (at most a few thousand L2-resident integers) rather
// than waiting for a separate scan launch.  A thread owns kMaskPer consecutive pixels, so a
// block's exclusive scan is one scan over its 256 thread totals.
constexpr int kMaskPer = 4;

// Count of pixel i from s_i (eq. holdout): stochastic floor(s) + [u < p]; holdout always
// requested floor(s) + [p > 0] (straight-through, Gumbel-Softmax); deterministic round(s)
// (Sec. 4.1 eq. kuz_fw).  p = s - floor(s) is exact in binary32.
__device__ inline int mask_count_one(float si, float u, int rounding, float& p, uint32_t* st) {
  p = 0.f;
  if (!(si >= 0.f) || !isfinite(si)) {
    status_or(st, APS_STATUS_NONFINITE);
    return 0;
  }
  const float fl = floorf(si);
  p = si - fl;
  int extra;
  if (rounding == APS_ROUND_STOCHASTIC) extra = u < p ? 1 : 0;
  else if (rounding == APS_ROUND_HOLDOUT) extra = p > 0.f ? 1 : 0;
  else extra = p >= 0.5f ? 1 : 0;
  int c = fl > 254.f ? 256 : (int)fl + extra;
  if (c > 255) {
    status_or(st, APS_STATUS_COUNT_OVERFLOW);
    c = 255;
  }
  return c;
}

// block sum over a block of 256 threads (fixed tree)
__device__ inline int block_isum(int v, int* red) {
  v = wave_isum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const int r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_mask_count(const float* __restrict__ s, int npix,
                                                    uint64_t seed, uint32_t frame, USource us,
                                                    int rounding, int vec,
                                                    uint8_t* __restrict__ count,
                                                    float* __restrict__ p_out,
                                                    int32_t* __restrict__ block_sum, uint32_t* st) {
  const int i0 = blockIdx.x * kMaskBlock + threadIdx.x * kMaskPer;
  float sv[kMaskPer];
  const bool full = vec && i0 + kMaskPer <= npix;
  if (full) {
#pragma unroll
    for (int k = 0; k < kMaskPer; k += 4) {
      const float4 v = *reinterpret_cast<const float4*>(s + i0 + k);
      sv[k] = v.x;
      sv[k + 1] = v.y;
      sv[k + 2] = v.z;
      sv[k + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kMaskPer; ++k) sv[k] = i0 + k < npix ? s[i0 + k] : 0.f;
  }
  // u of the thread's pixels: one Philox block per four (i0 is a multiple of 4)
  float u[kMaskPer];
  if (rounding == APS_ROUND_STOCHASTIC) {
    if (full && !us.tex) {
#pragma unroll
      for (int q = 0; q < kMaskPer / 4; ++q) {
        const uint4 r = uniform_block(seed, (uint32_t)(i0 / 4 + q), frame);
        u[4 * q] = u24(r.x);
        u[4 * q + 1] = u24(r.y);
        u[4 * q + 2] = u24(r.z);
        u[4 * q + 3] = u24(r.w);
      }
    } else {
#pragma unroll
      for (int k = 0; k < kMaskPer; ++k) u[k] = i0 + k < npix ? draw_u(us, seed, (uint32_t)(i0 + k), frame) : 0.f;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kMaskPer; ++k) u[k] = 0.f;
  }
  int c[kMaskPer];
  float p[kMaskPer];
  int tsum = 0;
#pragma unroll
  for (int k = 0; k < kMaskPer; ++k) {
    c[k] = i0 + k < npix ? mask_count_one(sv[k], u[k], rounding, p[k], st) : 0;
    tsum += c[k];
  }
  if (full) {
#pragma unroll
    for (int q = 0; q < kMaskPer / 4; ++q)
      reinterpret_cast<uint32_t*>(count + i0)[q] =
          (uint32_t)c[4 * q] | ((uint32_t)c[4 * q + 1] << 8) | ((uint32_t)c[4 * q + 2] << 16) |
          ((uint32_t)c[4 * q + 3] << 24);
    if (p_out) {
#pragma unroll
      for (int k = 0; k < kMaskPer; k += 4)
        *reinterpret_cast<float4*>(p_out + i0 + k) = make_float4(p[k], p[k + 1], p[k + 2], p[k + 3]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < kMaskPer; ++k)
      if (i0 + k < npix) {
        count[i0 + k] = (uint8_t)c[k];
        if (p_out) p_out[i0 + k] = p[k];
      }
  }
  __shared__ int red[4];
  const int bs = block_isum(tsum, red);
  if (threadIdx.x == 0) block_sum[blockIdx.x] = bs;
}

__global__ __launch_bounds__(256) void k_mask_compact(const uint8_t* __restrict__ count, int npix,
                                                      int vec, const int32_t* __restrict__ block_sum,
                                                      int nb, int32_t* __restrict__ pixel_offset,
                                                      int32_t* __restrict__ sample_pixel,
                                                      int64_t capacity, int32_t* __restrict__ total,
                                                      uint32_t* st) {
  const int b = blockIdx.x, t = threadIdx.x;
  __shared__ int red[4];
  __shared__ int wsum[4];
  // samples of the blocks before this one
  int before = 0;
  int j = t;
  for (; j + 768 < b; j += 1024)  // four independent loads in flight per thread
    before += (block_sum[j] + block_sum[j + 256]) + (block_sum[j + 512] + block_sum[j + 768]);
  for (; j < b; j += 256) before += block_sum[j];
  const int base = block_isum(before, red);
  const int i0 = b * kMaskBlock + t * kMaskPer;
  const bool full = vec && i0 + kMaskPer <= npix;
  int c[kMaskPer];
  if (full) {
#pragma unroll
    for (int q = 0; q < kMaskPer / 4; ++q) {
      const uint32_t w = reinterpret_cast<const uint32_t*>(count + i0)[q];
#pragma unroll
      for (int k = 0; k < 4; ++k) c[4 * q + k] = (int)((w >> (8 * k)) & 255u);
    }
  } else {
#pragma unroll
    for (int k = 0; k < kMaskPer; ++k) c[k] = i0 + k < npix ? (int)count[i0 + k] : 0;
  }
  int tsum = 0;
#pragma unroll
  for (int k = 0; k < kMaskPer; ++k) tsum += c[k];
  const int incl = wave_iscan(tsum);
  if ((t & 63) == 63) wsum[t >> 6] = incl;
  __syncthreads();
  int wbefore = 0;
  for (int w = 0; w < (t >> 6); ++w) wbefore += wsum[w];
  int off = base + wbefore + incl - tsum;
  if (b == nb - 1 && t == 255) *total = off + tsum;
  int o[kMaskPer];
#pragma unroll
  for (int k = 0; k < kMaskPer; ++k) {
    o[k] = off;
    if (i0 + k < npix) {
      for (int j = 0; j < c[k]; ++j) {
        if ((int64_t)off + j < capacity) sample_pixel[off + j] = i0 + k;
        else status_or(st, APS_STATUS_CAPACITY);
      }
    }
    off += c[k];
  }
  if (full) {
#pragma unroll
    for (int k = 0; k < kMaskPer; k += 4)
      *reinterpret_cast<int4*>(pixel_offset + i0 + k) = make_int4(o[k], o[k + 1], o[k + 2], o[k + 3]);
  } else {
#pragma unroll
    for (int k = 0; k < kMaskPer; ++k)
      if (i0 + k < npix) pixel_offset[i0 + k] = o[k];
  }
}

__global__ void k_zero_i32(int32_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

// ------------------------------------------------------------------ renderer stand-in
__global__ __launch_bounds__(256) void k_fixture_render(const float4* __restrict__ pool, int J,
                                                        const uint8_t* __restrict__ count,
                                                        const int32_t* __restrict__ pixel_offset,
                                                        int npix, int64_t capacity,
                                                        float4* __restrict__ samples) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= npix) return;
  const int c = count[i];
  const int off = pixel_offset[i];
  for (int j = 0; j < c; ++j)
    if ((int64_t)off + j < capacity) samples[off + j] = pool[(size_t)i * J + (j % J)];
}

// ------------------------------------------------------------------ scatter + pyramid
// One 16x16 tile of level-0 pixels per block.  Level 0 is the s-normalised estimate,
// Weight w of the holdout sample and dw/dp (p = s - floor(s)) for each scatter mode:
//   hard: w = 1 when the holdout was requested, no gradient through the indicator;
//   relaxed (Sec. 4.3, eqs. relaxed_holdout, h_factor; u mirrored): w = h clamp(lam (p - u)/p);
//   straight-through: w = [u < p], dw/dp taken as 1;
//   Gumbel-Softmax (binary concrete, temperature tau = param): w = sigmoid((logit p - logit u)/tau).
struct HoldW {
  float w, dwdp;
};
__device__ inline HoldW holdout_weight(int mode, float p, float u, float param, float hfac) {
  HoldW h{1.f, 0.f};
  if (mode == APS_RELAXED) {
    const float t = param * (p - u) / p;
    h.w = hfac * fminf(fmaxf(t, 0.f), 1.f);
    if (t > 0.f && t < 1.f) h.dwdp = hfac * param * u / (p * p);
  } else if (mode == APS_STRAIGHT_THROUGH) {
    h.w = u < p ? 1.f : 0.f;
    h.dwdp = 1.f;
  } else if (mode == APS_GUMBEL) {
    const float z = ((logf(p) - log1pf(-p)) - (logf(u) - log1pf(-u))) / param;
    h.w = 1.f / (1.f + expf(-z));
    h.dwdp = h.w * (1.f - h.w) / (param * p * (1.f - p));
  }
  return h;
}

// levels 1.. are 2x2 means of the level above, reduced in LDS (= 2^l x 2^l block means).
__global__ __launch_bounds__(256) void k_scatter(const float* __restrict__ s,
                                                 const uint8_t* __restrict__ count,
                                                 const int32_t* __restrict__ pixel_offset,
                                                 const float4* __restrict__ samples,
                                                 int64_t n_samples, int H, int W, int levels, int mode, float lam, float hfac,
                                                 uint64_t seed, uint32_t frame, USource us,
                                                 LevelPtrs Lp) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int x = blockIdx.x * 16 + tx, y = blockIdx.y * 16 + ty, n = blockIdx.z;
  __shared__ float4 tile[16][17];
  float4 L = make_float4(0.f, 0.f, 0.f, 0.f);
  const bool in = x < W && y < H;
  if (in) {
    const size_t i = ((size_t)n * H + y) * W + x;
    const float si = s[i];
    const int c = count[i];
    const int off = pixel_offset[i];
    const float fl = floorf(si);
    const int nb = min(c, (int)fl);
    // samples past the caller's buffer (a mask that overflowed its capacity) read as 0
    const int lim = (int)min((int64_t)c, max((int64_t)0, n_samples - off));
    float ax = 0.f, ay = 0.f, az = 0.f;
    if (mode == APS_DASR) {  // Sec. 4.1 eq. kuz_fw: the mean of the round(s) requested samples
      for (int j = 0; j < lim; ++j) {
        const float4 v = samples[off + j];
        ax += v.x;
        ay += v.y;
        az += v.z;
      }
      if (c > 0) L = make_float4(ax / (float)c, ay / (float)c, az / (float)c, 0.f);
    } else {
      for (int j = 0; j < min(nb, lim); ++j) {
        const float4 v = samples[off + j];
        ax += v.x;
        ay += v.y;
        az += v.z;
      }
      if (c > nb && nb < lim) {  // the holdout sample was requested
        const float4 r = samples[off + nb];
        const float u = mode == APS_HARD ? 0.f : draw_u(us, seed, (uint32_t)i, frame);
        const float w = holdout_weight(mode, si - fl, u, lam, hfac).w;
        ax += w * r.x;
        ay += w * r.y;
        az += w * r.z;
      }
      if (si > 0.f) L = make_float4(ax / si, ay / si, az / si, 0.f);
    }
    Lp.p[0][i] = L;
  }
  tile[ty][tx] = L;
  int Hl = H, Wl = W;
  for (int l = 1; l < levels; ++l) {
    __syncthreads();
    const int t = 16 >> l;
    Hl >>= 1;
    Wl >>= 1;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (tx < t && ty < t) {
      const float4 a = tile[2 * ty][2 * tx], b = tile[2 * ty][2 * tx + 1];
      const float4 c = tile[2 * ty + 1][2 * tx], d = tile[2 * ty + 1][2 * tx + 1];
      v = make_float4(((a.x + b.x) + (c.x + d.x)) * 0.25f, ((a.y + b.y) + (c.y + d.y)) * 0.25f,
                      ((a.z + b.z) + (c.z + d.z)) * 0.25f, 0.f);
    }
    __syncthreads();
    if (tx < t && ty < t) {
      tile[ty][tx] = v;
      const int xl = blockIdx.x * t + tx, yl = blockIdx.y * t + ty;
      if (xl < Wl && yl < Hl) Lp.p[l][((size_t)n * Hl + yl) * Wl + xl] = v;
    }
  }
}

// ------------------------------------------------------------------ feature assembly
// The forward feature transforms use the hardware base-2 logarithm and exponential
// (v_log_f32, v_exp_f32, about one ulp): network inputs need about 1e-5 relative, and the
// library-accurate log1p / log / exp / pow made the assembly bound by its arithmetic rather
// than by its memory traffic.  The backward keeps the accurate functions.
constexpr float kLn2 = 0.69314718055994531f, kLog2e = 1.4426950408889634f;
__device__ inline float fast_log(float x) { return __builtin_amdgcn_logf(x) * kLn2; }
__device__ inline float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
// log(1 + a) for a >= 0: 1 + a rounds by at most 2^-24, an absolute error of 6e-8 in the log
__device__ inline float slog1p_fwd(float v) { return copysignf(fast_log(1.f + fabsf(v)), v); }
__device__ inline float slog1p(float v) { return copysignf(log1pf(fabsf(v)), v); }

// Evaluation tonemapper of the feedback loop (Sec. 5): log, curve tau(x; 0.5, 0.5) with
// contrast 0.4, exposure 0, saturation 1, then the sRGB transfer function.
__device__ inline float tau_eval(float x) {
  const float s = 0.5f, h = 0.5f;
  if (x < s - 1.f) return 0.5f * s * fast_exp((x + 1.f - s) / s);
  if (x < 1.f - h) return 0.5f * (1.f + x);
  return 1.f - 0.5f * h * fast_exp(-(x + h - 1.f) / h);
}
__device__ inline float srgb(float v) {
  v = fminf(fmaxf(v, 0.f), 1.f);
  // v^(1/2.4) = 2^(log2(v) / 2.4) for v > 0.0031308
  return v <= 0.0031308f ? 12.92f * v
                         : 1.055f * __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(v) * (1.f / 2.4f)) - 0.055f;
}
__device__ inline float tonemap_eval(float L) {
  return srgb(tau_eval(0.4f * fast_log(fmaxf(L, 0.f) + 1e-4f)));
}

// Bilinear sample of prev at (x + mv.x, y + mv.y), both taps clamped to the edge; the
// integer cell comes from floor(mv) so the fractional weights are exact.
__device__ inline float4 warp_sample(const float4* __restrict__ prev, int H, int W, int n, int x,
                                     int y, float2 mv) {
  const float fxf = floorf(mv.x), fyf = floorf(mv.y);
  const float fx = mv.x - fxf, fy = mv.y - fyf;
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

// all four channels (the recurrent latents use the A channel as well)
__device__ inline float4 warp_sample4(const float4* __restrict__ src, int H, int W, int n, int x,
                                      int y, float2 mv) {
  const float fxf = floorf(mv.x), fyf = floorf(mv.y);
  const float fx = mv.x - fxf, fy = mv.y - fyf;
  const int x0 = x + (int)fxf, y0 = y + (int)fyf;
  const int xa = min(max(x0, 0), W - 1), xb = min(max(x0 + 1, 0), W - 1);
  const int ya = min(max(y0, 0), H - 1), yb = min(max(y0 + 1, 0), H - 1);
  const float4* P = src + (size_t)n * H * W;
  const float4 a = P[(size_t)ya * W + xa], b = P[(size_t)ya * W + xb];
  const float4 c = P[(size_t)yb * W + xa], d = P[(size_t)yb * W + xb];
  const float gx = 1.f - fx, gy = 1.f - fy;
  return make_float4(gy * (gx * a.x + fx * b.x) + fy * (gx * c.x + fx * d.x),
                     gy * (gx * a.y + fx * b.y) + fy * (gx * c.y + fx * d.y),
                     gy * (gx * a.z + fx * b.z) + fy * (gx * c.z + fx * d.z),
                     gy * (gx * a.w + fx * b.w) + fy * (gx * c.w + fx * d.w));
}

__device__ inline float mv_valid(int H, int W, int x, int y, float2 mv) {
  const float px = (float)x + mv.x, py = (float)y + mv.y;
  return (px >= -0.5f && px <= (float)W - 0.5f && py >= -0.5f && py <= (float)H - 0.5f) ? 1.f : 0.f;
}

// One pixel's feature row of C (8, 16 or 24) channels as 16-byte stores.
template <typename T>
__device__ inline void store_row(T* dst, int C, const float* f);
template <>
__device__ inline void store_row<float>(float* dst, int C, const float* f) {
  float4* d = reinterpret_cast<float4*>(dst);
  d[0] = make_float4(f[0], f[1], f[2], f[3]);
  d[1] = make_float4(f[4], f[5], f[6], f[7]);
  if (C >= 16) {
    d[2] = make_float4(f[8], f[9], f[10], f[11]);
    d[3] = make_float4(f[12], f[13], f[14], f[15]);
  }
  if (C == 24) {
    d[4] = make_float4(f[16], f[17], f[18], f[19]);
    d[5] = make_float4(f[20], f[21], f[22], f[23]);
  }
}
// bf16: the hardware packed conversion (round to nearest even, as f2bf for finite values)
__device__ inline u16x8 pack_bf8(const float* f) {
  const u16x4 lo = f2bf4(f[0], f[1], f[2], f[3]), hi = f2bf4(f[4], f[5], f[6], f[7]);
  return u16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}
template <>
__device__ inline void store_row<uint16_t>(uint16_t* dst, int C, const float* f) {
  u16x8* d = reinterpret_cast<u16x8*>(dst);
  d[0] = pack_bf8(f);
  if (C >= 16) d[1] = pack_bf8(f + 8);
  if (C == 24) d[2] = pack_bf8(f + 16);
}

// kind 0 (sampler input):   aux[0..6], then (temporal) tonemap(W prev) 3, valid 1; zero pad.
// kind 1 (kernel predictor): aux[0..6], slog1p(L0) 3, s 1, then (temporal) slog1p(W prev) 3,
//                            valid 1; zero pad.
// Both then (recurrent latents) the 4 channels of W lat, the previous frame's latents warped.
template <typename T>
__global__ __launch_bounds__(256) void k_features(int kind, const float* __restrict__ aux,
                                                  const float4* __restrict__ L0,
                                                  const float* __restrict__ s,
                                                  const float4* __restrict__ prev,
                                                  const float2* __restrict__ mv,
                                                  const float4* __restrict__ lat, int N, int H,
                                                  int W, int C, T* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t npix = (size_t)N * H * W;
  if (i >= npix) return;
  const int x = (int)(i % W), y = (int)((i / W) % H), n = (int)(i / ((size_t)W * H));
  float f[24];
#pragma unroll
  for (int c = 0; c < 24; ++c) f[c] = 0.f;
  {
    const float4 a0 = reinterpret_cast<const float4*>(aux)[2 * i];
    const float4 a1 = reinterpret_cast<const float4*>(aux)[2 * i + 1];
    f[0] = a0.x; f[1] = a0.y; f[2] = a0.z; f[3] = a0.w;
    f[4] = a1.x; f[5] = a1.y; f[6] = a1.z;
  }
  int o = 7;
  if (kind == 1) {
    const float4 l = L0[i];
    f[7] = slog1p_fwd(l.x);
    f[8] = slog1p_fwd(l.y);
    f[9] = slog1p_fwd(l.z);
    f[10] = s[i];
    o = 11;
  }
  if (prev) {
    const float2 m = mv[i];
    const float4 w = warp_sample(prev, H, W, n, x, y, m);
    if (kind == 0) {
      f[o] = tonemap_eval(w.x);
      f[o + 1] = tonemap_eval(w.y);
      f[o + 2] = tonemap_eval(w.z);
    } else {
      f[o] = slog1p_fwd(w.x);
      f[o + 1] = slog1p_fwd(w.y);
      f[o + 2] = slog1p_fwd(w.z);
    }
    f[o + 3] = mv_valid(H, W, x, y, m);
    if (lat) {
      const float4 v = warp_sample4(lat, H, W, n, x, y, m);
      f[o + 4] = v.x;
      f[o + 5] = v.y;
      f[o + 6] = v.z;
      f[o + 7] = v.w;
    }
  }
  store_row<T>(out + i * C, C, f);
}

// ======================================================================== backward
// ------------------------------------------------------------------ scatter + pyramid
// L0 = (base + w r) / s with the holdout weight w of the mode (holdout_weight), p = s - floor(s):
// dL0/ds = -L0 / s + (r / s) dw/dp.  DASR (Sec. 4.1 eq. kuz_grad): the surrogate
// dL0/ds = (L_ref - L0) / round(s) for s >= 1/2 and L_ref below.  The pyramid levels are block
// means of L0, so dLoss/dL0 collects dLoss/dL^l / 4^l from every ancestor.
struct GradLevels {
  const float4* p[APS_MAX_LEVELS];
};

__global__ __launch_bounds__(256) void k_scatter_bwd(const float* __restrict__ s,
                                                     const uint8_t* __restrict__ count,
                                                     const int32_t* __restrict__ pixel_offset,
                                                     const float4* __restrict__ samples,
                                                     int64_t n_samples, int N, int H, int W,
                                                     int levels, int mode, float lam, float hfac,
                                                     uint64_t seed, uint32_t frame, USource us,
                                                     const float4* __restrict__ Lref, GradLevels g,
                                                     float* __restrict__ grad_s, int accumulate) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)N * H * W) return;
  const int x = (int)(i % W), y = (int)((i / W) % H), n = (int)(i / ((size_t)W * H));
  float4 ge = g.p[0][i];
  float sc = 1.f;
  for (int l = 1; l < levels; ++l) {
    sc *= 0.25f;
    const int Hl = H >> l, Wl = W >> l;
    const float4 v = g.p[l][((size_t)n * Hl + (y >> l)) * Wl + (x >> l)];
    ge.x += sc * v.x;
    ge.y += sc * v.y;
    ge.z += sc * v.z;
  }
  const float si = s[i];
  float out = 0.f;
  if (mode == APS_DASR) {
    const int c = count[i];
    const int off = pixel_offset[i];
    const int lim = (int)min((int64_t)c, max((int64_t)0, n_samples - off));
    float ax = 0.f, ay = 0.f, az = 0.f;
    for (int j = 0; j < lim; ++j) {
      const float4 v = samples[off + j];
      ax += v.x;
      ay += v.y;
      az += v.z;
    }
    const float4 lr = Lref[i];
    if (si >= 0.5f && c > 0) {
      const float inv = 1.f / (float)c;
      out = ge.x * (lr.x - ax * inv) * inv + ge.y * (lr.y - ay * inv) * inv +
            ge.z * (lr.z - az * inv) * inv;
    } else {
      out = ge.x * lr.x + ge.y * lr.y + ge.z * lr.z;
    }
  } else if (si > 0.f) {
    const int c = count[i];
    const int off = pixel_offset[i];
    const float fl = floorf(si);
    const int nb = min(c, (int)fl);
    const int lim = (int)min((int64_t)c, max((int64_t)0, n_samples - off));
    float ax = 0.f, ay = 0.f, az = 0.f;
    for (int j = 0; j < min(nb, lim); ++j) {
      const float4 v = samples[off + j];
      ax += v.x;
      ay += v.y;
      az += v.z;
    }
    float dwdp = 0.f;
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    if (c > nb && nb < lim) {
      r = samples[off + nb];
      const float u = mode == APS_HARD ? 0.f : draw_u(us, seed, (uint32_t)i, frame);
      const HoldW h = holdout_weight(mode, si - fl, u, lam, hfac);
      dwdp = h.dwdp;
      ax += h.w * r.x;
      ay += h.w * r.y;
      az += h.w * r.z;
    }
    const float inv = 1.f / si;
    const float lx = ax * inv, ly = ay * inv, lz = az * inv;
    out = ge.x * (dwdp * r.x * inv - lx * inv) + ge.y * (dwdp * r.y * inv - ly * inv) +
          ge.z * (dwdp * r.z * inv - lz * inv);
  }
  grad_s[i] = (accumulate ? grad_s[i] : 0.f) + out;
}

// ------------------------------------------------------------------ normalisation
// s = c0 + c1 * sm(z):  dLoss/dz_j = c1 sm_j (g_j - sum_i sm_i g_i); the sum is a fixed tree.
__global__ __launch_bounds__(256) void k_norm_gdot_partial(const float* __restrict__ z,
                                                           const float* __restrict__ g, int npx,
                                                           int nb, const float2* __restrict__ stats,
                                                           float* __restrict__ part) {
  const int n = blockIdx.y, b = blockIdx.x;
  const float2 ms = stats[n];
  const float inv = 1.f / ms.y;
  float acc = 0.f;
  for (int k = 0; k < kNormElems / 256; ++k) {
    const int i = b * kNormElems + k * 256 + threadIdx.x;
    if (i < npx) acc += expf(z[(size_t)n * npx + i] - ms.x) * inv * g[(size_t)n * npx + i];
  }
  __shared__ float red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)n * nb + b] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_norm_gdot_combine(const float* __restrict__ part, int nb,
                                                           float* __restrict__ dots) {
  const int n = blockIdx.x;
  float acc = 0.f;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[(size_t)n * nb + b];
  __shared__ float red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) dots[n] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_norm_bwd_apply(const float* __restrict__ z,
                                                        const float* __restrict__ g, int npx,
                                                        const float2* __restrict__ stats,
                                                        const float* __restrict__ dots, float c1,
                                                        float* __restrict__ gz) {
  const int n = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= npx) return;
  const size_t k = (size_t)n * npx + i;
  const float2 ms = stats[n];
  const float sm = expf(z[k] - ms.x) / ms.y;
  gz[k] = c1 * sm * (g[k] - dots[n]);
}

// ------------------------------------------------------------------ feature assembly
__device__ inline float dtau_eval(float x) {
  const float s = 0.5f, h = 0.5f;
  if (x < s - 1.f) return 0.5f * expf((x + 1.f - s) / s);
  if (x < 1.f - h) return 0.5f;
  return 0.5f * expf(-(x + h - 1.f) / h);
}
__device__ inline float dsrgb(float v) {
  if (v <= 0.f || v >= 1.f) return v <= 0.0031308f ? 12.92f : 0.f;
  return v <= 0.0031308f ? 12.92f : (1.055f / 2.4f) * powf(v, 1.f / 2.4f - 1.f);
}
__device__ inline float dtonemap_eval(float L) {
  if (!(L > 0.f)) return 0.f;
  const float x = 0.4f * logf(L + 1e-4f);
  return dsrgb(tau_eval(x)) * dtau_eval(x) * 0.4f / (L + 1e-4f);
}

__device__ inline void splat_prev(float* __restrict__ gprev, int H, int W, int n, int x, int y,
                                  float2 m, float gx_, float gy_, float gz_, float gw_ = 0.f,
                                  bool four = false) {
  const float fxf = floorf(m.x), fyf = floorf(m.y);
  const float fx = m.x - fxf, fy = m.y - fyf, gx = 1.f - fx, gy = 1.f - fy;
  const int x0 = x + (int)fxf, y0 = y + (int)fyf;
  const int xa = min(max(x0, 0), W - 1), xb = min(max(x0 + 1, 0), W - 1);
  const int ya = min(max(y0, 0), H - 1), yb = min(max(y0 + 1, 0), H - 1);
  const int idx[4] = {ya * W + xa, ya * W + xb, yb * W + xa, yb * W + xb};
  const float wt[4] = {gy * gx, gy * fx, fy * gx, fy * fx};
  float* P = gprev + (size_t)n * H * W * 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (wt[k] == 0.f) continue;
    float* d = P + (size_t)idx[k] * 4;
    atomicAdd(d + 0, wt[k] * gx_);
    atomicAdd(d + 1, wt[k] * gy_);
    atomicAdd(d + 2, wt[k] * gz_);
    if (four) atomicAdd(d + 3, wt[k] * gw_);
  }
}

template <typename T>
__device__ inline float load_feat(const T* p, int c);
template <>
__device__ inline float load_feat<float>(const float* p, int c) { return p[c]; }
template <>
__device__ inline float load_feat<uint16_t>(const uint16_t* p, int c) { return bf2f(p[c]); }

// Transpose of k_features: adds to grad_L0 (RGB), grad_s, and (atomically) grad_prev.
template <typename T>
__global__ __launch_bounds__(256) void k_features_bwd(int kind, const float4* __restrict__ L0,
                                                      const float4* __restrict__ prev,
                                                      const float2* __restrict__ mv, int N, int H,
                                                      int W, int C, const T* __restrict__ gfeat,
                                                      float4* __restrict__ gL0,
                                                      float* __restrict__ gs,
                                                      float* __restrict__ gprev,
                                                      float* __restrict__ glat) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)N * H * W) return;
  const int x = (int)(i % W), y = (int)((i / W) % H), n = (int)(i / ((size_t)W * H));
  const T* g = gfeat + i * C;
  int o = 7;
  if (kind == 1) {
    const float4 l = L0[i];
    if (gL0) {
      float4 a = gL0[i];
      a.x += load_feat<T>(g, 7) / (1.f + fabsf(l.x));
      a.y += load_feat<T>(g, 8) / (1.f + fabsf(l.y));
      a.z += load_feat<T>(g, 9) / (1.f + fabsf(l.z));
      gL0[i] = a;
    }
    if (gs) gs[i] += load_feat<T>(g, 10);
    o = 11;
  }
  if (prev && gprev) {
    const float2 m = mv[i];
    const float4 w = warp_sample(prev, H, W, n, x, y, m);
    float d0, d1, d2;
    if (kind == 0) {
      d0 = dtonemap_eval(w.x);
      d1 = dtonemap_eval(w.y);
      d2 = dtonemap_eval(w.z);
    } else {
      d0 = 1.f / (1.f + fabsf(w.x));
      d1 = 1.f / (1.f + fabsf(w.y));
      d2 = 1.f / (1.f + fabsf(w.z));
    }
    splat_prev(gprev, H, W, n, x, y, m, load_feat<T>(g, o) * d0, load_feat<T>(g, o + 1) * d1,
               load_feat<T>(g, o + 2) * d2);
  }
  if (glat && mv) {  // the latents enter linearly through the warp
    splat_prev(glat, H, W, n, x, y, mv[i], load_feat<T>(g, o + 4), load_feat<T>(g, o + 5),
               load_feat<T>(g, o + 6), load_feat<T>(g, o + 7), true);
  }
}

// ------------------------------------------------------------------ static mask scratch
// The no-allocation variant of the mask keeps its block sums in this
// file-scope array instead of a caller workspace.  Each device holds its own copy; host code
// reaches it only through the address hipGetSymbolAddress returns for that device (the
// array's name is a host-side stand-in, not a device address).
constexpr size_t kMaskStaticPixels = size_t(1) << 25;  // 33.5M px: four 3840x2160 frames
constexpr size_t kMaskStaticBlocks = kMaskStaticPixels / kMaskBlock;
static __device__ __align__(256) int32_t scratch[kMaskStaticBlocks];  // 128 KiB

constexpr int kMaxDevices = 64;
std::atomic<int32_t*> g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

// The scratch address on the device `stream` belongs to (looked up once per device, with that
// device current); nullptr if a HIP call fails.
int32_t* mask_scratch(hipStream_t st) {
  int dev = -1;
  if (st) {
    if (hipStreamGetDevice(st, &dev) != hipSuccess) return nullptr;
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  int32_t* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (p) return p;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (p) return p;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return nullptr;
  if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
  void* addr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
  if (cur != dev && hipSetDevice(cur) != hipSuccess) return nullptr;
  if (e != hipSuccess || !addr) return nullptr;
  p = static_cast<int32_t*>(addr);
  g_scratch_ptr[dev].store(p, std::memory_order_release);
  return p;
}

// Counts, block sums and the compaction (eq. holdout); the int32 array of nb block sums comes
// from ws or, with use_static, from the device's static scratch.
int sample_mask_impl(const float* s, int N, int H, int W, uint64_t seed, uint32_t frame,
                     const float* u_tex, int tex_size, int rounding, uint8_t* count,
                     int32_t* pixel_offset, int32_t* sample_pixel, int64_t capacity,
                     int32_t* total, float* p_out, void* ws, size_t ws_bytes, bool use_static,
                     uint32_t* dev_status, void* stream) {
  if (N < 0 || H < 0 || W < 0 || capacity < 0) return APS_ERR_SHAPE;
  if (u_tex && (tex_size < 1 || tex_size > kMaxTexSize)) return APS_ERR_ARG;
  if (rounding != APS_ROUND_STOCHASTIC && rounding != APS_ROUND_HOLDOUT &&
      rounding != APS_ROUND_DETERMINISTIC)
    return APS_ERR_ARG;
  const size_t npix = (size_t)N * H * W;
  if (npix > 0x7fffffffull - kMaskBlock) return APS_ERR_SHAPE;  // pixel indices stay in int
  if (use_static && npix > kMaskStaticPixels) return APS_ERR_TOO_LARGE;
  if (!total) return APS_ERR_NULL;
  hipStream_t st = as_stream(stream);
  if (npix == 0) {  // a kernel, not a memset node: safe under stream capture
    k_zero_i32<<<1, 64, 0, st>>>(total);
    APS_LAUNCH_CHECK();
    return APS_OK;
  }
  if (!s || !count || !pixel_offset || (!sample_pixel && capacity > 0)) return APS_ERR_NULL;
  const int nb = (int)((npix + kMaskBlock - 1) / kMaskBlock);
  int32_t* bsum;
  if (use_static) {
    bsum = mask_scratch(st);
    if (!bsum) return APS_ERR_HIP;
  } else {
    if (!ws || ws_bytes < aps_sample_mask_workspace_size(N, H, W)) return APS_ERR_WORKSPACE;
    bsum = static_cast<int32_t*>(ws);
  }
  // every block sum is written (k_mask_count) before it is read (k_mask_compact): nothing has
  // to start at zero
  const USource us{u_tex, (uint32_t)tex_size, (uint32_t)H, (uint32_t)W};
  const int vec = ((reinterpret_cast<uintptr_t>(s) | reinterpret_cast<uintptr_t>(count) |
                    reinterpret_cast<uintptr_t>(pixel_offset) | reinterpret_cast<uintptr_t>(p_out)) &
                   15) == 0;
  k_mask_count<<<nb, 256, 0, st>>>(s, (int)npix, seed, frame, us, rounding, vec, count, p_out,
                                   bsum, dev_status);
  k_mask_compact<<<nb, 256, 0, st>>>(count, (int)npix, vec, bsum, nb, pixel_offset, sample_pixel,
                                     capacity, total, dev_status);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

}  // namespace

// ======================================================================== C ABI
extern "C" {

size_t aps_normalize_workspace_size(int N, int H, int W) {
  const int npx = H * W;
  const int nb = (npx + kNormElems - 1) / kNormElems;
  return (size_t)N * nb * sizeof(float2) + (size_t)N * sizeof(float2) + 256;
}

int aps_normalize_density(const float* z, int N, int H, int W, float budget_spp,
                          float uniform_frac, float* s_out, void* ws, size_t ws_bytes,
                          uint32_t* dev_status, void* stream) {
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!z || !s_out) return APS_ERR_NULL;
  if (!(budget_spp > 0.f) || !(uniform_frac >= 0.f && uniform_frac <= 1.f)) return APS_ERR_ARG;
  if ((size_t)H * W > 0x7fffffffull - kNormApply) return APS_ERR_SHAPE;
  if (ws_bytes < aps_normalize_workspace_size(N, H, W) || !ws) return APS_ERR_WORKSPACE;
  const int npx = H * W;
  const int nb = (npx + kNormElems - 1) / kNormElems;
  float2* part = static_cast<float2*>(ws);
  hipStream_t st = as_stream(stream);
  k_norm_partial<<<dim3(nb, N), 256, 0, st>>>(z, npx, nb, part);
  const float c0 = uniform_frac * budget_spp;
  const float c1 = (1.f - uniform_frac) * budget_spp * (float)npx;
  const int vec = ((reinterpret_cast<uintptr_t>(z) | reinterpret_cast<uintptr_t>(s_out)) & 15) == 0 &&
                  npx % 4 == 0;
  k_norm_apply<<<dim3((npx + kNormApply - 1) / kNormApply, N), 256, 0, st>>>(
      z, npx, part, nb, c0, c1, vec, s_out, dev_status);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

size_t aps_sample_mask_workspace_size(int N, int H, int W) {
  const size_t npix = (size_t)N * H * W;
  const size_t nb = (npix + kMaskBlock - 1) / kMaskBlock;
  return nb * sizeof(int32_t) + 256;
}

int aps_sample_mask(const float* s, int N, int H, int W, uint64_t seed, uint32_t frame,
                    uint8_t* count, int32_t* pixel_offset, int32_t* sample_pixel,
                    int64_t capacity, int32_t* total, float* p_out, void* ws, size_t ws_bytes,
                    uint32_t* dev_status, void* stream) {
  return aps_sample_mask_ex(s, N, H, W, seed, frame, nullptr, 0, APS_ROUND_STOCHASTIC, count,
                            pixel_offset, sample_pixel, capacity, total, p_out, ws, ws_bytes,
                            dev_status, stream);
}

int aps_sample_mask_ex(const float* s, int N, int H, int W, uint64_t seed, uint32_t frame,
                       const float* u_tex, int tex_size, int rounding, uint8_t* count,
                       int32_t* pixel_offset, int32_t* sample_pixel, int64_t capacity,
                       int32_t* total, float* p_out, void* ws, size_t ws_bytes,
                       uint32_t* dev_status, void* stream) {
  return sample_mask_impl(s, N, H, W, seed, frame, u_tex, tex_size, rounding, count, pixel_offset,
                          sample_pixel, capacity, total, p_out, ws, ws_bytes, false, dev_status,
                          stream);
}

int aps_sample_mask_noalloc(const float* s, int N, int H, int W, uint64_t seed, uint32_t frame,
                            const float* u_tex, int tex_size, int rounding, uint8_t* count,
                            int32_t* pixel_offset, int32_t* sample_pixel, int64_t capacity,
                            int32_t* total, float* p_out, uint32_t* dev_status, void* stream) {
  return sample_mask_impl(s, N, H, W, seed, frame, u_tex, tex_size, rounding, count, pixel_offset,
                          sample_pixel, capacity, total, p_out, nullptr, 0, true, dev_status,
                          stream);
}

int aps_fixture_render(const float* pool, int J, const uint8_t* count,
                       const int32_t* pixel_offset, int N, int H, int W, int64_t capacity,
                       float* samples, void* stream) {
  if (J <= 0 || N < 0 || H < 0 || W < 0 || capacity < 0) return APS_ERR_SHAPE;
  const size_t npix = (size_t)N * H * W;
  if (npix == 0) return APS_OK;
  if (!pool || !count || !pixel_offset || (!samples && capacity > 0)) return APS_ERR_NULL;
  if (npix > 0x7fffffffull) return APS_ERR_SHAPE;
  k_fixture_render<<<(int)((npix + 255) / 256), 256, 0, as_stream(stream)>>>(
      reinterpret_cast<const float4*>(pool), J, count, pixel_offset, (int)npix, capacity,
      reinterpret_cast<float4*>(samples));
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_scatter_samples(const float* s, const uint8_t* count, const int32_t* pixel_offset,
                        const float* samples, int64_t n_samples, int N, int H, int W, int levels,
                        int mode,
                        float lambda, uint64_t seed, uint32_t frame, float* const* L,
                        void* stream) {
  if (mode != APS_HARD && mode != APS_RELAXED) return APS_ERR_ARG;
  return aps_scatter_samples_ex(s, count, pixel_offset, samples, n_samples, N, H, W, levels, mode,
                                lambda, seed, frame, nullptr, 0, L, stream);
}

int aps_scatter_samples_ex(const float* s, const uint8_t* count, const int32_t* pixel_offset,
                           const float* samples, int64_t n_samples, int N, int H, int W,
                           int levels, int mode, float param, uint64_t seed, uint32_t frame,
                           const float* u_tex, int tex_size, float* const* L, void* stream) {
  const float lambda = param;
  if (n_samples < 0) return APS_ERR_SHAPE;
  if (u_tex && (tex_size < 1 || tex_size > kMaxTexSize)) return APS_ERR_ARG;
  if (levels < 1 || levels > APS_MAX_LEVELS) return APS_ERR_UNSUPPORTED;
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if (mode < APS_HARD || mode > APS_DASR) return APS_ERR_ARG;
  if (mode == APS_RELAXED && !(param >= 1.f)) return APS_ERR_ARG;
  if (mode == APS_GUMBEL && !(param > 0.f)) return APS_ERR_ARG;
  const int div = 1 << (levels - 1);
  if (H % div || W % div) return APS_ERR_SHAPE;
  if ((size_t)N * H * W > 0x7fffffffull) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!s || !count || !pixel_offset || !L || (!samples && n_samples > 0)) return APS_ERR_NULL;
  LevelPtrs lp{};
  for (int l = 0; l < levels; ++l) {
    if (!L[l]) return APS_ERR_NULL;
    lp.p[l] = reinterpret_cast<float4*>(L[l]);
  }
  const float hfac = mode == APS_RELAXED ? 2.f * lambda / (2.f * lambda - 1.f) : 1.f;
  dim3 grid((W + 15) / 16, (H + 15) / 16, N);
  k_scatter<<<grid, 256, 0, as_stream(stream)>>>(s, count, pixel_offset,
                                                 reinterpret_cast<const float4*>(samples),
                                                 n_samples, H, W, levels, mode, param, hfac, seed,
                                                 frame, USource{u_tex, (uint32_t)tex_size, (uint32_t)H, (uint32_t)W},
                                                 lp);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_assemble_features(int kind, const float* aux, const float* L0, const float* s,
                          const float* prev, const float* mv, int N, int H, int W, int C,
                          int out_dtype, void* out, void* stream) {
  return aps_assemble_features_ex(kind, aux, L0, s, prev, mv, nullptr, N, H, W, C, out_dtype, out,
                                  stream);
}

int aps_assemble_features_ex(int kind, const float* aux, const float* L0, const float* s,
                             const float* prev, const float* mv, const float* lat, int N, int H,
                             int W, int C, int out_dtype, void* out, void* stream) {
  if (kind != APS_FEAT_SAMPLER && kind != APS_FEAT_KERNEL) return APS_ERR_ARG;
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!aux || !out) return APS_ERR_NULL;
  if (kind == APS_FEAT_KERNEL && (!L0 || !s)) return APS_ERR_NULL;
  if (prev && !mv) return APS_ERR_NULL;
  if (lat && !prev) return APS_ERR_NULL;
  const int need = (kind == APS_FEAT_KERNEL ? 11 : 7) + (prev ? 4 : 0) + (lat ? 4 : 0);
  if (C < need || (C != 8 && C != 16 && C != 24)) return APS_ERR_SHAPE;  // 16-byte row vectors
  const size_t npix = (size_t)N * H * W;
  if (npix == 0) return APS_OK;
  const int blocks = (int)((npix + 255) / 256);
  hipStream_t st = as_stream(stream);
  const float4* L4 = reinterpret_cast<const float4*>(L0);
  const float4* P4 = reinterpret_cast<const float4*>(prev);
  const float2* M2 = reinterpret_cast<const float2*>(mv);
  const float4* T4 = reinterpret_cast<const float4*>(lat);
  if (out_dtype == APS_F32)
    k_features<float><<<blocks, 256, 0, st>>>(kind, aux, L4, s, P4, M2, T4, N, H, W, C,
                                              static_cast<float*>(out));
  else if (out_dtype == APS_BF16)
    k_features<uint16_t><<<blocks, 256, 0, st>>>(kind, aux, L4, s, P4, M2, T4, N, H, W, C,
                                                 static_cast<uint16_t*>(out));
  else
    return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

}  // extern "C"

// ======================================================================== backward C ABI
extern "C" {

int aps_scatter_samples_bwd(const float* s, const uint8_t* count, const int32_t* pixel_offset,
                            const float* samples, int64_t n_samples, int N, int H, int W,
                            int levels, int mode, float lambda, uint64_t seed, uint32_t frame,
                            const float* const* grad_L, float* grad_s, int accumulate,
                            void* stream) {
  if (mode != APS_HARD && mode != APS_RELAXED) return APS_ERR_ARG;
  return aps_scatter_samples_bwd_ex(s, count, pixel_offset, samples, n_samples, N, H, W, levels,
                                    mode, lambda, seed, frame, nullptr, 0, nullptr, grad_L, grad_s,
                                    accumulate, stream);
}

int aps_scatter_samples_bwd_ex(const float* s, const uint8_t* count, const int32_t* pixel_offset,
                               const float* samples, int64_t n_samples, int N, int H, int W,
                               int levels, int mode, float param, uint64_t seed, uint32_t frame,
                               const float* u_tex, int tex_size, const float* L_ref,
                               const float* const* grad_L, float* grad_s, int accumulate,
                               void* stream) {
  const float lambda = param;
  if (n_samples < 0) return APS_ERR_SHAPE;
  if (u_tex && (tex_size < 1 || tex_size > kMaxTexSize)) return APS_ERR_ARG;
  if (levels < 1 || levels > APS_MAX_LEVELS) return APS_ERR_UNSUPPORTED;
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if (mode < APS_HARD || mode > APS_DASR) return APS_ERR_ARG;
  if (mode == APS_RELAXED && !(param >= 1.f)) return APS_ERR_ARG;
  if (mode == APS_GUMBEL && !(param > 0.f)) return APS_ERR_ARG;
  const int div = 1 << (levels - 1);
  if (H % div || W % div) return APS_ERR_SHAPE;
  const size_t npix = (size_t)N * H * W;
  if (npix > 0x7fffffffull) return APS_ERR_SHAPE;
  if (npix == 0) return APS_OK;
  if (!s || !count || !pixel_offset || !grad_L || !grad_s || (!samples && n_samples > 0))
    return APS_ERR_NULL;
  if (mode == APS_DASR && !L_ref) return APS_ERR_NULL;
  GradLevels g{};
  for (int l = 0; l < levels; ++l) {
    if (!grad_L[l]) return APS_ERR_NULL;
    g.p[l] = reinterpret_cast<const float4*>(grad_L[l]);
  }
  const float hfac = mode == APS_RELAXED ? 2.f * lambda / (2.f * lambda - 1.f) : 1.f;
  k_scatter_bwd<<<(unsigned)((npix + 255) / 256), 256, 0, as_stream(stream)>>>(
      s, count, pixel_offset, reinterpret_cast<const float4*>(samples), n_samples, N, H, W, levels,
      mode, param, hfac, seed, frame, USource{u_tex, (uint32_t)tex_size, (uint32_t)H, (uint32_t)W},
      reinterpret_cast<const float4*>(L_ref), g, grad_s, accumulate);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

size_t aps_normalize_bwd_workspace_size(int N, int H, int W) {
  const int npx = H * W;
  const int nb = (npx + kNormElems - 1) / kNormElems;
  return (size_t)N * nb * sizeof(float2) + (size_t)N * sizeof(float2) + (size_t)N * nb * 4 +
         (size_t)N * 4 + 1024;
}

int aps_normalize_density_bwd(const float* z, int N, int H, int W, float budget_spp,
                              float uniform_frac, const float* grad_s, float* grad_z, void* ws,
                              size_t ws_bytes, void* stream) {
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!z || !grad_s || !grad_z) return APS_ERR_NULL;
  if (!(budget_spp > 0.f) || !(uniform_frac >= 0.f && uniform_frac <= 1.f)) return APS_ERR_ARG;
  if ((size_t)H * W > 0x7fffffffull) return APS_ERR_SHAPE;
  if (!ws || ws_bytes < aps_normalize_bwd_workspace_size(N, H, W)) return APS_ERR_WORKSPACE;
  const int npx = H * W;
  const int nb = (npx + kNormElems - 1) / kNormElems;
  char* p = static_cast<char*>(ws);
  float2* part = reinterpret_cast<float2*>(p);
  p += (((size_t)N * nb * sizeof(float2)) + 255) / 256 * 256;
  float2* stats = reinterpret_cast<float2*>(p);
  p += (((size_t)N * sizeof(float2)) + 255) / 256 * 256;
  float* gpart = reinterpret_cast<float*>(p);
  p += (((size_t)N * nb * 4) + 255) / 256 * 256;
  float* dots = reinterpret_cast<float*>(p);
  hipStream_t st = as_stream(stream);
  k_norm_partial<<<dim3(nb, N), 256, 0, st>>>(z, npx, nb, part);
  k_norm_combine<<<N, 256, 0, st>>>(part, nb, stats);
  k_norm_gdot_partial<<<dim3(nb, N), 256, 0, st>>>(z, grad_s, npx, nb, stats, gpart);
  k_norm_gdot_combine<<<N, 256, 0, st>>>(gpart, nb, dots);
  const float c1 = (1.f - uniform_frac) * budget_spp * (float)npx;
  k_norm_bwd_apply<<<dim3((npx + 255) / 256, N), 256, 0, st>>>(z, grad_s, npx, stats, dots, c1,
                                                               grad_z);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_assemble_features_bwd(int kind, const float* L0, const float* prev, const float* mv,
                              int N, int H, int W, int C, int feat_dtype, const void* grad_feat,
                              float* grad_L0, float* grad_s, float* grad_prev, void* stream) {
  return aps_assemble_features_bwd_ex(kind, L0, prev, mv, 0, N, H, W, C, feat_dtype, grad_feat,
                                      grad_L0, grad_s, grad_prev, nullptr, stream);
}

int aps_assemble_features_bwd_ex(int kind, const float* L0, const float* prev, const float* mv,
                                 int has_lat, int N, int H, int W, int C, int feat_dtype,
                                 const void* grad_feat, float* grad_L0, float* grad_s,
                                 float* grad_prev, float* grad_lat, void* stream) {
  if (kind != APS_FEAT_SAMPLER && kind != APS_FEAT_KERNEL) return APS_ERR_ARG;
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!grad_feat) return APS_ERR_NULL;
  if (kind == APS_FEAT_KERNEL && !L0) return APS_ERR_NULL;
  if (prev && !mv) return APS_ERR_NULL;
  if (has_lat && !mv) return APS_ERR_NULL;
  const int need = (kind == APS_FEAT_KERNEL ? 11 : 7) + (prev ? 4 : 0) + (has_lat ? 4 : 0);
  if (C < need || C > 24) return APS_ERR_SHAPE;
  if (!has_lat) grad_lat = nullptr;
  const size_t npix = (size_t)N * H * W;
  const unsigned blocks = (unsigned)((npix + 255) / 256);
  hipStream_t st = as_stream(stream);
  const float4* L4 = reinterpret_cast<const float4*>(L0);
  const float4* P4 = reinterpret_cast<const float4*>(prev);
  const float2* M2 = reinterpret_cast<const float2*>(mv);
  float4* G4 = reinterpret_cast<float4*>(grad_L0);
  if (feat_dtype == APS_F32)
    k_features_bwd<float><<<blocks, 256, 0, st>>>(kind, L4, P4, M2, N, H, W, C,
                                                  static_cast<const float*>(grad_feat), G4, grad_s,
                                                  grad_prev, grad_lat);
  else if (feat_dtype == APS_BF16)
    k_features_bwd<uint16_t><<<blocks, 256, 0, st>>>(kind, L4, P4, M2, N, H, W, C,
                                                     static_cast<const uint16_t*>(grad_feat), G4,
                                                     grad_s, grad_prev, grad_lat);
  else
    return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

}  // extern "C"
