// Learned demodulation (Sec. 6.2): the denoiser predicts a three-channel map d = exp(z) per pixel
// (z: three channels of the level-0 logits, clamped to [-8, 8]); the noisy radiance is divided by
// d before the pyramid is built and filtered, and the reconstruction is multiplied by d.
#include "aps_common.h"

using namespace aps;

namespace {

constexpr float kZMax = 8.f;

struct ZRef {  // three channels of a [N, H, W, stride] logits tensor, from channel offset
  const void* p;
  int dtype, stride, offset;
};

__device__ inline void load_z(const ZRef& z, size_t i, float (&v)[3]) {
  const size_t o = i * (size_t)z.stride + z.offset;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    v[c] = z.dtype == APS_BF16 ? bf2f(static_cast<const uint16_t*>(z.p)[o + c])
                               : static_cast<const float*>(z.p)[o + c];
}

// d = exp(clamp(z)); live = 0 where the clamp is active (no gradient reaches z there)
__device__ inline float dmap(float z, float& live) {
  live = fabsf(z) < kZMax ? 1.f : 0.f;
  return expf(fminf(fmaxf(z, -kZMax), kZMax));
}

// L0 / d and its 2x2 block-mean pyramid (App. A eq. app-pyramid), reduced in LDS per 16x16 tile.
__global__ __launch_bounds__(256) void k_demodulate(const float4* __restrict__ L0, ZRef z, int H,
                                                    int W, int levels, LevelPtrs Lp) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int x = blockIdx.x * 16 + tx, y = blockIdx.y * 16 + ty, n = blockIdx.z;
  __shared__ float4 tile[16][17];
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (x < W && y < H) {
    const size_t i = ((size_t)n * H + y) * W + x;
    float zv[3], live;
    load_z(z, i, zv);
    const float4 l = L0[i];
    v = make_float4(l.x / dmap(zv[0], live), l.y / dmap(zv[1], live), l.z / dmap(zv[2], live), 0.f);
    Lp.p[0][i] = v;
  }
  tile[ty][tx] = v;
  int Hl = H, Wl = W;
  for (int l = 1; l < levels; ++l) {
    __syncthreads();
    const int t = 16 >> l;
    Hl >>= 1;
    Wl >>= 1;
    float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
    if (tx < t && ty < t) {
      const float4 a = tile[2 * ty][2 * tx], b = tile[2 * ty][2 * tx + 1];
      const float4 c = tile[2 * ty + 1][2 * tx], d = tile[2 * ty + 1][2 * tx + 1];
      m = make_float4(((a.x + b.x) + (c.x + d.x)) * 0.25f, ((a.y + b.y) + (c.y + d.y)) * 0.25f,
                      ((a.z + b.z) + (c.z + d.z)) * 0.25f, 0.f);
    }
    __syncthreads();
    if (tx < t && ty < t) {
      tile[ty][tx] = m;
      const int xl = blockIdx.x * t + tx, yl = blockIdx.y * t + ty;
      if (xl < Wl && yl < Hl) Lp.p[l][((size_t)n * Hl + yl) * Wl + xl] = m;
    }
  }
}

// in and out may be the same buffer: each thread reads and writes only its own pixel.  With
// lat_offset >= 0 the four latent channels of the same logit row are copied to lat (float4).
__global__ __launch_bounds__(256) void k_remodulate(const float4* in, ZRef z, size_t npix,
                                                    float4* out, int lat_offset,
                                                    float4* __restrict__ lat) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npix) return;
  float zv[3], live;
  load_z(z, i, zv);
  const float4 v = in[i];
  out[i] = make_float4(v.x * dmap(zv[0], live), v.y * dmap(zv[1], live), v.z * dmap(zv[2], live), 0.f);
  if (lat) {
    const size_t o = i * (size_t)z.stride + lat_offset;
    float t[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      t[c] = z.dtype == APS_BF16 ? bf2f(static_cast<const uint16_t*>(z.p)[o + c])
                                 : static_cast<const float*>(z.p)[o + c];
    lat[i] = make_float4(t[0], t[1], t[2], t[3]);
  }
}

struct GradPtrs {
  const float4* p[APS_MAX_LEVELS];
};

// dLoss/dLd0 collects dLoss/dLd^l / 4^l from every ancestor; Ld0 = L0 / d gives
// dLoss/dL0 = g / d and dLoss/dz = -g Ld0 (d = exp z).
__global__ __launch_bounds__(256) void k_demodulate_bwd(const float4* __restrict__ L0, ZRef z,
                                                        int N, int H, int W, int levels, GradPtrs g,
                                                        float4* __restrict__ gL0,
                                                        float* __restrict__ gz, int accumulate) {
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
  float zv[3], live[3];
  load_z(z, i, zv);
  const float d0 = dmap(zv[0], live[0]), d1 = dmap(zv[1], live[1]), d2 = dmap(zv[2], live[2]);
  const float4 l = L0[i];
  float4 a = make_float4(ge.x / d0, ge.y / d1, ge.z / d2, 0.f);
  const float b0 = -ge.x * (l.x / d0) * live[0], b1 = -ge.y * (l.y / d1) * live[1],
              b2 = -ge.z * (l.z / d2) * live[2];
  if (accumulate) {
    const float4 p = gL0[i];
    a.x += p.x;
    a.y += p.y;
    a.z += p.z;
  }
  gL0[i] = a;
  float* q = gz + 3 * i;
  q[0] = (accumulate ? q[0] : 0.f) + b0;
  q[1] = (accumulate ? q[1] : 0.f) + b1;
  q[2] = (accumulate ? q[2] : 0.f) + b2;
}

// out = d * in: dLoss/din = g d, dLoss/dz = g * out
__global__ __launch_bounds__(256) void k_remodulate_bwd(const float4* __restrict__ in, ZRef z,
                                                        size_t npix, const float4* __restrict__ g,
                                                        float4* __restrict__ gin,
                                                        float* __restrict__ gz, int accumulate) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npix) return;
  float zv[3], live[3];
  load_z(z, i, zv);
  const float d0 = dmap(zv[0], live[0]), d1 = dmap(zv[1], live[1]), d2 = dmap(zv[2], live[2]);
  const float4 v = in[i], gv = g[i];
  float4 a = make_float4(gv.x * d0, gv.y * d1, gv.z * d2, 0.f);
  const float b0 = gv.x * v.x * d0 * live[0], b1 = gv.y * v.y * d1 * live[1],
              b2 = gv.z * v.z * d2 * live[2];
  if (accumulate) {
    const float4 p = gin[i];
    a.x += p.x;
    a.y += p.y;
    a.z += p.z;
  }
  gin[i] = a;
  float* q = gz + 3 * i;
  q[0] = (accumulate ? q[0] : 0.f) + b0;
  q[1] = (accumulate ? q[1] : 0.f) + b1;
  q[2] = (accumulate ? q[2] : 0.f) + b2;
}

int check_z(int z_dtype, int z_stride, int z_offset) {
  if (z_dtype != APS_F32 && z_dtype != APS_BF16) return APS_ERR_UNSUPPORTED;
  if (z_offset < 0 || z_stride < z_offset + 3) return APS_ERR_SHAPE;
  return APS_OK;
}

}  // namespace

extern "C" {

int aps_demodulate(const float* L0, const void* z, int z_dtype, int z_stride, int z_offset, int N,
                   int H, int W, int levels, float* const* Ld, void* stream) {
  if (levels < 1 || levels > APS_MAX_LEVELS) return APS_ERR_UNSUPPORTED;
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  const int div = 1 << (levels - 1);
  if (H % div || W % div) return APS_ERR_SHAPE;
  const int zr = check_z(z_dtype, z_stride, z_offset);
  if (zr != APS_OK) return zr;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!L0 || !z || !Ld) return APS_ERR_NULL;
  LevelPtrs lp{};
  for (int l = 0; l < levels; ++l) {
    if (!Ld[l]) return APS_ERR_NULL;
    lp.p[l] = reinterpret_cast<float4*>(Ld[l]);
  }
  dim3 grid((W + 15) / 16, (H + 15) / 16, N);
  k_demodulate<<<grid, 256, 0, as_stream(stream)>>>(reinterpret_cast<const float4*>(L0),
                                                    ZRef{z, z_dtype, z_stride, z_offset}, H, W,
                                                    levels, lp);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_remodulate(const float* in, const void* z, int z_dtype, int z_stride, int z_offset,
                   int lat_offset, int N, int H, int W, float* out, float* lat_out, void* stream) {
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  const int zr = check_z(z_dtype, z_stride, z_offset);
  if (zr != APS_OK) return zr;
  if (lat_out && (lat_offset < 0 || z_stride < lat_offset + 4)) return APS_ERR_SHAPE;
  const size_t npix = (size_t)N * H * W;
  if (npix == 0) return APS_OK;
  if (!in || !z || !out) return APS_ERR_NULL;
  k_remodulate<<<(unsigned)((npix + 255) / 256), 256, 0, as_stream(stream)>>>(
      reinterpret_cast<const float4*>(in), ZRef{z, z_dtype, z_stride, z_offset}, npix,
      reinterpret_cast<float4*>(out), lat_offset, reinterpret_cast<float4*>(lat_out));
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_demodulate_bwd(const float* L0, const void* z, int z_dtype, int z_stride, int z_offset,
                       int N, int H, int W, int levels, const float* const* grad_Ld,
                       float* grad_L0, float* grad_z, int accumulate, void* stream) {
  if (levels < 1 || levels > APS_MAX_LEVELS) return APS_ERR_UNSUPPORTED;
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  const int div = 1 << (levels - 1);
  if (H % div || W % div) return APS_ERR_SHAPE;
  const int zr = check_z(z_dtype, z_stride, z_offset);
  if (zr != APS_OK) return zr;
  const size_t npix = (size_t)N * H * W;
  if (npix == 0) return APS_OK;
  if (!L0 || !z || !grad_Ld || !grad_L0 || !grad_z) return APS_ERR_NULL;
  GradPtrs g{};
  for (int l = 0; l < levels; ++l) {
    if (!grad_Ld[l]) return APS_ERR_NULL;
    g.p[l] = reinterpret_cast<const float4*>(grad_Ld[l]);
  }
  k_demodulate_bwd<<<(unsigned)((npix + 255) / 256), 256, 0, as_stream(stream)>>>(
      reinterpret_cast<const float4*>(L0), ZRef{z, z_dtype, z_stride, z_offset}, N, H, W, levels,
      g, reinterpret_cast<float4*>(grad_L0), grad_z, accumulate);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_remodulate_bwd(const float* in, const void* z, int z_dtype, int z_stride, int z_offset,
                       int N, int H, int W, const float* grad_out, float* grad_in, float* grad_z,
                       int accumulate, void* stream) {
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  const int zr = check_z(z_dtype, z_stride, z_offset);
  if (zr != APS_OK) return zr;
  const size_t npix = (size_t)N * H * W;
  if (npix == 0) return APS_OK;
  if (!in || !z || !grad_out || !grad_in || !grad_z) return APS_ERR_NULL;
  k_remodulate_bwd<<<(unsigned)((npix + 255) / 256), 256, 0, as_stream(stream)>>>(
      reinterpret_cast<const float4*>(in), ZRef{z, z_dtype, z_stride, z_offset}, npix,
      reinterpret_cast<const float4*>(grad_out), reinterpret_cast<float4*>(grad_in), grad_z,
      accumulate);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

}  // extern "C"
