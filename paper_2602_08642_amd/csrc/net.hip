// Network entry points: the sampler CNN followed by budget normalisation (Sec. 3,
// Overview), and the kernel-predictor U-Net producing per-level kernel logits (App. A,
// kernel prediction).  Every layer runs in the MFMA convolution of conv.hip; this file
// only sequences launches on the caller's stream and carves the caller's workspace.
#include "aps_common.h"

using namespace aps;

namespace {

size_t esize(int dtype) { return dtype == APS_BF16 ? 2 : 4; }
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int conv(const aps_conv_layer& L, const void* x, const void* x2, int N, int H, int W, int Cx,
         int C2, int mode, int dtype, void* y, int ldy, int y_dtype, void* stream) {
  if (!L.w || !L.b) return APS_ERR_NULL;
  if (L.cin != Cx + C2) return APS_ERR_SHAPE;
  return aps_conv2d_fwd(x, x2, N, H, W, Cx, C2, mode, L.w, L.b, L.cout, L.ksize, L.relu, dtype,
                        y, ldy, y_dtype, stream);
}

#define APS_TRY(expr)            \
  do {                           \
    const int _r = (expr);       \
    if (_r != APS_OK) return _r; \
  } while (0)

const int kUnetConvs = 14;

__device__ inline void load4(const float* p, float* a) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a[0] = v.x;
  a[1] = v.y;
  a[2] = v.z;
  a[3] = v.w;
}
__device__ inline void load4(const uint16_t* p, float* a) {
  const u16x4 v = *reinterpret_cast<const u16x4*>(p);
#pragma unroll
  for (int e = 0; e < 4; ++e) a[e] = bf2f(v[e]);
}
__device__ inline void store4(float* p, const float* v) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ inline void store4(uint16_t* p, const float* v) {
  *reinterpret_cast<u16x4*>(p) = f2bf4(v[0], v[1], v[2], v[3]);
}

// 2x2 block mean of NHWC features, four channels per thread, summed in the order of the conv
// kernels' POOL2 input transform.
template <typename T>
__global__ __launch_bounds__(256) void k_avgpool2(const T* __restrict__ x, int N, int Ho, int Wo,
                                                  int C, T* __restrict__ y) {
  const int cq = C / 4;
  const size_t total = (size_t)N * Ho * Wo * cq;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
    const int q = (int)(i % cq);
    const size_t p = i / cq;
    const int xo = (int)(p % Wo);
    const size_t r = p / Wo;
    const int yo = (int)(r % Ho), n = (int)(r / Ho);
    const size_t W = 2 * (size_t)Wo;
    const size_t o00 = (((size_t)n * 2 * Ho + 2 * yo) * W + 2 * xo) * C + 4 * q;
    float a[4], b[4], c[4], d[4];
    load4(x + o00, a);
    load4(x + o00 + C, b);
    load4(x + o00 + W * C, c);
    load4(x + o00 + W * C + C, d);
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = ((a[e] + b[e]) + (c[e] + d[e])) * 0.25f;
    store4(y + p * C + 4 * q, v);
  }
}

__global__ __launch_bounds__(256) void k_upsample_nearest2(const float* __restrict__ sq, int N,
                                                           int Hq, int Wq, float* __restrict__ s) {
  // one thread per output pair (2x, 2x + 1) of a row
  const size_t total = (size_t)N * 2 * Hq * Wq;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
    const int xq = (int)(i % Wq);
    const size_t r = i / Wq;  // output row index over N * 2Hq
    const int y = (int)(r % (2 * Hq)), n = (int)(r / (2 * Hq));
    const float v = sq[((size_t)n * Hq + y / 2) * Wq + xq];
    *reinterpret_cast<float2*>(s + r * 2 * Wq + 2 * xq) = make_float2(v, v);
  }
}

int grid_for(size_t items) {
  const size_t b = (items + 255) / 256;
  return (int)(b < 65536 ? (b ? b : 1) : 65536);
}

}  // namespace

extern "C" {

size_t aps_density_predict_workspace_size(int N, int H, int W, int width, int dtype) {
  return 2 * align256((size_t)N * H * W * width * esize(dtype)) + align256((size_t)N * H * W * 4) +
         align256(aps_normalize_workspace_size(N, H, W));
}

int aps_density_predict(const aps_net* net, const void* feat, int N, int H, int W, int C,
                        float budget_spp, float uniform_frac, float* z_out, float* s_out,
                        void* ws, size_t ws_bytes, uint32_t* dev_status, void* stream) {
  if (!net) return APS_ERR_NULL;
  if (net->n_layers != 3) return APS_ERR_SHAPE;
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!feat || !s_out) return APS_ERR_NULL;
  const int dt = net->dtype;
  if (dt != APS_F32 && dt != APS_BF16) return APS_ERR_UNSUPPORTED;
  const aps_conv_layer* L = net->layer;
  const int width = L[0].cout;
  if (L[1].cin != width || L[2].cin != L[1].cout || L[2].cout != 1 || L[0].cin != C)
    return APS_ERR_SHAPE;
  const int wmax = width > L[1].cout ? width : L[1].cout;
  if (!ws || ws_bytes < aps_density_predict_workspace_size(N, H, W, wmax, dt)) return APS_ERR_WORKSPACE;
  char* p = static_cast<char*>(ws);
  void* t0 = p;
  p += align256((size_t)N * H * W * wmax * esize(dt));
  void* t1 = p;
  p += align256((size_t)N * H * W * wmax * esize(dt));
  float* z = reinterpret_cast<float*>(p);
  p += align256((size_t)N * H * W * 4);
  if (z_out) z = z_out;
  // the three layers in one kernel when they have the configured shape (16-channel hidden
  // layers with ReLU, linear 1-channel output, 3x3 kernels)
  int fused = APS_ERR_UNSUPPORTED;
  if (L[0].w && L[0].b && L[1].w && L[1].b && L[2].w && L[2].b && width == 16 && L[1].cout == 16 &&
      L[0].ksize == 3 && L[1].ksize == 3 && L[2].ksize == 3 && L[0].relu && L[1].relu && !L[2].relu)
    fused = sampler_cnn(feat, N, H, W, C, C, L[0].w, L[0].b, L[1].w, L[1].b, L[2].w, L[2].b, dt, z,
                        as_stream(stream));
  if (fused != APS_OK) {
    if (fused != APS_ERR_UNSUPPORTED) return fused;
    APS_TRY(conv(L[0], feat, nullptr, N, H, W, C, 0, APS_CONV_DIRECT, dt, t0, width, dt, stream));
    APS_TRY(conv(L[1], t0, nullptr, N, H, W, width, 0, APS_CONV_DIRECT, dt, t1, L[1].cout, dt, stream));
    APS_TRY(conv(L[2], t1, nullptr, N, H, W, L[1].cout, 0, APS_CONV_DIRECT, dt, z, 1, APS_F32, stream));
  }
  return aps_normalize_density(z, N, H, W, budget_spp, uniform_frac, s_out, p,
                               aps_normalize_workspace_size(N, H, W), dev_status, stream);
}

size_t aps_density_predict_bwd_workspace_size(const aps_net* net, int N, int H, int W) {
  if (!net || net->n_layers != 3) return 0;
  const aps_conv_layer* L = net->layer;
  const size_t px = (size_t)N * H * W, e = esize(net->dtype);
  const int c0 = L[0].cout, c1 = L[1].cout;
  const int ld2 = net->dtype == APS_BF16 ? 8 : 4;  // padded 1-channel gradient (16-byte rows)
  size_t wg = 0;
  for (int i = 0; i < 3; ++i) {
    const size_t b = aps_conv2d_bwd_weight_workspace_size(N, H, W, L[i].cin, 0, L[i].cout, L[i].ksize);
    if (b > wg) wg = b;
  }
  return align256(px * c0 * e) + align256(px * c1 * e)          // a0, a1 (post-ReLU)
         + align256(px * 4) + align256(px * 4)                  // z, dLoss/dz
         + align256(px * ld2 * e)                               // dLoss/dz as the last layer's dy
         + align256(px * c1 * e) + align256(px * c0 * e)        // dLoss/da1, dLoss/da0
         + align256(aps_normalize_bwd_workspace_size(N, H, W)) + align256(wg)
         + 256;
}

int aps_density_predict_bwd(const aps_net* net, const void* const* packed_dgrad, const void* feat,
                            int N, int H, int W, int C, float budget_spp, float uniform_frac,
                            const float* grad_s, float* const* grad_w, float* const* grad_b,
                            void* grad_feat, void* ws, size_t ws_bytes, void* stream) {
  if (!net) return APS_ERR_NULL;
  if (net->n_layers != 3) return APS_ERR_SHAPE;
  if (N < 0 || H < 0 || W < 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!feat || !grad_s || !grad_w || !grad_b || !packed_dgrad) return APS_ERR_NULL;
  const int dt = net->dtype;
  if (dt != APS_F32 && dt != APS_BF16) return APS_ERR_UNSUPPORTED;
  const aps_conv_layer* L = net->layer;
  for (int i = 0; i < 3; ++i) {
    if (!L[i].w || !L[i].b || !grad_w[i] || !grad_b[i]) return APS_ERR_NULL;
    if (i > 0 && !packed_dgrad[i]) return APS_ERR_NULL;
  }
  if (grad_feat && !packed_dgrad[0]) return APS_ERR_NULL;
  if (L[0].cin != C || L[1].cin != L[0].cout || L[2].cin != L[1].cout || L[2].cout != 1 ||
      !L[0].relu || !L[1].relu || L[2].relu)
    return APS_ERR_SHAPE;
  if (!ws || ws_bytes < aps_density_predict_bwd_workspace_size(net, N, H, W)) return APS_ERR_WORKSPACE;
  const size_t px = (size_t)N * H * W, e = esize(dt);
  const int c0 = L[0].cout, c1 = L[1].cout;
  const int ld2 = dt == APS_BF16 ? 8 : 4;
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t bytes) {
    void* r = p;
    p += align256(bytes);
    return r;
  };
  void* a0 = take(px * c0 * e);
  void* a1 = take(px * c1 * e);
  float* z = static_cast<float*>(take(px * 4));
  float* gz = static_cast<float*>(take(px * 4));
  void* dy2 = take(px * ld2 * e);
  void* da1 = take(px * c1 * e);
  void* da0 = take(px * c0 * e);
  const size_t nws = aps_normalize_bwd_workspace_size(N, H, W);
  void* nw = take(nws);
  void* wg = p;
  const size_t wg_bytes = ws_bytes - (size_t)(p - static_cast<char*>(ws));
  // forward recomputation, layer by layer (the post-ReLU activations are the ReLU masks and
  // the inputs of the weight gradients)
  APS_TRY(conv(L[0], feat, nullptr, N, H, W, C, 0, APS_CONV_DIRECT, dt, a0, c0, dt, stream));
  APS_TRY(conv(L[1], a0, nullptr, N, H, W, c0, 0, APS_CONV_DIRECT, dt, a1, c1, dt, stream));
  APS_TRY(conv(L[2], a1, nullptr, N, H, W, c1, 0, APS_CONV_DIRECT, dt, z, 1, APS_F32, stream));
  // budget normalisation: dLoss/dz
  APS_TRY(aps_normalize_density_bwd(z, N, H, W, budget_spp, uniform_frac, grad_s, gz, nw, nws,
                                    stream));
  // output layer (linear): dLoss/dz in the network dtype, padded to a 16-byte row
  APS_TRY(aps_copy_channels(gz, APS_F32, 1, dy2, dt, ld2, (int64_t)px, 1, stream));
  APS_TRY(aps_conv2d_bwd_weight(a1, nullptr, APS_CONV_DIRECT, N, H, W, c1, 0, dy2, nullptr, ld2, 1,
                                L[2].ksize, dt, grad_w[2], grad_b[2], wg, wg_bytes, stream));
  APS_TRY(aps_conv2d_bwd_data(dy2, nullptr, ld2, N, H, W, 1, packed_dgrad[2], L[2].ksize, c1, dt,
                              da1, stream));
  // hidden layers: the gradient masked by their ReLU outputs
  APS_TRY(aps_conv2d_bwd_weight(a0, nullptr, APS_CONV_DIRECT, N, H, W, c0, 0, da1, a1, c1, c1,
                                L[1].ksize, dt, grad_w[1], grad_b[1], wg, wg_bytes, stream));
  APS_TRY(aps_conv2d_bwd_data(da1, a1, c1, N, H, W, c1, packed_dgrad[1], L[1].ksize, c0, dt, da0,
                              stream));
  APS_TRY(aps_conv2d_bwd_weight(feat, nullptr, APS_CONV_DIRECT, N, H, W, C, 0, da0, a0, c0, c0,
                                L[0].ksize, dt, grad_w[0], grad_b[0], wg, wg_bytes, stream));
  if (grad_feat)
    APS_TRY(aps_conv2d_bwd_data(da0, a0, c0, N, H, W, c0, packed_dgrad[0], L[0].ksize, C, dt,
                                grad_feat, stream));
  return APS_OK;
}

int aps_avgpool2(const void* x, int N, int H, int W, int C, int dtype, void* y, void* stream) {
  if (N < 0 || H < 0 || W < 0 || C <= 0 || H % 2 || W % 2 || C % 4) return APS_ERR_SHAPE;
  if (dtype != APS_F32 && dtype != APS_BF16) return APS_ERR_UNSUPPORTED;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!x || !y) return APS_ERR_NULL;
  const size_t items = (size_t)N * (H / 2) * (W / 2) * (C / 4);
  if (dtype == APS_F32)
    k_avgpool2<float><<<grid_for(items), 256, 0, as_stream(stream)>>>(
        static_cast<const float*>(x), N, H / 2, W / 2, C, static_cast<float*>(y));
  else
    k_avgpool2<uint16_t><<<grid_for(items), 256, 0, as_stream(stream)>>>(
        static_cast<const uint16_t*>(x), N, H / 2, W / 2, C, static_cast<uint16_t*>(y));
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_upsample_nearest2(const float* s_q, int N, int Hq, int Wq, float* s, void* stream) {
  if (N < 0 || Hq < 0 || Wq < 0) return APS_ERR_SHAPE;
  if ((size_t)N * Hq * Wq == 0) return APS_OK;
  if (!s_q || !s) return APS_ERR_NULL;
  const size_t items = (size_t)N * 2 * Hq * Wq;
  k_upsample_nearest2<<<grid_for(items), 256, 0, as_stream(stream)>>>(s_q, N, Hq, Wq, s);
  APS_LAUNCH_CHECK();
  return APS_OK;
}

size_t aps_kernel_predict_workspace_size(const aps_net* net, int N, int H, int W) {
  if (!net || net->n_layers < kUnetConvs + 1) return 0;
  const aps_conv_layer* L = net->layer;
  const size_t px = (size_t)N * H * W, e = esize(net->dtype);
  const size_t c0 = L[1].cout, c1 = L[3].cout, c2 = L[5].cout, c3 = L[7].cout;
  size_t b = 0;
  b += align256(px * c0 * e);            // e0
  b += align256(px / 4 * c1 * e);        // e1
  b += align256(px / 16 * c2 * e);       // e2
  b += align256(px / 64 * c3 * e);       // e3
  b += align256(px / 4 * c0 * e);        // pooled e0 (input of enc1a)
  b += align256(px / 16 * c1 * e);       // pooled e1
  b += align256(px / 64 * c2 * e);       // pooled e2
  b += align256(px / 16 * c2 * e);       // d2
  b += align256(px / 4 * c1 * e);        // d1
  b += align256(px * c0 * e);            // d0
  size_t t = px * c0;                    // scratch for the first conv of each pair
  if (px / 4 * c1 > t) t = px / 4 * c1;
  if (px / 16 * c2 > t) t = px / 16 * c2;
  if (px / 64 * c3 > t) t = px / 64 * c3;
  b += align256(t * e);
  return b;
}

int aps_kernel_predict(const aps_net* net, const void* feat, int N, int H, int W, int C,
                       int n_heads, void* const* logits, int logit_dtype, const int* kstride,
                       void* ws, size_t ws_bytes, void* stream) {
  return aps_kernel_predict_ex(net, feat, N, H, W, C, n_heads, logits, logit_dtype, kstride,
                               nullptr, -1, ws, ws_bytes, stream);
}

int aps_kernel_predict_ex(const aps_net* net, const void* feat, int N, int H, int W, int C,
                          int n_heads, void* const* logits, int logit_dtype, const int* kstride,
                          void* side0, int side0_offset, void* ws, size_t ws_bytes,
                          void* stream) {
  if (!net) return APS_ERR_NULL;
  if (n_heads < 1 || n_heads > 5 || net->n_layers != kUnetConvs + n_heads) return APS_ERR_SHAPE;
  const int div = n_heads > 4 ? 16 : 8;
  if (N < 0 || H < 0 || W < 0 || H % div || W % div) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!feat || !logits || !kstride) return APS_ERR_NULL;
  const int dt = net->dtype;
  if (dt != APS_F32 && dt != APS_BF16) return APS_ERR_UNSUPPORTED;
  if (logit_dtype != APS_F32 && logit_dtype != dt) return APS_ERR_UNSUPPORTED;
  if (!ws || ws_bytes < aps_kernel_predict_workspace_size(net, N, H, W)) return APS_ERR_WORKSPACE;
  const aps_conv_layer* L = net->layer;
  const int c0 = L[1].cout, c1 = L[3].cout, c2 = L[5].cout, c3 = L[7].cout;
  const size_t px = (size_t)N * H * W, e = esize(dt);
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t bytes) {
    void* r = p;
    p += align256(bytes);
    return r;
  };
  void* e0 = take(px * c0 * e);
  void* e1 = take(px / 4 * c1 * e);
  void* e2 = take(px / 16 * c2 * e);
  void* e3 = take(px / 64 * c3 * e);
  void* p0 = take(px / 4 * c0 * e);
  void* p1 = take(px / 16 * c1 * e);
  void* p2 = take(px / 64 * c2 * e);
  void* d2 = take(px / 16 * c2 * e);
  void* d1 = take(px / 4 * c1 * e);
  void* d0 = take(px * c0 * e);
  void* t = p;
  const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
  // encoder: the second conv of each level also writes its 2x2-pooled output when the kernel
  // supports it, and the next level reads that directly; otherwise the next level pools on load
  auto down = [&](int li, const void* in, int h, int w, int cin, void* skip, int cskip, void* pooled,
                  const void*& next_in, int& next_mode) -> int {
    const aps_conv_layer& A = L[li];
    if (!A.w || !A.b) return APS_ERR_NULL;
    if (A.cin != cin || A.cout != cskip) return APS_ERR_SHAPE;
    const int r = aps_conv2d_fwd_pool(in, nullptr, N, h, w, cin, 0, APS_CONV_DIRECT, A.w, A.b,
                                      A.cout, A.relu, dt, skip, pooled, stream);
    if (r == APS_OK) {
      next_in = pooled;
      next_mode = APS_CONV_DIRECT;
      return APS_OK;
    }
    if (r != APS_ERR_UNSUPPORTED) return r;
    next_in = skip;
    next_mode = APS_CONV_POOL2;
    return conv(A, in, nullptr, N, h, w, cin, 0, APS_CONV_DIRECT, dt, skip, cskip, dt, stream);
  };
  const void* nin = nullptr;
  int nmode = APS_CONV_DIRECT;
  APS_TRY(conv(L[0], feat, nullptr, N, H, W, C, 0, APS_CONV_DIRECT, dt, t, L[0].cout, dt, stream));
  APS_TRY(down(1, t, H, W, L[0].cout, e0, c0, p0, nin, nmode));
  APS_TRY(conv(L[2], nin, nullptr, N, H1, W1, c0, 0, nmode, dt, t, L[2].cout, dt, stream));
  APS_TRY(down(3, t, H1, W1, L[2].cout, e1, c1, p1, nin, nmode));
  APS_TRY(conv(L[4], nin, nullptr, N, H2, W2, c1, 0, nmode, dt, t, L[4].cout, dt, stream));
  APS_TRY(down(5, t, H2, W2, L[4].cout, e2, c2, p2, nin, nmode));
  APS_TRY(conv(L[6], nin, nullptr, N, H3, W3, c2, 0, nmode, dt, t, L[6].cout, dt, stream));
  APS_TRY(conv(L[7], t, nullptr, N, H3, W3, L[6].cout, 0, APS_CONV_DIRECT, dt, e3, c3, dt, stream));
  // decoder: concat [nearest-2x(deeper), skip]
  APS_TRY(conv(L[8], e3, e2, N, H2, W2, c3, c2, APS_CONV_UP2_CAT, dt, t, L[8].cout, dt, stream));
  APS_TRY(conv(L[9], t, nullptr, N, H2, W2, L[8].cout, 0, APS_CONV_DIRECT, dt, d2, c2, dt, stream));
  APS_TRY(conv(L[10], d2, e1, N, H1, W1, c2, c1, APS_CONV_UP2_CAT, dt, t, L[10].cout, dt, stream));
  // dec1b with head1 fused into its epilogue (d1 is stored too: dec0a reads it)
  bool fused1 = false;
  if (n_heads > 1 && logit_dtype == dt && logits && logits[1] && kstride) {
    const aps_conv_layer& A = L[11];
    const aps_conv_layer& Hd = L[kUnetConvs + 1];
    if (A.w && A.b && Hd.w && Hd.b && A.cin == L[10].cout && Hd.cin == A.cout && Hd.ksize == 1 &&
        A.ksize == 3) {
      const int r = aps_conv2d_fwd_head(t, nullptr, N, H1, W1, L[10].cout, 0, APS_CONV_DIRECT, A.w,
                                        A.b, A.cout, A.relu, Hd.w, Hd.b, Hd.cout, dt, d1, c1,
                                        logits[1], kstride[1], stream);
      if (r == APS_OK) fused1 = true;
      else if (r != APS_ERR_UNSUPPORTED) return r;
    }
  }
  if (!fused1)
    APS_TRY(conv(L[11], t, nullptr, N, H1, W1, L[10].cout, 0, APS_CONV_DIRECT, dt, d1, c1, dt, stream));
  APS_TRY(conv(L[12], d1, e0, N, H, W, c1, c0, APS_CONV_UP2_CAT, dt, t, L[12].cout, dt, stream));
  for (int l = 0; l < n_heads; ++l)
    if (!logits[l]) return APS_ERR_NULL;
  // dec0b with head0 fused into its epilogue (d0 feeds nothing else: it is not stored)
  bool fused0 = false;
  if (logit_dtype == dt) {
    const aps_conv_layer& A = L[13];
    const aps_conv_layer& Hd = L[kUnetConvs];
    if (A.w && A.b && Hd.w && Hd.b && A.cin == L[12].cout && Hd.cin == A.cout && Hd.ksize == 1 &&
        A.ksize == 3) {
      const int r = aps_conv2d_fwd_head_ex(t, nullptr, N, H, W, L[12].cout, 0, APS_CONV_DIRECT,
                                           A.w, A.b, A.cout, A.relu, Hd.w, Hd.b, Hd.cout, dt,
                                           nullptr, 0, logits[0], kstride[0], side0, side0_offset,
                                           stream);
      if (r == APS_OK) fused0 = true;
      else if (r != APS_ERR_UNSUPPORTED) return r;
    }
  }
  if (side0 && !fused0) return APS_ERR_UNSUPPORTED;  // the side output comes from the fused head
  if (!fused0)
    APS_TRY(conv(L[13], t, nullptr, N, H, W, L[12].cout, 0, APS_CONV_DIRECT, dt, d0, c0, dt, stream));
  // remaining 1x1 heads (head 4 reads the bottleneck through the 2x2-pool input transform)
  const void* feats[5] = {d0, d1, d2, e3, e3};
  const int fc[5] = {c0, c1, c2, c3, c3};
  for (int l = 0; l < n_heads; ++l) {
    if ((l == 0 && fused0) || (l == 1 && fused1)) continue;
    APS_TRY(conv(L[kUnetConvs + l], feats[l], nullptr, N, H >> l, W >> l, fc[l], 0,
                 l == 4 ? APS_CONV_POOL2 : APS_CONV_DIRECT, dt, logits[l], kstride[l],
                 logit_dtype, stream));
  }
  return APS_OK;
}

}  // extern "C"
