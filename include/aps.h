/* libaps -- sub-1-spp adaptive sampling and gathering-pyramid reconstruction on MI355X.
 *
 * C ABI of the per-frame hot path of "Forget Superresolution, Sample Adaptively (when
 * Path Tracing)" (arXiv 2602.08642).  Every entry point:
 *   - takes DEVICE pointers owned by the caller (no pointer is retained after return),
 *     NHWC contiguous, batch-major, 16-byte aligned;
 *   - enqueues its kernels on `stream` (a hipStream_t; NULL = the null stream) and never
 *     synchronises;
 *   - validates its arguments on the host first and returns an aps_status code; nothing
 *     is launched when the code is not APS_OK.  Conditions only the device can see set
 *     bits in the optional caller-provided `dev_status` word (APS_STATUS_*), via atomic OR;
 *   - allocates nothing: scratch comes from the caller's workspace `ws` of `ws_bytes`
 *     (query with the matching *_workspace_size function); the one exception,
 *     aps_sample_mask_noalloc, uses a fixed static device array instead.
 * An empty problem (N, H or W == 0) returns APS_OK after the size checks, before any pointer
 * check, and launches nothing (aps_sample_mask only sets *total = 0).
 * Radiance buffers are RGBA float32 (16-byte pixels, A unused and written as 0).
 * Densities, counts and offsets are indexed by the global pixel id n*H*W + y*W + x.
 */
#ifndef APS_H
#define APS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum aps_status {
  APS_OK = 0,
  APS_ERR_NULL = 1,        /* a required pointer is NULL */
  APS_ERR_SHAPE = 2,       /* sizes inconsistent or outside the documented limits */
  APS_ERR_UNSUPPORTED = 3, /* a kernel size / dtype / level count with no compiled kernel */
  APS_ERR_WORKSPACE = 4,   /* ws missing or smaller than the query returns */
  APS_ERR_HIP = 5,         /* a HIP launch or runtime call failed */
  APS_ERR_ARG = 6,         /* a scalar argument is out of range */
  APS_ERR_TOO_LARGE = 7    /* larger than the static scratch of a no-allocation entry point */
};

enum aps_dtype { APS_F32 = 0, APS_BF16 = 1 };
enum aps_mode {
  APS_HARD = 0,
  APS_RELAXED = 1,
  APS_STRAIGHT_THROUGH = 2, /* compared estimators (Sec. 4.1, 4.3): see aps_scatter_samples_ex */
  APS_GUMBEL = 3,
  APS_DASR = 4
};
enum aps_rounding { APS_ROUND_STOCHASTIC = 0, APS_ROUND_HOLDOUT = 1, APS_ROUND_DETERMINISTIC = 2 };
enum aps_feature_kind { APS_FEAT_SAMPLER = 0, APS_FEAT_KERNEL = 1 };
enum aps_conv_mode { APS_CONV_DIRECT = 0, APS_CONV_POOL2 = 1, APS_CONV_UP2_CAT = 2 };

#define APS_MAX_LEVELS 5
#define APS_MAX_NET_LAYERS 20

/* device status bits */
#define APS_STATUS_COUNT_OVERFLOW 1u /* floor(s) > 254: count clamped to 255 */
#define APS_STATUS_NONFINITE 2u      /* a density was NaN, infinite or negative */
#define APS_STATUS_CAPACITY 4u       /* the sample list capacity was too small */

const char* aps_status_string(int status);
int aps_version(void); /* major*10000 + minor*100 + patch */

/* ---------------------------------------------------------------- networks
 * One conv layer: packed weights (aps_conv_pack_weights), bias [cout] float32.
 * A network is an ordered list of layers sharing one compute dtype.
 *   sampler CNN (3 layers):  d0 (C->16, ReLU), d1 (16->16, ReLU), d2 (16->1)
 *   U-Net (14 + n_heads):    enc0a enc0b enc1a enc1b enc2a enc2b bota botb
 *                            dec2a dec2b dec1a dec1b dec0a dec0b head0 .. head{n-1}
 */
typedef struct {
  const void* w;
  const float* b;
  int cin, cout, ksize, relu;
} aps_conv_layer;

typedef struct {
  int n_layers;
  int dtype; /* APS_F32 or APS_BF16: weights and activations; accumulation is fp32 */
  aps_conv_layer layer[APS_MAX_NET_LAYERS];
} aps_net;

/* Elements of the packed weight buffer of one layer (0 for unsupported sizes). */
size_t aps_conv_packed_elems(int Cout, int ksize, int Cin);

/* Pack OHWI float32 weights w[Cout][k][k][Cin] (device) into MFMA fragment order, in
 * dtype (bf16: round to nearest even).  packed holds aps_conv_packed_elems elements. */
int aps_conv_pack_weights(const float* w, int Cout, int ksize, int Cin, int dtype, void* packed,
                          void* stream);

/* 'Same' convolution (ksize 1 or 3, zero padding) + bias (+ ReLU), NHWC, output [N,H,W]
 * with row stride ldy >= Cout channels (channels [Cout, round_up(Cout,4)) are written 0 when
 * ldy allows).  Input transform `mode`:
 *   APS_CONV_DIRECT : x [N,H,W,Cx]
 *   APS_CONV_POOL2  : x [N,2H,2W,Cx], 2x2 average-pooled on the fly
 *   APS_CONV_UP2_CAT: x [N,H/2,W/2,Cx] nearest-2x upsampled, concatenated with x2 [N,H,W,C2]
 *                     (channels [0,Cx) from x, [Cx,Cx+C2) from x2)
 * Cx and C2 must be multiples of 8.  dtype/y_dtype: (F32,F32), (BF16,BF16) or (BF16,F32).
 * For 3x3 layers with Cx + C2 > 16, Cout a multiple of 16 above 16, ldy a multiple of 4 and
 * (F32,F32) or (BF16,BF16), the fp32 sum of each output has one order whichever kernel the
 * shape selects (the bias, then 16-channel (fp32) or 32-channel (bf16) input chunks, taps dx
 * outer and dy inner), so this call, the main output of aps_conv2d_fwd_head(_ex) and y of
 * aps_conv2d_fwd_pool agree bit for bit. */
int aps_conv2d_fwd(const void* x, const void* x2, int N, int H, int W, int Cx, int C2, int mode,
                   const void* packed_w, const float* bias, int Cout, int ksize, int relu,
                   int dtype, void* y, int ldy, int y_dtype, void* stream);

/* A 3x3 conv (input as aps_conv2d_fwd, dtype APS_BF16 or APS_F32 for inputs, weights and
 * outputs, Cx + C2 > 16, Cout a multiple of 16 and > 16, H and W even, output row stride Cout)
 * that also writes the 2x2 average pool of its output: pooled [N,H/2,W/2,Cout], equal bit for
 * bit to the APS_CONV_POOL2 input transform of the next layer applied to y (the U-Net's down
 * path: Sec. 6.3, App. A).  Returns APS_ERR_UNSUPPORTED for other shapes; the caller then pools
 * in the consumer. */
int aps_conv2d_fwd_pool(const void* x, const void* x2, int N, int H, int W, int Cx, int C2,
                        int mode, const void* packed_w, const float* bias, int Cout, int relu,
                        int dtype, void* y, void* pooled, void* stream);

/* A 3x3 conv (Cout 32 or 64, input as aps_conv2d_fwd, Cx + C2 > 16) with a 1x1 head
 * (K <= 64 outputs, packed_head from aps_conv_pack_weights(.., K, 1, Cout, ..)) applied to its
 * output in the same kernel: logits [N,H,W,kstride] = head(y).  y (nullable) receives the
 * conv output itself [N,H,W,ldy]; when NULL it is not written.  Inputs, y and logits share
 * dtype.  The logits equal those of the two separate calls bit for bit. */
int aps_conv2d_fwd_head(const void* x, const void* x2, int N, int H, int W, int Cx, int C2,
                        int mode, const void* packed_w, const float* bias, int Cout, int relu,
                        const void* packed_head, const float* head_bias, int K, int dtype,
                        void* y, int ldy, void* logits, int kstride, void* stream);
/* The same with a side output for learned demodulation (Sec. 6.2): side [N,H,W,4] (dtype)
 * receives logit channels [side_offset, side_offset + 3) of every pixel and a 0, the
 * compact demodulation map that aps_demodulate reads with z_stride 4 and z_offset 0 instead
 * of whole logit rows.  side NULL: as aps_conv2d_fwd_head.  Requires side_offset + 3 <= K;
 * APS_ERR_UNSUPPORTED unless kstride <= 64, kstride * element size is a multiple of 16 bytes,
 * logits is 16-byte aligned and side aligned to one pixel (8 or 16 bytes). */
int aps_conv2d_fwd_head_ex(const void* x, const void* x2, int N, int H, int W, int Cx, int C2,
                           int mode, const void* packed_w, const float* bias, int Cout, int relu,
                           const void* packed_head, const float* head_bias, int K, int dtype,
                           void* y, int ldy, void* logits, int kstride, void* side,
                           int side_offset, void* stream);

/* ---------------------------------------------------------------- a1 + a2: density
 * Sec. 3 (Overview): the sampler predicts one channel z; s = f*B + (1-f)*B*Npx*softmax(z)
 * with the softmax over the H*W pixels of each frame, so sum(s) = Npx*B and s >= f*B
 * (f = 1/8 in the paper).  The reduction is a fixed tree: results are deterministic. */
size_t aps_normalize_workspace_size(int N, int H, int W);
int aps_normalize_density(const float* z, int N, int H, int W, float budget_spp,
                          float uniform_frac, float* s_out, void* ws, size_t ws_bytes,
                          uint32_t* dev_status, void* stream);

/* Sampler CNN on features feat [N,H,W,C] (dtype of the net) -> z (optional, float32 [N,H,W])
 * -> s float32 [N,H,W].  The configured shape (3x3 layers Cin -> 16 -> 16 -> 1, ReLU on the
 * hidden layers) runs as one kernel; in bf16 it addresses one image's features with 32-bit
 * byte offsets, so H*W*C*2 < 2^31 (APS_ERR_SHAPE otherwise). */
size_t aps_density_predict_workspace_size(int N, int H, int W, int width, int dtype);
int aps_density_predict(const aps_net* net, const void* feat, int N, int H, int W, int C,
                        float budget_spp, float uniform_frac, float* z_out, float* s_out,
                        void* ws, size_t ws_bytes, uint32_t* dev_status, void* stream);

/* Quarter-resolution density map (Sec. 7, density-map resolution): the sampler runs on the
 * 2x2 block means of the features and each full-resolution pixel takes its block's density.
 * aps_avgpool2: x [N,H,W,C] -> y [N,H/2,W/2,C], y = ((x00 + x01) + (x10 + x11)) * 0.25 in
 * float32, stored in dtype (APS_F32 or APS_BF16, round to nearest even); H, W even, C a
 * multiple of 4.  aps_upsample_nearest2: s_q float32 [N,Hq,Wq] -> s [N,2Hq,2Wq],
 * s[n][y][x] = s_q[n][y/2][x/2].  Normalising z_q with the full-resolution budget B per pixel
 * keeps sum(s) = 4 * sum(s_q) = Npx * B.  Device pointers; no workspace; APS_ERR_SHAPE for odd
 * H or W or C % 4 != 0, APS_ERR_UNSUPPORTED for other dtypes. */
int aps_avgpool2(const void* x, int N, int H, int W, int C, int dtype, void* y, void* stream);
int aps_upsample_nearest2(const float* s_q, int N, int Hq, int Wq, float* s, void* stream);

/* ---------------------------------------------------------------- a3: sample mask
 * Sec. 4.2, eq. holdout: count = floor(s) + [u < p], p = s - floor(s) (exact in binary32),
 * u = (w >> 8) * 2^-24 with w the word (pixel mod 4) of Philox4x32-10(key = seed,
 * counter = (pixel div 4, frame, 0, 0)): one block serves four consecutive pixels.
 * Outputs: count uint8 [N,H,W]; pixel_offset int32 [N,H,W] = exclusive prefix sum of count
 * in pixel order; sample_pixel int32 [capacity] = the pixel id of every requested sample,
 * ascending (the renderer's request list); total int32 (device) = sum of counts; p_out
 * (optional) float32 [N,H,W].  Bit-exact and deterministic.  N*H*W <= 2^31 - 1 - 1024.
 * Capacity N*H*W*(B + 1) always suffices for budget-normalised s; entries past capacity are
 * dropped and flagged APS_STATUS_CAPACITY. */
size_t aps_sample_mask_workspace_size(int N, int H, int W);
int aps_sample_mask(const float* s, int N, int H, int W, uint64_t seed, uint32_t frame,
                    uint8_t* count, int32_t* pixel_offset, int32_t* sample_pixel,
                    int64_t capacity, int32_t* total, float* p_out, void* ws, size_t ws_bytes,
                    uint32_t* dev_status, void* stream);

/* The mask with two options.  u: from a blue-noise threshold texture (Sec. 6.3 dithers with
 * blue noise): u_tex float32 [tex_size][tex_size] on the device (e.g. void-and-cluster
 * thresholds (rank + 1/2) / tex_size^2), tiled over each image with a toroidal offset per image
 * and frame, (ox, oy) = (word0, word1) mod tex_size of Philox4x32-10(key = seed,
 * counter = (n, frame, 2, 0)): u[n][y][x] = u_tex[(y + oy) mod T][(x + ox) mod T]; u_tex == NULL
 * gives the Philox u above.  rounding: APS_ROUND_STOCHASTIC count = floor(s) + [u < p] (as
 * above); APS_ROUND_HOLDOUT count = floor(s) + [p > 0], the holdout requested for every pixel
 * with p > 0 (what the straight-through and Gumbel-Softmax scatter modes read);
 * APS_ROUND_DETERMINISTIC count = round(s) = floor(s) + [p >= 1/2] (Sec. 4.1 eq. kuz_fw, the
 * DASR mode).  APS_ERR_ARG for tex_size outside 1..4096 with a texture, or another rounding.
 * The caller keeps u_tex alive until the work on the stream has finished. */
int aps_sample_mask_ex(const float* s, int N, int H, int W, uint64_t seed, uint32_t frame,
                       const float* u_tex, int tex_size, int rounding, uint8_t* count,
                       int32_t* pixel_offset, int32_t* sample_pixel, int64_t capacity,
                       int32_t* total, float* p_out, void* ws, size_t ws_bytes,
                       uint32_t* dev_status, void* stream);

/* No-allocation variant of aps_sample_mask_ex, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as aps_sample_mask_ex without ws / ws_bytes: the block
 * sums live in a static device array of the library (128 KiB per device,
 * kept until the process ends; its address is looked up on the stream's device at the first
 * call there).  Limit: N*H*W <= 2^25 pixels (four 3840x2160 frames), else APS_ERR_TOO_LARGE
 * before anything is launched.  Nothing in the array has to start at zero (every entry is
 * written before it is read).  All calls on one device share the array: calls that overlap
 * on one GPU (on different streams, or from different host threads) race; calls ordered on
 * one stream do not. */
int aps_sample_mask_noalloc(const float* s, int N, int H, int W, uint64_t seed, uint32_t frame,
                            const float* u_tex, int tex_size, int rounding, uint8_t* count,
                            int32_t* pixel_offset, int32_t* sample_pixel, int64_t capacity,
                            int32_t* total, float* p_out, uint32_t* dev_status, void* stream);

/* Renderer stand-in (not part of the method): writes sample j of pixel i as
 * pool[i][j mod J] (pool float32 [N*H*W][J][4]) at samples[pixel_offset[i] + j]. */
int aps_fixture_render(const float* pool, int J, const uint8_t* count,
                       const int32_t* pixel_offset, int N, int H, int W, int64_t capacity,
                       float* samples, void* stream);

/* ---------------------------------------------------------------- a4: scatter + pyramid
 * Sec. 4.2 eq. stoch_rnoisy: L0 = (sum_{j<floor(s)} S_j + H) / s (0 where s == 0), with
 * the holdout S_floor(s) taken iff count > floor(s):
 *   APS_HARD:    H = S_floor(s)
 *   APS_RELAXED: H = S_floor(s) * h * clamp(lambda * (p - u) / p, 0, 1), h = 2 lambda/(2 lambda - 1)
 *   (Sec. 4.3 eqs. relaxed_holdout, h_factor, with the variate mirrored u -> 1 - u so the
 *    ramp is non-zero exactly when u < p; u is regenerated from (seed, frame)).
 * App. A eq. app-pyramid: L[l] = 2^l x 2^l block means of L0, l < levels.
 * samples float32 [n_samples][4] in request order (entries at or past n_samples, which
 * only a mask that overflowed its capacity requests, contribute 0); L[l] float32 RGBA
 * [N, H>>l, W>>l].  H and W must be divisible by 2^(levels-1). */
int aps_scatter_samples(const float* s, const uint8_t* count, const int32_t* pixel_offset,
                        const float* samples, int64_t n_samples, int N, int H, int W, int levels,
                        int mode,
                        float lambda, uint64_t seed, uint32_t frame, float* const* L,
                        void* stream);
/* aps_scatter_samples with more modes and the optional u texture of aps_sample_mask_ex (pass
 * the texture the mask was drawn with).  The holdout (sample floor(s) of the pixel, when
 * requested) enters with weight w:
 *   APS_HARD, APS_RELAXED: as above (param = lambda >= 1 for RELAXED); APS_ROUND_STOCHASTIC masks;
 *   APS_STRAIGHT_THROUGH: w = [u < p] (the hard forward; its backward takes dw/dp = 1);
 *   APS_GUMBEL: w = sigmoid((logit p - logit u) / tau), tau = param > 0 (the binary
 *     Gumbel-Softmax relaxation the paper contrasts with its ramp, Sec. 4.3);
 *   both with APS_ROUND_HOLDOUT masks, so the holdout of every pixel with p > 0 is present;
 *   APS_DASR (Sec. 4.1 eq. kuz_fw): L0 = mean of the count requested samples (0 for count 0),
 *     with APS_ROUND_DETERMINISTIC masks. */
int aps_scatter_samples_ex(const float* s, const uint8_t* count, const int32_t* pixel_offset,
                           const float* samples, int64_t n_samples, int N, int H, int W,
                           int levels, int mode, float param, uint64_t seed, uint32_t frame,
                           const float* u_tex, int tex_size, float* const* L, void* stream);

/* Network inputs (C <= 16 channels, zero padded), out [N,H,W,C] in out_dtype.
 *   APS_FEAT_SAMPLER: aux[0..6], then with prev: tonemap(W prev) RGB, valid
 *   APS_FEAT_KERNEL : aux[0..6], slog1p(L0) RGB, s, then with prev: slog1p(W prev) RGB, valid
 * aux float32 [N,H,W,8] (albedo 3, normal 3, log-depth 1, pad); C is 8 or 16 (24 with
 * latents, below); W prev = bilinear warp of the
 * previous output along mv (see aps_reproject); valid = the back-projected position lies in
 * the frame; slog1p(v) = sign(v) log(1+|v|); tonemap = the evaluation filmic curve of Sec. 5
 * (s = h = 0.5, contrast 0.4, exposure 0, saturation 1) followed by the sRGB transfer. */
int aps_assemble_features(int kind, const float* aux, const float* L0, const float* s,
                          const float* prev, const float* mv, int N, int H, int W, int C,
                          int out_dtype, void* out, void* stream);
/* The same with the recurrent latents (Sec. 3: the sampler and the denoiser share a latent
 * feature space fed forward from the previous frame): lat float32 [N,H,W,4] (the previous
 * frame's latents, see aps_remodulate) warped along mv like prev and appended as 4 channels
 * after the temporal ones (requires prev); C is 8, 16 or 24. */
int aps_assemble_features_ex(int kind, const float* aux, const float* L0, const float* s,
                             const float* prev, const float* mv, const float* lat, int N, int H,
                             int W, int C, int out_dtype, void* out, void* stream);

/* ---------------------------------------------------------------- a5: kernel prediction
 * U-Net (2 x (3x3 conv + ReLU) per level, 2x2 average pool down, nearest-2x up + concat
 * [up, skip]) with 1x1 heads: logits[l] [N, H>>l, W>>l, kstride[l]] in logit_dtype (F32 or
 * the net's dtype) for l < n_heads (1..5).  Heads 0-2 read the decoder levels, head 3 the
 * bottleneck, head 4 (the five-level pyramid of App. A) the 2x2 average pool of the
 * bottleneck.  H, W divisible by 8 (by 16 with five heads). */
size_t aps_kernel_predict_workspace_size(const aps_net* net, int N, int H, int W);
int aps_kernel_predict(const aps_net* net, const void* feat, int N, int H, int W, int C,
                       int n_heads, void* const* logits, int logit_dtype, const int* kstride,
                       void* ws, size_t ws_bytes, void* stream);
/* The same with the compact demodulation map of head 0 (Sec. 6.2): side0 [N,H,W,4] in the
 * logit dtype receives logits[0] channels [side0_offset, side0_offset + 3) and a 0 (see
 * aps_conv2d_fwd_head_ex).  It is written by the fused level-0 head, so it needs logit_dtype
 * equal to the net's dtype; APS_ERR_UNSUPPORTED when that head cannot be fused or the
 * conditions of aps_conv2d_fwd_head_ex do not hold.  side0 NULL: as aps_kernel_predict. */
int aps_kernel_predict_ex(const aps_net* net, const void* feat, int N, int H, int W, int C,
                          int n_heads, void* const* logits, int logit_dtype, const int* kstride,
                          void* side0, int side0_offset, void* ws, size_t ws_bytes,
                          void* stream);

/* ---------------------------------------------------------------- a6-a9: reconstruction
 * Logits of level l: [N, H_l, W_l, kstride_l] (float32 or bf16; kstride_l a multiple of 4
 * for float32 and of 8 for bf16, >= the level's channel count K_l), channel blocks in order
 * [kd: KD*KD | ku: KU*KU if l < levels-1 | kt: KT*KT if l == 0 and prev != NULL], each block
 * row-major over (dy, dx) in [-r, r]: channel (dy+r)*K + (dx+r) weights (x+dx, y+dy).
 * One softmax per pixel over all blocks of its level (App. A eqs. app-softmax-mid/full),
 * evaluated in float32.  All gathers clamp coordinates to the image edge.
 *   G (eq. app-gather):   sum kd * L^l[x+dx, y+dy]
 *   U (eq. app-upsample): KU = 3: sum ku * Lhat^{l+1}[x/2+dx, y/2+dy];
 *                         KU = 2: sum ku[j*2+i] * Lhat^{l+1}[(x+i)/2, (y+j)/2]
 *   T (eq. app-recon-full): sum kt * Wprev[x+dx, y+dy], Wprev = bilinear sample of prev at
 *                         (x + mv.x, y + mv.y) with both taps edge-clamped; mv float32
 *                         [N,H,W,2] backward motion in pixels.
 * Compiled (KD, KU, KT): (5,3,3), (7,3,3), (5,2,5), (3,3,3). */

/* Coarse-to-fine: Lhat^{L-1} = G; Lhat^l = G + U; out = Lhat^0 (+ T when prev != NULL). */
size_t aps_denoise_pyramid_workspace_size(int N, int H, int W, int levels);
int aps_denoise_pyramid(const float* const* L, const void* const* logits, int logit_dtype,
                        const int* kstride, int levels, int KD, int KU, int KT,
                        const float* prev, const float* mv, int N, int H, int W, float* out,
                        void* ws, size_t ws_bytes, void* stream);

/* The same with learned demodulation (Sec. 6.2) fused into level 0: L is the demodulated
 * pyramid (aps_demodulate); with demod_offset >= 0, out_demod [N,H,W,4] float32 receives the
 * reconstruction o (the next frame's filter history) and out = o * exp(clamp(z, -8, 8)) with z
 * = logits[0][..., demod_offset .. +2] (as aps_remodulate); with lat_out (requires
 * demod_offset >= 0) the four latent channels logits[0][..., lat_offset .. +3] are copied to
 * lat_out [N,H,W,4] float32.  demod_offset < 0 gives aps_denoise_pyramid. */
int aps_denoise_pyramid_ex(const float* const* L, const void* const* logits, int logit_dtype,
                           const int* kstride, int levels, int KD, int KU, int KT,
                           const float* prev, const float* mv, int N, int H, int W,
                           int demod_offset, int lat_offset, float* out, float* out_demod,
                           float* lat_out, void* ws, size_t ws_bytes, void* stream);

/* accum_out += T with the level-0 joint softmax (ku block present iff has_upsample). */
int aps_reproject(const float* prev, const float* mv, const void* logits0, int logit_dtype,
                  int kstride, int KD, int KU, int KT, int has_upsample, int N, int H, int W,
                  float* accum_out, void* stream);

/* accum_out += U(coarse) with the level's joint softmax (kt block present iff has_temporal);
 * H, W are the fine sizes, coarse is [N, H/2, W/2]. */
int aps_upsample(const float* coarse, const void* logits, int logit_dtype, int kstride, int KD,
                 int KU, int KT, int has_temporal, int N, int H, int W, float* accum_out,
                 void* stream);

/* ---------------------------------------------------------------- learned demodulation
 * Sec. 6.2 (learned demodulation): the denoiser predicts d = exp(clamp(z, -8, 8)) per pixel
 * and channel, z being three channels of the level-0 logits tensor z [N,H,W,z_stride] (z_dtype
 * APS_F32 or APS_BF16) from channel z_offset (z_stride >= z_offset + 3).  aps_demodulate: Ld[0]
 * = L0 / d (RGB; A written 0) and Ld[l] its 2^l x 2^l block means (App. A eq. app-pyramid),
 * Ld[l] float32 RGBA [N, H>>l, W>>l], H and W divisible by 2^(levels-1); the filter then runs on
 * Ld.  aps_remodulate: out = d * in (RGB), in and out float32 RGBA [N,H,W]; out may alias in.
 * It also copies the recurrent latents (Sec. 3, the shared latent feature loop) when lat_out is
 * not NULL: lat_out float32 [N,H,W,4] = z[..., lat_offset .. lat_offset + 3] (the level-0 head's
 * four latent channels, z_stride >= lat_offset + 4), read from the logit row the map comes
 * from; the next frame's feature assembly warps them (aps_assemble_features_ex). */
int aps_demodulate(const float* L0, const void* z, int z_dtype, int z_stride, int z_offset, int N,
                   int H, int W, int levels, float* const* Ld, void* stream);
int aps_remodulate(const float* in, const void* z, int z_dtype, int z_stride, int z_offset,
                   int lat_offset, int N, int H, int W, float* out, float* lat_out, void* stream);

/* ---------------------------------------------------------------- a10: backward passes
 * All gradients are float32 unless a dtype argument says otherwise.  "Written" outputs are
 * overwritten; "accumulated" ones are added to (the caller zeroes them first). */

/* Gathering pyramid (App. A) backward.  The coarse reconstructed levels are recomputed from
 * L and the logits (not stored), then levels run fine to coarse:
 *   grad_logits[l] [N,H_l,W_l,gstride[l]] (grad_dtype F32|BF16; written, padding zeroed):
 *     w_k (<g, v_k> - <g, y>) for the joint softmax (eqs. app-softmax-mid/full);
 *   grad_L[l] [N,H_l,W_l,4] (written): the transpose of the kd gather (eq. app-gather),
 *     a gather over each input pixel's edge-clamped preimages (deterministic);
 *   grad_prev [N,H,W,4] (accumulated, nullable): the transpose of the kt gather and of the
 *     bilinear warp (eq. app-recon-full), by float atomics (order not fixed).
 * Arguments otherwise as aps_denoise_pyramid. */
size_t aps_denoise_pyramid_bwd_workspace_size(int N, int H, int W, int levels, int KD, int KU,
                                              int KT, int temporal);
int aps_denoise_pyramid_bwd(const float* const* L, const void* const* logits, int logit_dtype,
                            const int* kstride, int levels, int KD, int KU, int KT,
                            const float* prev, const float* mv, int N, int H, int W,
                            const float* grad_out, void* const* grad_logits, int grad_dtype,
                            const int* gstride, float* const* grad_L, float* grad_prev, void* ws,
                            size_t ws_bytes, void* stream);

/* Backward of aps_reproject (App. A eq. app-recon-full: the kt gather of the bilinearly warped
 * previous output, weighted by the level-0 joint softmax).  grad_accum [N,H,W,4] float32 is
 * dLoss/d(accum_out) after the call; the gradient w.r.t. the accum_out input is grad_accum
 * itself (the term is added), so nothing is written for it.
 *   grad_logits0 [N,H,W,gstride] (grad_dtype F32|BF16; written, channels >= K zeroed):
 *     w_k (<g, v_k> [k in the kt block] - <g, T>) over all K = KD^2 (+ KU^2) + KT^2 channels,
 *     the softmax being shared with the level's other terms (eq. app-softmax-full);
 *   grad_prev [N,H,W,4] float32 (accumulated, nullable): the transpose of the kt gather (a
 *     gather over each pixel's edge-clamped preimages) and of the bilinear warp (float atomics,
 *     order not fixed).
 * Motion vectors are not differentiated.  Workspace: the normalised weights, N*H*W*K floats.
 * Other arguments and errors as aps_reproject; APS_ERR_UNSUPPORTED for another grad_dtype. */
size_t aps_reproject_bwd_workspace_size(int N, int H, int W, int KD, int KU, int KT,
                                        int has_upsample);
int aps_reproject_bwd(const float* prev, const float* mv, const void* logits0, int logit_dtype,
                      int kstride, int KD, int KU, int KT, int has_upsample, int N, int H, int W,
                      const float* grad_accum, void* grad_logits0, int grad_dtype, int gstride,
                      float* grad_prev, void* ws, size_t ws_bytes, void* stream);

/* Backward of aps_upsample (App. A eq. app-upsample: the ku gather of the coarser
 * reconstructed level around each pixel's parent, with the level's joint softmax).
 *   grad_logits [N,H,W,gstride] (written, channels >= K zeroed): w_k (<g, v_k> [k in the ku
 *     block] - <g, U>) over all K = KD^2 + KU^2 (+ KT^2) channels;
 *   grad_coarse [N,H/2,W/2,4] float32 (written): for each coarse pixel the sum over the fine
 *     pixels and ku taps that read it (gather form, deterministic).
 * The accum_out input passes grad_accum through unchanged (nothing written).  Workspace:
 * N*H*W*K floats.  Other arguments and errors as aps_upsample. */
size_t aps_upsample_bwd_workspace_size(int N, int H, int W, int KD, int KU, int KT,
                                       int has_temporal);
int aps_upsample_bwd(const float* coarse, const void* logits, int logit_dtype, int kstride, int KD,
                     int KU, int KT, int has_temporal, int N, int H, int W,
                     const float* grad_accum, void* grad_logits, int grad_dtype, int gstride,
                     float* grad_coarse, void* ws, size_t ws_bytes, void* stream);

/* Backward of aps_density_predict (Sec. 3, Overview: the sampler network and the budget
 * normalisation; Sec. 4.3: the density is trained through the relaxed sampling step, whose
 * gradient dLoss/ds aps_scatter_samples_bwd gives).  The three layers are recomputed layer by
 * layer from feat (nothing is kept from the forward), then:
 *   dLoss/dz = aps_normalize_density_bwd of grad_s [N,H,W] float32;
 *   grad_w[i] [Cout][k][k][Cin] float32 and grad_b[i] [Cout] float32 (written, i = 0, 1, 2):
 *     weight and bias gradients (MFMA, fixed-order split reduction: deterministic), the
 *     hidden layers' gradients masked by their ReLU outputs;
 *   grad_feat [N,H,W,C] in the net dtype (written, nullable): the input gradient.
 * packed_dgrad[i]: layer i's data-gradient operator (aps_conv_pack_weights_dgrad of its
 * float32 weights, in the net dtype); packed_dgrad[0] may be NULL when grad_feat is NULL.  In
 * bf16 dLoss/dz and the hidden gradients are rounded to bf16 between layers.  The layers must
 * have the shapes aps_density_predict takes (C -> c0 ReLU -> c1 ReLU -> 1 linear), else
 * APS_ERR_SHAPE. */
size_t aps_density_predict_bwd_workspace_size(const aps_net* net, int N, int H, int W);
int aps_density_predict_bwd(const aps_net* net, const void* const* packed_dgrad, const void* feat,
                            int N, int H, int W, int C, float budget_spp, float uniform_frac,
                            const float* grad_s, float* const* grad_w, float* const* grad_b,
                            void* grad_feat, void* ws, size_t ws_bytes, void* stream);

/* Scatter backward (Sec. 4.2 eq. stoch_rnoisy, Sec. 4.3 eq. relaxed_holdout): grad_s (written,
 * or accumulated when accumulate != 0) = <dLoss/dL0, dL0/ds> with
 *   dL0/ds = -L0/s + (S_holdout/s) dw/dp,  dw/dp = h lambda u / p^2 inside the relaxed ramp,
 *   0 on its clamped parts and in hard mode;
 * dLoss/dL0 collects grad_L[l] / 4^l of every pyramid ancestor (eq. app-pyramid).
 * Arguments as aps_scatter_samples; grad_L[l] float32 RGBA [N, H>>l, W>>l]. */
int aps_scatter_samples_bwd(const float* s, const uint8_t* count, const int32_t* pixel_offset,
                            const float* samples, int64_t n_samples, int N, int H, int W,
                            int levels, int mode, float lambda, uint64_t seed, uint32_t frame,
                            const float* const* grad_L, float* grad_s, int accumulate,
                            void* stream);
/* aps_scatter_samples_bwd for the modes of aps_scatter_samples_ex: dL0/ds = -L0/s + (r/s) dw/dp
 * with dw/dp = 1 (straight-through), w (1 - w) / (tau p (1 - p)) (Gumbel-Softmax), the ramp's
 * slope (relaxed), 0 (hard); APS_DASR the surrogate of Sec. 4.1 eq. kuz_grad,
 * dL0/ds = (L_ref - L0) / round(s) for s >= 1/2 and L_ref below, L_ref float32 RGBA [N,H,W]
 * (the reference radiance; required for APS_DASR, ignored otherwise). */
int aps_scatter_samples_bwd_ex(const float* s, const uint8_t* count, const int32_t* pixel_offset,
                               const float* samples, int64_t n_samples, int N, int H, int W,
                               int levels, int mode, float param, uint64_t seed, uint32_t frame,
                               const float* u_tex, int tex_size, const float* L_ref,
                               const float* const* grad_L, float* grad_s, int accumulate,
                               void* stream);

/* Backward of aps_demodulate / aps_remodulate.  grad_Ld[l] float32 RGBA per level (the
 * filter's gradient w.r.t. its input pyramid); grad_L0 float32 RGBA [N,H,W]; grad_z float32
 * [N,H,W,3] (dLoss/dz of the three demodulation channels, 0 where the clamp is active); with
 * accumulate != 0 both outputs are added to, else written.  aps_remodulate_bwd: grad_out of
 * out = d * in gives grad_in = grad_out * d and grad_z = grad_out * out. */
int aps_demodulate_bwd(const float* L0, const void* z, int z_dtype, int z_stride, int z_offset,
                       int N, int H, int W, int levels, const float* const* grad_Ld,
                       float* grad_L0, float* grad_z, int accumulate, void* stream);
int aps_remodulate_bwd(const float* in, const void* z, int z_dtype, int z_stride, int z_offset,
                       int N, int H, int W, const float* grad_out, float* grad_in, float* grad_z,
                       int accumulate, void* stream);

/* Budget normalisation backward (Sec. 3): grad_z (written) = c1 sm (g - sum(sm g)) per frame,
 * c1 = (1-f) B Npx; fixed-tree reductions (deterministic). */
size_t aps_normalize_bwd_workspace_size(int N, int H, int W);
int aps_normalize_density_bwd(const float* z, int N, int H, int W, float budget_spp,
                              float uniform_frac, const float* grad_s, float* grad_z, void* ws,
                              size_t ws_bytes, void* stream);

/* Feature assembly backward: accumulates into grad_L0 (RGB of float32 RGBA [N,H,W,4]),
 * grad_s [N,H,W], and, through the warp, grad_prev [N,H,W,4] (float atomics); each output is
 * skipped when NULL.  grad_feat [N,H,W,C] in feat_dtype. */
int aps_assemble_features_bwd(int kind, const float* L0, const float* prev, const float* mv,
                              int N, int H, int W, int C, int feat_dtype, const void* grad_feat,
                              float* grad_L0, float* grad_s, float* grad_prev, void* stream);
/* Backward of aps_assemble_features_ex: has_lat says whether the features carried latents;
 * grad_lat float32 [N,H,W,4] (nullable) receives their gradient through the warp (float
 * atomics, added to). */
int aps_assemble_features_bwd_ex(int kind, const float* L0, const float* prev, const float* mv,
                                 int has_lat, int N, int H, int W, int C, int feat_dtype,
                                 const void* grad_feat, float* grad_L0, float* grad_s,
                                 float* grad_prev, float* grad_lat, void* stream);

/* Data-gradient operator of a conv layer: the same MFMA kernel with w'[ci][tap][co] =
 * w[co][k*k-1-tap][ci].  packed holds aps_conv_packed_elems(Cin, ksize, Cout) elements. */
int aps_conv_pack_weights_dgrad(const float* w, int Cout, int ksize, int Cin, int dtype,
                                void* packed, void* stream);

/* dX [N,H,W,Cin] (written, dtype) = gradient w.r.t. the conv's transformed input, from
 * dy [N,H,W,ldy] (channels >= Cout ignored) masked by ymask > 0 when ymask (the layer's
 * post-ReLU output [N,H,W,Cout], then ldy == Cout) is given.  ldy*sizeof(dtype) % 16 == 0. */
int aps_conv2d_bwd_data(const void* dy, const void* ymask, int ldy, int N, int H, int W, int Cout,
                        const void* packed_wT, int ksize, int Cin, int dtype, void* dX,
                        void* stream);

/* Transpose of the fused input transform (H, W = the conv's output size):
 *   APS_CONV_DIRECT : dx [N,H,W,Cx] (+)= dX
 *   APS_CONV_POOL2  : dx [N,2H,2W,Cx] (+)= dX / 4 on each 2x2 child
 *   APS_CONV_UP2_CAT: dx [N,H/2,W/2,Cx] (+)= sum of dX[..., :Cx] over the 2x2 children;
 *                     dx2 [N,H,W,C2] (+)= dX[..., Cx:]
 * "(+)=" adds when the matching accumulate flag is set, else writes. */
int aps_conv_input_grad(int mode, const void* dX, int N, int H, int W, int Cx, int C2, int dtype,
                        void* dx, int accumulate, void* dx2, int accumulate2, void* stream);

/* Weight and bias gradients of a conv layer (MFMA, split over pixel blocks, fixed-order
 * reduction: deterministic): dw [Cout][k][k][Cin] float32 (written) = sum over pixels of
 * dy (masked as above) times the transformed input; db [Cout] float32 (written, nullable).
 * Input arguments as aps_conv2d_fwd; Cout <= 256. */
size_t aps_conv2d_bwd_weight_workspace_size(int N, int H, int W, int Cx, int C2, int Cout,
                                            int ksize);
int aps_conv2d_bwd_weight(const void* x, const void* x2, int mode, int N, int H, int W, int Cx,
                          int C2, const void* dy, const void* ymask, int ldy, int Cout, int ksize,
                          int dtype, float* dw, float* db, void* ws, size_t ws_bytes,
                          void* stream);

/* ---------------------------------------------------------------- a11: training
 * Loss of Sec. 6.3 (eqs. loss_spatial, loss_temporal, loss_combined, visual mask m = 1) on the
 * tonemapped images of Sec. 5: I = sRGB(tau(alpha (sat_beta(log(max(L,0) + 1e-4)) + k); s, h)),
 * params [N][5] = (k, alpha, beta, s, h) per frame (device).  loss (device scalar, written) =
 * mean over pixels and RGB of max(1.25 |dI - dI_ref|, |I - I_ref|), with dI = I - W(I_prev) and
 * the temporal term 0 where the back-projection leaves the frame (or without prev_out).
 * grad_out [N,H,W,4] written; grad_prev [N,H,W,4] accumulated through the warp (nullable). */
size_t aps_tmo_loss_workspace_size(int N, int H, int W);
int aps_tmo_loss(const float* out, const float* ref, const float* prev_out, const float* prev_ref,
                 const float* mv, const float* params, int N, int H, int W, float* loss,
                 float* grad_out, float* grad_prev, void* ws, size_t ws_bytes, void* stream);

/* AdamW with decoupled weight decay on float32 master parameters (Sec. 6.3 uses
 * beta = (0.8, 0.985), weight decay 0.02); step >= 1 is the 1-based step count for the bias
 * corrections; the gradient is multiplied by grad_scale first. */
int aps_adamw_step(float* param, float* m, float* v, const float* grad, int64_t n, float lr,
                   float beta1, float beta2, float eps, float weight_decay, int step,
                   float grad_scale, void* stream);

/* Layout / dtype copy: dst[p][c] = src[p][c] for c < C, 0 for C <= c < dst_ld, p < npix
 * (F32 or BF16 on either side; bf16 by round to nearest even). */
int aps_copy_channels(const void* src, int src_dtype, int src_ld, void* dst, int dst_dtype,
                      int dst_ld, int64_t npix, int C, void* stream);

/* x[i] *= *scale (scale a device scalar), i < n. */
int aps_scale_by(float* x, int64_t n, const float* scale, void* stream);

/* out (device scalar) = sum of x^2, fixed-order reduction (gradient-norm guard). */
size_t aps_sumsq_workspace_size(int64_t n);
int aps_sumsq(const float* x, int64_t n, float* out, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* APS_H */
