// The density (sampler) CNN (Sec. 3, overview; Sec. 6.3) as one kernel: three 3x3 'same'
// convolutions, Cin -> 16 (ReLU), 16 -> 16 (ReLU), 16 -> 1, with the two intermediates kept on
// chip, rounded to the storage type and zero outside the image as the layer-by-layer path
// stores them.  Weights come in the packed (tap, 8-channel group) pair order of the convolution
// kernels.  bf16 runs the row-sweep form (k_sampler_sweep), fp32 the tiled form (k_sampler_cnn).
#include <algorithm>
#include <type_traits>

#include "aps_common.h"
#include "mfma_frag.h"

using namespace aps;

namespace {

struct SamplerArgs {
  const void* x;
  int N, H, W, C, ntx;
  const void* w[3];  // packed weights of the three layers
  const float* b[3];
  float* z;
};

// LDS layouts of a pixel's channels, in 16-byte chunks (8 bf16 or 4 floats).  The layouts were
// chosen with the LDS bank-conflict counter on gfx950 (probe kernels of each access shape).
// bf16, 16 channels: 32-byte pixels whose two chunks swap on every other run of 4 pixels (an XOR
// swizzle on pixel bit 2): the B-operand reads (16 pixels x 2 chunks x 2 shifts per
// instruction) are conflict-free and the 8-byte C-fragment writes take the cycles of a plain
// 8-byte store, where swapping on bit 3, or a 48-byte pitch, costs the reads a quarter more
// cycles and no swizzle doubles the writes.  fp32, 16 channels: 64-byte pixels whose chunk c
// sits at c ^ ((p >> 1) & 3): the 16-byte C-fragment writes (lane group q writes chunk q of 16
// consecutive pixels) take 8 cycles, as with an 80-byte pitch, against 16-32 unswizzled, and
// the group reads are unchanged (so a block needs 20 % less LDS: three blocks per CU).  8
// channels: the chunks in order at a 16-byte (bf16) or 32-byte (fp32) pixel stride.
template <typename T, int NG>
struct SLay {
  static constexpr int kPs = 8 * NG;  // elements per pixel
  static constexpr int kCh = 16 / sizeof(T);  // elements per chunk
  static __device__ inline int chunk(int p, int c) {  // element offset of chunk c of pixel p
    if constexpr (NG == 2 && sizeof(T) == 2) return p * 16 + ((c ^ ((p >> 2) & 1)) << 3);
    else if constexpr (NG == 2) return p * 16 + ((c ^ ((p >> 1) & 3)) << 2);
    else return p * kPs + c * kCh;
  }
  // element offset of 8-channel group g (bf16: one chunk; fp32: its first chunk, see group_load)
  static __device__ inline int at(int p, int g) { return chunk(p, g * (8 / kCh)); }
  // the 4-channel slice c4 (channels 4 c4 .. 4 c4 + 3)
  static __device__ inline int quad(int p, int c4) {
    if constexpr (sizeof(T) == 2) return chunk(p, c4 >> 1) + 4 * (c4 & 1);
    else return chunk(p, c4);
  }
};
// 8 channels of group g of pixel p as an MFMA fragment (fp32: two chunks, wherever they sit)
template <int NG>
__device__ inline void group_load(Frag<uint16_t>& f, const uint16_t* X, int p, int g) {
  frag_load(f, X + SLay<uint16_t, NG>::at(p, g));
}
template <int NG>
__device__ inline void group_load(Frag<float>& f, const float* X, int p, int g) {
  const float4 a = *reinterpret_cast<const float4*>(X + SLay<float, NG>::chunk(p, 2 * g));
  const float4 b = *reinterpret_cast<const float4*>(X + SLay<float, NG>::chunk(p, 2 * g + 1));
  f.v[0] = a.x; f.v[1] = a.y; f.v[2] = a.z; f.v[3] = a.w;
  f.v[4] = b.x; f.v[5] = b.y; f.v[6] = b.z; f.v[7] = b.w;
}
// One hidden layer (16 outputs, ReLU) on MFMA: output grid WOUT x WOUT at image (oy, ox), input
// grid WIN x WIN in LDS (layout SLay<T, CG>), output to Y (layout SLay<T, 2>).
template <typename T, int CG, int WIN, int WOUT>
__device__ inline void sampler_hidden(const T* Xin, T* Y, const T* wp, const float* bias, int H, int W,
                                      int oy, int ox, int lane, int wave) {
  using LI = SLay<T, CG>;
  using LO = SLay<T, 2>;
  constexpr int NPAIR = 9 * CG, STEPS = (NPAIR + 3) / 4, NPX = WOUT * WOUT;
  Frag<T> wf[STEPS];
  int toff[STEPS], grp[STEPS];  // this lane's (tap, group) pair at each K step: pixel offset, group
#pragma unroll
  for (int s = 0; s < STEPS; ++s) {
    frag_load(wf[s], wp + ((size_t)s * 64 + lane) * 8);
    const int p = 4 * s + (lane >> 4);
    const int tap = p < NPAIR ? p / CG : 0, g = p < NPAIR ? p % CG : 0;  // padded pairs: zero weights
    toff[s] = (tap / 3) * WIN + tap % 3;
    grp[s] = g;
  }
  const f32x4 b = *reinterpret_cast<const f32x4*>(bias + 4 * (lane >> 4));  // added after the sum
  const int co = 4 * (lane >> 4);  // this lane's four output channels
  for (int tile = wave; tile * 16 < NPX; tile += 4) {
    const int pix = tile * 16 + (lane & 15);
    const bool valid = pix < NPX;
    const int pp = valid ? pix : 0, r = pp / WOUT, c = pp - r * WOUT;
    const int p0 = r * WIN + c;
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      Frag<T> bf;
      group_load<CG>(bf, Xin, p0 + toff[s], grp[s]);
      acc = mma(wf[s], bf, acc);
    }
    if (valid) {
      const int iy = oy + r, ix = ox + c;
      const bool inside = iy >= 0 && iy < H && ix >= 0 && ix < W;
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = inside ? fmaxf(acc[q] + b[q], 0.f) : 0.f;
      T* d = Y + LO::quad(pix, co >> 2);
      if constexpr (sizeof(T) == 2) *reinterpret_cast<u16x4*>(d) = f2bf4(v[0], v[1], v[2], v[3]);
      else *reinterpret_cast<float4*>(d) = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

// Tiled form (fp32).  A block stages its 22x22 input tile (16x16 outputs + 3-pixel halo) once;
// the two intermediates (20x20 and 18x18 pixels x 16 channels) stay in LDS.  The hidden layers
// run on v_mfma_f32_16x16x4f32 with K = (tap, 8-channel group) pairs and n-tiles of 16
// consecutive pixels of a layer's output grid (B fragments gathered per lane); the 16 -> 1 layer
// runs on the vector ALU, one output pixel per thread, since an fp32 MFMA tile would spend 15 of
// its 16 rows on padding.
template <int CG0>
__global__ __launch_bounds__(256) void k_sampler_cnn(SamplerArgs a) {
  using T = float;
  using L0 = SLay<T, CG0>;
  using L1 = SLay<T, 2>;
  constexpr int X0N = 22 * 22 * L0::kPs, H2N = 18 * 18 * L1::kPs;
  __shared__ __attribute__((aligned(16))) T X0[X0N > H2N ? X0N : H2N];  // the 18x18 map reuses it
  __shared__ __attribute__((aligned(16))) T H1[20 * 20 * L1::kPs];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tx0 = (blockIdx.x % a.ntx) * 16, ty0 = (blockIdx.x / a.ntx) * 16, n = blockIdx.z;
  const T* x = static_cast<const T*>(a.x);
  for (int it = tid; it < 22 * 22 * CG0; it += 256) {
    const int g = it % CG0, p = it / CG0, r = p / 22, c = p - r * 22;
    const int iy = ty0 - 3 + r, ix = tx0 - 3 + c;
    float* d0 = X0 + L0::chunk(p, 2 * g);
    float* d1 = X0 + L0::chunk(p, 2 * g + 1);
    float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
    if (iy >= 0 && iy < a.H && ix >= 0 && ix < a.W) {
      const float4* src = reinterpret_cast<const float4*>(x + (((size_t)n * a.H + iy) * a.W + ix) * a.C + g * 8);
      v0 = src[0];
      v1 = src[1];
    }
    *reinterpret_cast<float4*>(d0) = v0;
    *reinterpret_cast<float4*>(d1) = v1;
  }
  __syncthreads();
  sampler_hidden<T, CG0, 22, 20>(X0, H1, static_cast<const T*>(a.w[0]), a.b[0], a.H, a.W, ty0 - 2,
                                 tx0 - 2, lane, wave);
  __syncthreads();
  sampler_hidden<T, 2, 20, 18>(H1, X0, static_cast<const T*>(a.w[1]), a.b[1], a.H, a.W, ty0 - 1,
                               tx0 - 1, lane, wave);
  __syncthreads();
  // 16 -> 1: weights read from the packed buffer (output channel 0: lane 16 (p % 4) of step
  // p / 4 for pair p = 2 tap + ci / 8)
  const int r = tid >> 4, c = tid & 15;
  const float* wp2 = static_cast<const float*>(a.w[2]);
  float acc = 0.f;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int pp = (r + tap / 3) * 18 + c + tap % 3;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int pr = 2 * tap + g;
      const float* wv = wp2 + ((pr / 4) * 64 + 16 * (pr % 4)) * 8;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float* px = X0 + L1::chunk(pp, 2 * g + h);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = fmaf(wv[4 * h + e], px[e], acc);
      }
    }
  }
  const int iy = ty0 + r, ix = tx0 + c;
  if (iy < a.H && ix < a.W) a.z[((size_t)n * a.H + iy) * a.W + ix] = acc + a.b[2][0];
}

// Row-sweep form of the bf16 sampler CNN.  Each wave runs on its own, with no block barrier:
// it owns a band of 26 output columns and R output rows, and walks down the band one image row
// at a time through all three layers.  Per layer and row it computes 32 positions (two 16-pixel
// MFMA n-tiles; the last positions of the band are halo garbage that no kept output reads).  An
// input row is read from LDS once per layer, as the B operands of the three kernel rows dy, and
// each dy adds into the accumulator of a different output row, so three rolling accumulators
// per n-tile hold the output rows in progress; the one that receives its dy = 2 term is complete
// and is written, biased, rectified and rounded, as the next layer's input row.  K per dy is the
// (dx, 8-channel group) pairs in order, so the B operand of a row is read 2 (16 input channels)
// or 1 (8) times per n-tile instead of 5 (3) times as in the tiled kernel.  The 16 -> 1 layer
// puts its three kernel rows in MFMA rows 0..2, which land in one lane's first three
// accumulators.  Layers run one row apart (layer 2 reads the row layer 1 wrote one step
// earlier), so a step's LDS reads of the three layers are independent.  LDS operations of one
// wave complete in program order, so a row written at the end of a step is read safely at the
// next, and a single buffer per layer suffices.
// dword 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format, no swizzle)
constexpr int kBufferWord3 = 0x00020000;
constexpr int kSweepCols = 26;  // output columns per band (32 positions minus 6 halo)
constexpr int kSweepRB = 36;    // row buffer: 32 positions + the 2 read past the last + pad (zero)

template <int CG>
__device__ inline void sweep_weights(const uint16_t* wp, int lane, Frag<uint16_t> (&w)[3][2]) {
  const int m = lane & 15, t = lane >> 4;
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = 4 * h + t;  // (dx, group) pair of this lane's K slot within kernel row dy
      if (p < 3 * CG) {
        const int P = 3 * CG * dy + p;  // pair index of the (tap, group) packing
        frag_load(w[dy][h], wp + ((size_t)(P / 4) * 64 + 16 * (P % 4) + m) * 8);
      } else {
        w[dy][h].v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      }
    }
}

// LDS offset (elements) of this lane's B operand for n-tile s and K half h of a kernel row; a K
// slot past the pairs points at the zero pad (position 32) for both n-tiles.
template <int CG>
__device__ inline int sweep_boff(int lane, int s, int h) {
  using L = SLay<uint16_t, CG>;
  const int p = 4 * h + (lane >> 4);
  return p < 3 * CG ? L::at(16 * s + (lane & 15) + p / CG, p % CG) : L::at(32, 0);
}

template <int CG0>
__global__ __launch_bounds__(256) void k_sampler_sweep(SamplerArgs a, int R, int nseg, int nunit) {
  using T = uint16_t;
  using L0 = SLay<T, CG0>;
  using L1 = SLay<T, 2>;
  constexpr int NH0 = CG0 == 2 ? 2 : 1;  // K halves of a kernel row of layer 1
  constexpr int XN = kSweepRB * L0::kPs, HN = kSweepRB * L1::kPs;
  constexpr int D = 6;                   // input rows in flight (registers)
  __shared__ __attribute__((aligned(16))) T lds[4][XN + 2 * HN];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int unit = blockIdx.x * 4 + wave, n = blockIdx.y;
  if (unit >= nunit) return;  // the whole wave; nothing below synchronises waves
  const int x0 = (unit / nseg) * kSweepCols, y0 = (unit % nseg) * R;
  T* X = lds[wave];
  T* H1 = X + XN;
  T* H2 = H1 + HN;
  for (int e = lane * 8; e < XN + 2 * HN; e += 512) zero8(X + e);

  Frag<T> w1[3][2], w2[3][2], w3[2];
  sweep_weights<CG0>(static_cast<const T*>(a.w[0]), lane, w1);
  sweep_weights<2>(static_cast<const T*>(a.w[1]), lane, w2);
  {
    // 16 -> 1: MFMA row m < 3 holds kernel row dy = m of output channel 0
    const T* wp = static_cast<const T*>(a.w[2]);
    const int m = lane & 15, t = lane >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int p = 4 * h + t;
      if (m < 3 && p < 6) {
        const int P = 6 * m + p;
        frag_load(w3[h], wp + ((size_t)(P / 4) * 64 + 16 * (P % 4)) * 8);
      } else {
        w3[h].v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      }
    }
  }
  // biases enter as the starting value of an output row's first MFMA (layer 3: MFMA row 0)
  const int co = 4 * (lane >> 4);
  const f32x4 b1 = *reinterpret_cast<const f32x4*>(a.b[0] + co);
  const f32x4 b2 = *reinterpret_cast<const f32x4*>(a.b[1] + co);
  const f32x4 b3 = f32x4{a.b[2][0], 0.f, 0.f, 0.f};
  int bo1[2][2], bo2[2][2];
  // ReLU and the zero padding outside the image in one med3(v, 0, lim): lim = +inf keeps
  // max(v, 0), lim = 0 gives 0 (columns outside here, rows outside per step)
  float lim1[2], lim2[2];
  bool zok[2];  // this lane stores a layer-3 output of n-tile s
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bo1[s][h] = sweep_boff<CG0>(lane, s, h);
      bo2[s][h] = sweep_boff<2>(lane, s, h);
    }
    const int pos = (lane & 15) + 16 * s;
    lim1[s] = x0 - 2 + pos >= 0 && x0 - 2 + pos < a.W ? __builtin_inff() : 0.f;
    lim2[s] = x0 - 1 + pos >= 0 && x0 - 1 + pos < a.W ? __builtin_inff() : 0.f;
    zok[s] = lane < 16 && pos < kSweepCols && x0 + pos < a.W;
  }
  // this lane's input chunk: pixel position jc, channel group gc (lanes past the row idle)
  const int jc = lane / CG0, gc = lane % CG0;
  const bool ldr = lane < 32 * CG0;
  const int xc = x0 - 3 + jc;
  // Input rows come through a buffer resource over this image: a lane outside the image (or
  // past the row's chunks) passes an offset past its end, which the hardware's range check
  // answers with zeros.  No load sits under a branch, so the compiler can count the rows in
  // flight instead of waiting for all of them before each row's LDS write.
  const uint32_t img_bytes = (uint32_t)((size_t)a.H * a.W * a.C * sizeof(T));
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<T*>(static_cast<const T*>(a.x) + (size_t)n * a.H * a.W * a.C), 0, img_bytes,
      kBufferWord3);
  const bool col_in = ldr && xc >= 0 && xc < a.W;
  auto load_row = [&](int iy) {
    const bool in = col_in && iy >= 0 && iy < a.H;
    const uint32_t off = in ? (uint32_t)((((size_t)iy * a.W + xc) * a.C + gc * 8) * sizeof(T)) : img_bytes;
    return __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
  };
  auto store_row = [&](u16x8 v) {
    if (ldr) *reinterpret_cast<u16x8*>(X + L0::at(jc, gc)) = v;
  };
  // emission of a hidden layer's completed image row oy: position (lane & 15) + 16 s
  auto emit = [&](const f32x4 (&acc)[2], const float (&lim)[2], int oy, T* Y) {
    const bool rin = oy >= 0 && oy < a.H;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const float l = rin ? lim[s] : 0.f;
      const int pos = (lane & 15) + 16 * s;
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = __builtin_amdgcn_fmed3f(acc[s][q], 0.f, l);
      *reinterpret_cast<u16x4*>(Y + L1::at(pos, co >> 3) + (co & 7)) = f2bf4(v[0], v[1], v[2], v[3]);
    }
  };

  const int I0 = y0 - 3;  // first input row
  store_row(load_row(I0));
  u16x8 gx[D];
#pragma unroll
  for (int k = 1; k <= D; ++k) gx[k % D] = load_row(I0 + k);
  f32x4 acc1[3][2], acc2[3][2];
  float s3[3][2];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      acc1[k][s] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc2[k][s] = f32x4{0.f, 0.f, 0.f, 0.f};
      s3[k][s] = 0.f;
    }
  float* zimg = a.z + (size_t)n * a.H * a.W + x0;
  const int ylast = min(y0 + R, a.H) - 1;  // last output row of this band segment

  // one step: input row I0 + i through layer 1, the row layer 1 wrote at step i - 1 through
  // layer 2, the row layer 2 wrote at step i - 1 through layer 3.  i mod 3 picks the rolling
  // accumulators: F starts an output row (dy = 0), M continues one (dy = 1), C completes one;
  // i mod D picks the register set of the input row written to LDS at the end of the step.
  auto step = [&](auto ph, int i) {
    constexpr int PH = decltype(ph)::value;
    constexpr int F = (PH + 1) % 3, M = PH % 3, C = (PH + 2) % 3, G = (PH + 1) % D;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    Frag<T> bx[2][2], bh[2][2], bq[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h < NH0) frag_load(bx[s][h], X + bo1[s][h]);
        frag_load(bh[s][h], H1 + bo2[s][h]);
        frag_load(bq[s][h], H2 + bo2[s][h]);
      }
    float c3[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      f32x4 f1 = mma(w1[0][0], bx[s][0], b1);
      f32x4 f2 = mma(w2[0][0], bh[s][0], b2);
      f32x4 q = mma(w3[0], bq[s][0], b3);
      acc1[M][s] = mma(w1[1][0], bx[s][0], acc1[M][s]);
      acc2[M][s] = mma(w2[1][0], bh[s][0], acc2[M][s]);
      acc1[C][s] = mma(w1[2][0], bx[s][0], acc1[C][s]);
      acc2[C][s] = mma(w2[2][0], bh[s][0], acc2[C][s]);
      if constexpr (NH0 == 2) {
        f1 = mma(w1[0][1], bx[s][1], f1);
        acc1[M][s] = mma(w1[1][1], bx[s][1], acc1[M][s]);
        acc1[C][s] = mma(w1[2][1], bx[s][1], acc1[C][s]);
      }
      f2 = mma(w2[0][1], bh[s][1], f2);
      acc2[M][s] = mma(w2[1][1], bh[s][1], acc2[M][s]);
      acc2[C][s] = mma(w2[2][1], bh[s][1], acc2[C][s]);
      q = mma(w3[1], bq[s][1], q);
      acc1[F][s] = f1;
      acc2[F][s] = f2;
      c3[s][0] = q[0];
      c3[s][1] = q[1];
      c3[s][2] = q[2];
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    // layer 1 completes row I0 + i - 1 (image columns from x0 - 2), layer 2 row I0 + i - 3
    // (from x0 - 1), layer 3 row I0 + i - 5 (from x0)
    emit(acc1[C], lim1, I0 + i - 1, H1);
    emit(acc2[C], lim2, I0 + i - 3, H2);
    const int oy = I0 + i - 5;
    const bool zrow = oy >= y0 && oy <= ylast;
    float* zr = zimg + (size_t)oy * a.W;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      s3[F][s] = c3[s][0];
      s3[M][s] += c3[s][1];
      const float zv = s3[C][s] + c3[s][2];
      if (zrow && zok[s]) zr[(lane & 15) + 16 * s] = zv;
    }
    store_row(gx[G]);
    gx[G] = load_row(I0 + i + 1 + D);
  };
  const int nstep = R + 8;
  for (int i = 0; i < nstep; i += 6) {
    step(std::integral_constant<int, 0>{}, i);
    step(std::integral_constant<int, 1>{}, i + 1);
    step(std::integral_constant<int, 2>{}, i + 2);
    step(std::integral_constant<int, 3>{}, i + 3);
    step(std::integral_constant<int, 4>{}, i + 4);
    step(std::integral_constant<int, 5>{}, i + 5);
  }
}

}  // namespace

namespace aps {
int sampler_cnn(const void* x, int N, int H, int W, int C, int Cin, const void* w0, const float* b0,
                const void* w1, const float* b1, const void* w2, const float* b2, int dtype, float* z,
                hipStream_t st) {
  if (Cin > 16 || C % 8 || C < Cin) return APS_ERR_UNSUPPORTED;
  SamplerArgs a{};
  a.x = x;
  a.N = N;
  a.H = H;
  a.W = W;
  a.C = C;
  a.ntx = (W + 15) / 16;
  a.w[0] = w0;
  a.w[1] = w1;
  a.w[2] = w2;
  a.b[0] = b0;
  a.b[1] = b1;
  a.b[2] = b2;
  a.z = z;
  dim3 grid(a.ntx * ((H + 15) / 16), 1, N);
  const bool cg1 = Cin <= 8;
  if (dtype == APS_BF16) {
    // row sweep: band segments of R rows, R chosen so that about kSweepWaves waves cover the
    // images (all resident at once at two waves per SIMD)
    constexpr long kSweepWaves = 2048;
    const long nband = (W + kSweepCols - 1) / kSweepCols;
    const int R = (int)std::max<long>(8, ((long)N * H * nband + kSweepWaves - 1) / kSweepWaves);
    const int nseg = (H + R - 1) / R;
    const long nunit = nband * nseg;
    // the buffer resource addresses one image with 32-bit byte offsets
    if (nunit > (1L << 30) / 4 || N > 65535 || (size_t)H * W * C * 2 >= (1ull << 31))
      return APS_ERR_SHAPE;
    dim3 g((unsigned)((nunit + 3) / 4), N);
    if (cg1) k_sampler_sweep<1><<<g, 256, 0, st>>>(a, R, nseg, (int)nunit);
    else k_sampler_sweep<2><<<g, 256, 0, st>>>(a, R, nseg, (int)nunit);
  } else if (dtype == APS_F32) {
    if (cg1) k_sampler_cnn<1><<<grid, 256, 0, st>>>(a);
    else k_sampler_cnn<2><<<grid, 256, 0, st>>>(a);
  } else {
    return APS_ERR_UNSUPPORTED;
  }
  APS_LAUNCH_CHECK();
  return APS_OK;
}
}  // namespace aps
