// NHWC convolution (k = 1 or 3, zero padding) as an implicit GEMM on gfx950 MFMA:
//   M = output channels (16 per MFMA tile), N = pixels (a 16-pixel row segment per tile),
//   K = taps x input channels, walked in chunks of 32 channels.
// The input tile of a chunk, with its 1-pixel halo, is staged once in LDS and read by all
// taps; weights are pre-packed in MFMA fragment order and read straight into registers.
// bf16: v_mfma_f32_16x16x32_bf16 (fp32 accumulate).  f32: v_mfma_f32_16x16x4f32.
// Input transforms fused into the staging: 2x2 average pool of a finer tensor, or nearest
// 2x upsampling of a coarser tensor concatenated with a skip tensor (U-Net decoder).
// Epilogue: bias, optional ReLU, store (f32 or bf16).
#include <algorithm>
#include <type_traits>

#include "aps_common.h"
#include "mfma_frag.h"

using namespace aps;

namespace {

constexpr int kChunk = 32;
constexpr int kMaxTM = 4;
constexpr int kModeReluMask = 3;  // internal staging mode of the data-gradient convolution

struct ConvArgs {
  const void* x;
  const void* x2;
  int N, H, W;   // output (= conv input after the transform) size
  int Cx, C2, mode;
  const void* wp;
  const float* bias;
  int Cout, nchunk, ntx;
  void* y;
  int ldy, relu;
  // optional 1x1 head fused into the epilogue (see k_conv); store_main = also write y
  const void* hw;
  const float* hb;
  int hK;
  void* hy;
  int hldy, store_main;
  // optional side output of three head channels [hside_off, hside_off + 3) as [N,H,W,4] (the
  // fourth entry 0), written from the staged logit rows (conv_epilogue)
  void* hside;
  int hside_off;
  // optional 2x2 average pool of the (bf16-rounded) output, [N, H/2, W/2, Cout] (k_conv_lds)
  void* pool;
  int ntiles, nco;  // pixel tiles per image, output-channel blocks (block order: xcd_tile)
};

// Blocks are dispatched round-robin over the 8 XCDs (block id % 8), each with its own L2.  XCD x
// takes the contiguous tile range [x T8, (x+1) T8) and, per tile, all channel blocks back to back,
// so the halo rows shared by neighbouring tiles and the input tile shared by a tile's channel
// blocks are re-read from that XCD's L2 rather than from HBM.  grid.x = 8 T8 nco; blocks past the
// last tile exit.
struct TileId {
  int tile, cob;
};
__device__ inline TileId xcd_tile(int id, int ntiles, int nco) {
  const int t8 = (ntiles + 7) / 8, xcd = id & 7, k = id >> 3;
  return TileId{xcd * t8 + k / nco, k % nco};
}
inline int xcd_grid(int ntiles, int nco) { return 8 * ((ntiles + 7) / 8) * nco; }

// ---- 8-element vectors of the storage type ---------------------------------------------
struct V8f {
  float v[8];
};

__device__ inline V8f load8(const float* p) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  return V8f{{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w}};
}
__device__ inline V8f load8(const uint16_t* p) {
  const u16x8 h = *reinterpret_cast<const u16x8*>(p);
  V8f r;
#pragma unroll
  for (int e = 0; e < 8; ++e) r.v[e] = bf2f(h[e]);
  return r;
}
__device__ inline void store8(float* p, const V8f& r) {
  *reinterpret_cast<float4*>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
  *reinterpret_cast<float4*>(p + 4) = make_float4(r.v[4], r.v[5], r.v[6], r.v[7]);
}
__device__ inline void store8(uint16_t* p, const V8f& r) {
  u16x8 h;
#pragma unroll
  for (int e = 0; e < 8; ++e) h[e] = f2bf(r.v[e]);
  *reinterpret_cast<u16x8*>(p) = h;
}
// Stage channels [ci, ci+8) of input pixel (iy, ix) into LDS.
template <typename T>
__device__ inline void stage8(const ConvArgs& a, int n, int iy, int ix, int ci, T* dst) {
  const int Cin = a.Cx + a.C2;
  if (iy < 0 || iy >= a.H || ix < 0 || ix >= a.W || ci >= Cin) {
    zero8(dst);
    return;
  }
  const T* x = static_cast<const T*>(a.x);
  if ((a.mode == APS_CONV_DIRECT || a.mode == kModeReluMask) && ci + 8 > a.Cx) {
    // channel tail of a row whose stride is not a multiple of 8 (padded logit gradients)
    const size_t o = (((size_t)n * a.H + iy) * a.W + ix) * a.Cx + ci;
    const T* y = static_cast<const T*>(a.x2);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const bool ok = ci + e < a.Cx && (a.mode == APS_CONV_DIRECT || Ld<T>::get(y, o + e) > 0.f);
      dst[e] = ok ? x[o + e] : T(0);
    }
  } else if (a.mode == APS_CONV_DIRECT) {
    copy8(dst, x + (((size_t)n * a.H + iy) * a.W + ix) * a.Cx + ci);
  } else if (a.mode == kModeReluMask) {
    // x = dLoss/dy, x2 = y (post-ReLU output, same layout): stage dy where y > 0, else 0
    const size_t o = (((size_t)n * a.H + iy) * a.W + ix) * a.Cx + ci;
    const V8f g = load8(x + o), y = load8(static_cast<const T*>(a.x2) + o);
    V8f r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r.v[e] = y.v[e] > 0.f ? g.v[e] : 0.f;
    store8(dst, r);
  } else if (a.mode == APS_CONV_POOL2) {
    const int W2 = 2 * a.W;
    const T* p = x + (((size_t)n * 2 * a.H + 2 * iy) * W2 + 2 * ix) * a.Cx + ci;
    const V8f q0 = load8(p), q1 = load8(p + a.Cx), q2 = load8(p + (size_t)W2 * a.Cx),
              q3 = load8(p + (size_t)W2 * a.Cx + a.Cx);
    V8f r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r.v[e] = ((q0.v[e] + q1.v[e]) + (q2.v[e] + q3.v[e])) * 0.25f;
    store8(dst, r);
  } else {  // APS_CONV_UP2_CAT
    if (ci < a.Cx) {
      const int Hh = a.H / 2, Wh = a.W / 2;
      copy8(dst, x + (((size_t)n * Hh + iy / 2) * Wh + ix / 2) * a.Cx + ci);
    } else {
      const T* x2 = static_cast<const T*>(a.x2);
      copy8(dst, x2 + (((size_t)n * a.H + iy) * a.W + ix) * a.C2 + (ci - a.Cx));
    }
  }
}

template <typename TO>
__device__ inline void store_out(TO* p, int ldy, int co0, int Cout, const float* v);
template <>
__device__ inline void store_out<float>(float* p, int ldy, int co0, int Cout, const float* v) {
  if ((ldy & 3) == 0 && co0 + 4 <= ldy) {
    *reinterpret_cast<float4*>(p + co0) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (co0 + q < Cout) p[co0 + q] = v[q];
  }
}
template <>
__device__ inline void store_out<uint16_t>(uint16_t* p, int ldy, int co0, int Cout, const float* v) {
  if ((ldy & 3) == 0 && co0 + 4 <= ldy) {
    *reinterpret_cast<u16x4*>(p + co0) = f2bf4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (co0 + q < Cout) p[co0 + q] = f2bf(v[q]);
  }
}

// Epilogue shared by the convolution kernels: bias, optional ReLU, store; with HEAD, the fused
// 1x1 head.  acc[m][j] holds output rows row0 + j, channels 16 (cob TM + m) + 4 (lane / 16) + q,
// pixel column tx0 + lane % 16.  Xs is the block's LDS tile, reused by the head's re-layout.
// s_waitcnt immediate (gfx9 encoding) that waits for all vector memory operations only:
// vmcnt = 0, expcnt = 7 and lgkmcnt = 15 (no wait on those).
constexpr int kWaitVm0 = 0x0F70;

// LDS the fused head's epilogue needs, in elements of the tile type T: per wave a [16 px][16 TM
// ch] re-layout region (row pitch 16 TM + 8 or + 4), then per wave a [16 px][<= 16 HM ch] staging
// region for the head outputs (type TO).  The kernels size their input tile at least this large.
// HM = head m-tiles (4: up to 64 logits, 5: up to 80); 0 = no fused head.
template <typename T, typename TO, int TM, int HM>
constexpr int head_lds_elems() {
  return 4 * 16 * (TM * 16 + (sizeof(T) == 2 ? 8 : 4)) + 4 * 16 * 16 * HM * (int)(sizeof(TO) / sizeof(T));
}

template <typename T, typename TO, int TM, int TN, int HEAD, bool BIAS_IN_ACC = false>
__device__ inline void conv_epilogue(const ConvArgs& a, f32x4 (&acc)[TM][TN], int row0, int tx0,
                                     int cob, int n, int lane, int wave, T* Xs) {
  TO* y = static_cast<TO*>(a.y);
  const int col = tx0 + (lane & 15);
  float bv[TM][4];  // this lane's bias values, loaded once
#pragma unroll
  for (int m = 0; m < TM; ++m) {
    const int co0 = (cob * TM + m) * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      bv[m][q] = !BIAS_IN_ACC && co0 + q < a.Cout && a.bias ? a.bias[co0 + q] : 0.f;
  }
  if constexpr (!HEAD) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int row = row0 + j;
      if (row >= a.H || col >= a.W) continue;
      TO* py = y + (((size_t)n * a.H + row) * a.W + col) * a.ldy;
#pragma unroll
      for (int m = 0; m < TM; ++m) {
        const int co0 = (cob * TM + m) * 16 + 4 * (lane >> 4);
        if (co0 >= a.Cout) continue;
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float t = acc[m][j][q] + bv[m][q];
          v[q] = a.relu ? fmaxf(t, 0.f) : t;
        }
        store_out<TO>(py, a.ldy, co0, a.Cout, v);
      }
    }
  } else {
    // Fused 1x1 head on this layer's output (all Cout = 16 TM channels are in this block):
    // each wave re-lays its row-j tile [16 px][16 TM ch] out through its own LDS region as MFMA
    // B fragments and multiplies it by the packed head weights (held in registers), the same
    // operands in the same order as the stand-alone 1x1 convolution of the stored tile.  The
    // regions are per wave, so after the caller's barrier only wave-local ordering is needed.
    // Head outputs go out through a second per-wave region: the row's [npx][hldy] run of
    // logits is contiguous in memory, so the wave writes it with 16-byte vector stores to
    // consecutive addresses (channels in [hK, hldy) as zeros) instead of one 8- or 16-byte piece
    // per lane and 16-channel group at the pixel stride, which measured about twice as slow.
    constexpr int CC = TM * 16, YP = CC + (sizeof(T) == 2 ? 8 : 4), HM = HEAD;
    T* Ys = Xs + wave * 16 * YP;
    TO* Os = reinterpret_cast<TO*>(Xs + 4 * 16 * YP) + wave * 16 * 16 * HM;
    const bool staged = a.hldy <= 16 * HM && (a.hldy * (int)sizeof(TO)) % 16 == 0 &&
                        (reinterpret_cast<uintptr_t>(a.hy) & 15) == 0;
    const int npx = a.W - tx0 < 16 ? a.W - tx0 : 16;
    const T* hw = static_cast<const T*>(a.hw);
    TO* hy = static_cast<TO*>(a.hy);
    Frag<T> hwf[HM][TM / 2];
#pragma unroll
    for (int mh = 0; mh < HM; ++mh)
#pragma unroll
      for (int cc = 0; cc < TM / 2; ++cc)
        if (mh * 16 < a.hK) frag_load(hwf[mh][cc], hw + ((((size_t)mh * (TM / 2)) + cc) * 64 + lane) * 8);
    // head biases: unconditional loads (index clamped to a valid entry), then one wait for them
    // and the head weights here.  Left to the compiler, the wait for a value loaded under a
    // branch is placed at each use inside the later (branching) store code, and as vmcnt also
    // counts stores, every one of those waits would drain all stores issued before it.
    float hb[HM][4];
#pragma unroll
    for (int mh = 0; mh < HM; ++mh)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = mh * 16 + 4 * (lane >> 4) + q;
        const float v = a.hb[k < a.hK ? k : 0];
        hb[mh][q] = k < a.hK ? v : 0.f;
      }
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int row = row0 + j;
      const bool inpx = row < a.H && col < a.W;
#pragma unroll
      for (int m = 0; m < TM; ++m) {
        const int co0 = m * 16 + 4 * (lane >> 4);
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float t = acc[m][j][q] + bv[m][q];
          v[q] = a.relu ? fmaxf(t, 0.f) : t;
        }
        if constexpr (sizeof(T) == 2)
          *reinterpret_cast<u16x4*>(Ys + (lane & 15) * YP + co0) = f2bf4(v[0], v[1], v[2], v[3]);
        else
          *reinterpret_cast<float4*>(Ys + (lane & 15) * YP + co0) = make_float4(v[0], v[1], v[2], v[3]);
        if (a.store_main && inpx)
          store_out<TO>(y + (((size_t)n * a.H + row) * a.W + col) * a.ldy, a.ldy, co0, a.Cout, v);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      Frag<T> bf[TM / 2];
#pragma unroll
      for (int cc = 0; cc < TM / 2; ++cc) frag_load(bf[cc], Ys + (lane & 15) * YP + 32 * cc + 8 * (lane >> 4));
      if (staged) {
#pragma unroll
        for (int mh = 0; mh < HM; ++mh) {
          const int k0 = mh * 16 + 4 * (lane >> 4);
          if (mh * 16 >= a.hldy) break;
          f32x4 h = f32x4{0.f, 0.f, 0.f, 0.f};
          if (mh * 16 < a.hK) {
#pragma unroll
            for (int cc = 0; cc < TM / 2; ++cc) h = mma(hwf[mh][cc], bf[cc], h);
          }
          float o[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) o[q] = k0 + q < a.hK ? h[q] + hb[mh][q] : 0.f;
          if (k0 < a.hldy) {
            if constexpr (sizeof(TO) == 2)
              *reinterpret_cast<u16x4*>(Os + (lane & 15) * a.hldy + k0) = f2bf4(o[0], o[1], o[2], o[3]);
            else
              *reinterpret_cast<f32x4*>(Os + (lane & 15) * a.hldy + k0) = f32x4{o[0], o[1], o[2], o[3]};
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (row < a.H) {
          const int nvec = npx * a.hldy * (int)sizeof(TO) / 16;
          uint4* dst = reinterpret_cast<uint4*>(hy + (((size_t)n * a.H + row) * a.W + tx0) * a.hldy);
          const uint4* src = reinterpret_cast<const uint4*>(Os);
          // nontemporal: the logits are read back only by the filter, after the other heads
          for (int v = lane; v < nvec; v += 64)
            __builtin_nontemporal_store(reinterpret_cast<const u32x4*>(src)[v], reinterpret_cast<u32x4*>(dst) + v);
          if (a.hside && lane < npx) {
            const TO* op = Os + lane * a.hldy + a.hside_off;
            TO* sp = static_cast<TO*>(a.hside) + (((size_t)n * a.H + row) * a.W + tx0 + lane) * 4;
            if constexpr (sizeof(TO) == 2)
              *reinterpret_cast<u16x4*>(sp) = u16x4{op[0], op[1], op[2], (uint16_t)0};
            else
              *reinterpret_cast<f32x4*>(sp) = f32x4{op[0], op[1], op[2], 0.f};
          }
        }
      } else {
#pragma unroll
        for (int mh = 0; mh < HM; ++mh) {
          if (mh * 16 >= a.hK) break;
          f32x4 h = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int cc = 0; cc < TM / 2; ++cc) h = mma(hwf[mh][cc], bf[cc], h);
          const int k0 = mh * 16 + 4 * (lane >> 4);
          if (inpx && k0 < a.hK) {
            float o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = h[q] + hb[mh][q];
            store_out<TO>(hy + (((size_t)n * a.H + row) * a.W + col) * a.hldy, a.hldy, k0, a.hK, o);
          }
        }
      }
      // the next row's re-layout overwrites Ys
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// CG = 8-channel input groups per pixel in the K layout.  CG = 4: K walks 32-channel chunks,
// one tap per MFMA step.  CG = 1 or 2 (inputs of at most 8 or 16 channels, a single chunk): K
// enumerates (tap, group) pairs, so one MFMA step covers 4 / CG taps and no MFMA work is
// spent on channel padding; lane group q of step s takes pair p = 4 s + q.
template <typename T, typename TO, int KS, int TM, int TN, int CG, int HEAD = 0>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
  constexpr int R = KS / 2;
  constexpr int TH = 4 * TN, TWp = 16;
  constexpr int SW = TWp + 2 * R, SH = TH + 2 * R;
  constexpr int PS = sizeof(T) == 2 ? 40 : 36;  // padded LDS pixel stride (elements)
  constexpr int XS_HEAD = HEAD ? head_lds_elems<T, TO, TM, HEAD>() : 0;
  __shared__ __attribute__((aligned(16))) T Xs[SH * SW * PS > XS_HEAD ? SH * SW * PS : XS_HEAD];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const TileId tid_ = xcd_tile(blockIdx.x, a.ntiles, a.nco);
  if (tid_.tile >= a.ntiles) return;
  const int tx0 = (tid_.tile % a.ntx) * TWp, ty0 = (tid_.tile / a.ntx) * TH;
  const int cob = tid_.cob, n = blockIdx.z;
  const T* wp = static_cast<const T*>(a.wp);

  f32x4 acc[TM][TN];
#pragma unroll
  for (int m = 0; m < TM; ++m)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  if constexpr (CG < 4) {
    constexpr int NPAIR = KS * KS * CG, STEPS = (NPAIR + 3) / 4;
    for (int it = tid; it < SH * SW * CG; it += 256) {
      const int g = it % CG, p = it / CG;
      const int r = p / SW, col = p % SW;
      stage8<T>(a, n, ty0 - R + r, tx0 - R + col, g * 8, Xs + p * PS + g * 8);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      const int p = 4 * s + (lane >> 4);
      const int tap = p < NPAIR ? p / CG : 0, g = p < NPAIR ? p % CG : 0;  // padded pairs: zero weights
      const int dy = tap / KS - R, dx = tap % KS - R;
      Frag<T> wf[TM];
#pragma unroll
      for (int m = 0; m < TM; ++m)
        frag_load(wf[m], wp + ((((size_t)(cob * TM + m) * STEPS + s) * 64 + lane) * 8));
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int row = wave * TN + j + R + dy, col = (lane & 15) + R + dx;
        Frag<T> bf;
        frag_load(bf, Xs + (row * SW + col) * PS + g * 8);
#pragma unroll
        for (int m = 0; m < TM; ++m) acc[m][j] = mma(wf[m], bf, acc[m][j]);
      }
    }
  }

  for (int c = 0; c < (CG < 4 ? 0 : a.nchunk); ++c) {
    for (int it = tid; it < SH * SW * 4; it += 256) {
      const int g = it & 3, p = it >> 2;
      const int r = p / SW, col = p % SW;
      stage8<T>(a, n, ty0 - R + r, tx0 - R + col, c * kChunk + g * 8, Xs + p * PS + g * 8);
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < KS * KS; ++tap) {
      const int dy = tap / KS - R, dx = tap % KS - R;
      Frag<T> wf[TM];
#pragma unroll
      for (int m = 0; m < TM; ++m) {
        const size_t idx = ((((size_t)(cob * TM + m) * KS * KS + tap) * a.nchunk + c) * 64 + lane) * 8;
        frag_load(wf[m], wp + idx);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int row = wave * TN + j + R + dy, col = (lane & 15) + R + dx;
        Frag<T> bf;
        frag_load(bf, Xs + (row * SW + col) * PS + (lane >> 4) * 8);
#pragma unroll
        for (int m = 0; m < TM; ++m) acc[m][j] = mma(wf[m], bf, acc[m][j]);
      }
    }
    __syncthreads();
  }

  conv_epilogue<T, TO, TM, TN, HEAD>(a, acc, ty0 + wave * TN, tx0, cob, n, lane, wave, Xs);
}

// ---- bf16 3x3 convolution with both MFMA operands in LDS ---------------------------------
// Block: 4 waves stacked vertically, each owning TN output rows x 16 px; all four share the
// block's TM m-tiles (16 TM output channels).  Per 32-channel chunk, the block's weight
// fragments (TM x 9 fragments of 1 KB, one per m-tile and tap) and the input tile (4 TN + 2
// rows x 18 px with the 1-px halo) sit in LDS.  The global loads of chunk c+1 are issued
// before the MFMAs of chunk c and held in registers until the chunk's barrier, so the MFMA loop
// waits on LDS reads only.  For each column offset dx, every input-row fragment is read once
// and feeds the (up to) three output rows it contributes to: 3 TM A and TN + 2 B reads per
// 3 TN TM MFMAs.

constexpr uint32_t kNoPixel = 0xffffffffu;

// bf16 y > 0 (positive, finite or +inf), decided on the bits
__device__ inline bool bf_pos(uint16_t b) { return (int16_t)b > 0 && (b & 0x7fffu) <= 0x7f80u; }

template <int MODE, int TM, int TN, int HEAD>
__global__ __launch_bounds__(256, 2) void k_conv_lds(ConvArgs a) {
  constexpr int ROWS = 4 * TN, SH = ROWS + 2, SW = 18, PS = 40;
  constexpr int NXV = SH * SW * 4, NXT = (NXV + 255) / 256;  // input 16-B vectors per chunk
  constexpr int NAV = TM * 9 * 64, NAT = (NAV + 255) / 256;  // weight 16-B vectors per chunk
  constexpr int XS_TILE = SH * SW * PS, XS_HEAD = HEAD ? head_lds_elems<uint16_t, uint16_t, TM, HEAD>() : 0;
  __shared__ __attribute__((aligned(16))) uint16_t Xs[XS_TILE > XS_HEAD ? XS_TILE : XS_HEAD];
  __shared__ __attribute__((aligned(16))) uint16_t As[NAV * 8];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const TileId tid_ = xcd_tile(blockIdx.x, a.ntiles, a.nco);
  if (tid_.tile >= a.ntiles) return;
  const int tx0 = (tid_.tile % a.ntx) * 16, ty0 = (tid_.tile / a.ntx) * ROWS;
  const int cob = tid_.cob, n = blockIdx.z;
  const uint16_t* x = static_cast<const uint16_t*>(a.x);
  const uint16_t* x2 = static_cast<const uint16_t*>(a.x2);
  const uint16_t* wp = static_cast<const uint16_t*>(a.wp);
  const int Cin = a.Cx + a.C2;
  // This thread stages channel group g (8 channels) of tile pixels (tid / 4) + 64 k.  Their
  // element offsets at chunk 0 are computed once (32-bit; kNoPixel outside the image):
  // xo into x (for POOL2 the top-left of the 2x2 window, for UP2_CAT the parent pixel of the
  // coarse tensor), so into the skip tensor x2 (UP2_CAT only).
  // Lane l of wave w stages pixel 16 w + l % 16 (+ 64 k) and channel group l / 16: a 16-lane
  // group writes 16 consecutive tile pixels at the padded pixel stride, which hits distinct LDS
  // banks (four lanes per pixel at one stride would collide every fourth pixel).
  const int g8 = ((tid >> 4) & 3) * 8;
  const int pl = (tid >> 6) * 16 + (tid & 15);
  uint32_t xo[NXT], so[MODE == APS_CONV_UP2_CAT ? NXT : 1];
#pragma unroll
  for (int k = 0; k < NXT; ++k) {
    const int p = pl + 64 * k, r = p / SW, col = p - r * SW;
    const int iy = ty0 - 1 + r, ix = tx0 - 1 + col;
    const bool in = p < SH * SW && iy >= 0 && iy < a.H && ix >= 0 && ix < a.W;
    uint32_t o = kNoPixel;
    if (in) {
      if constexpr (MODE == APS_CONV_POOL2)
        o = (uint32_t)((((size_t)n * 2 * a.H + 2 * iy) * (2 * a.W) + 2 * ix) * a.Cx + g8);
      else if constexpr (MODE == APS_CONV_UP2_CAT)
        o = (uint32_t)((((size_t)n * (a.H / 2) + iy / 2) * (a.W / 2) + ix / 2) * a.Cx + g8);
      else
        o = (uint32_t)((((size_t)n * a.H + iy) * a.W + ix) * a.Cx + g8);
    }
    xo[k] = o;
    if constexpr (MODE == APS_CONV_UP2_CAT)
      so[k] = in ? (uint32_t)((((size_t)n * a.H + iy) * a.W + ix) * a.C2 + g8) : kNoPixel;
  }
  // weights: vector v = tid + 256 k of the chunk is fragment f = v / 64 (m-tile f / 9, tap f % 9)
  const uint32_t wo = (uint32_t)((((size_t)cob * TM * 9 + wave) * a.nchunk) * 512 + lane * 8);
  const uint32_t wstep = (uint32_t)(4 * a.nchunk * 512);

  // Global loads of the next chunk are issued unconditionally (out-of-range lanes read a valid
  // dummy address) so that no branch join forces the compiler to wait for them before the
  // current chunk's MFMAs; the zero fill of halo pixels and channels beyond Cin is applied when
  // the registers are written to LDS.  The pooled and masked transforms combine several loads
  // and are evaluated at fetch time.
  u16x8 px[NXT], pa[NAT];
  uint32_t okbits = 0;
  auto fetch = [&](int c) {
    const int cb = c * kChunk;
    const bool in_ch = cb + g8 < Cin;
    okbits = 0;
#pragma unroll
    for (int k = 0; k < NXT; ++k) {
      const bool ok = xo[k] != kNoPixel && in_ch;
      okbits |= (uint32_t)ok << k;
      if constexpr (MODE == APS_CONV_DIRECT) {
        px[k] = *reinterpret_cast<const u16x8*>(x + (ok ? xo[k] + cb : 0u));
      } else if constexpr (MODE == APS_CONV_UP2_CAT) {
        // channels [0, Cx) from the coarse tensor, then the skip tensor
        const uint16_t* src = cb + g8 < a.Cx ? x + (xo[k] + cb) : x2 + (so[k] + (cb - a.Cx));
        px[k] = *reinterpret_cast<const u16x8*>(ok ? src : x);
      } else {
        u16x8 v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        if (ok) {
          if constexpr (MODE == kModeReluMask) {
            // x = dLoss/dy, x2 = the layer's post-ReLU output: dy where y > 0
            const u16x8 gr = *reinterpret_cast<const u16x8*>(x + (xo[k] + cb));
            const u16x8 yv = *reinterpret_cast<const u16x8*>(x2 + (xo[k] + cb));
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = bf_pos(yv[e]) ? gr[e] : (uint16_t)0;
          } else {  // APS_CONV_POOL2
            const uint32_t rs = (uint32_t)(2 * a.W * a.Cx);
            const uint32_t o = xo[k] + cb;
            const V8f q0 = load8(x + o), q1 = load8(x + (o + a.Cx)), q2 = load8(x + (o + rs)),
                      q3 = load8(x + (o + rs + a.Cx));
            float r[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) r[e] = ((q0.v[e] + q1.v[e]) + (q2.v[e] + q3.v[e])) * 0.25f;
            const u16x4 lo = f2bf4(r[0], r[1], r[2], r[3]), hi = f2bf4(r[4], r[5], r[6], r[7]);
            v = u16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
          }
        }
        px[k] = v;
      }
    }
#pragma unroll
    for (int k = 0; k < NAT; ++k)
      pa[k] = *reinterpret_cast<const u16x8*>(wp + ((tid + 256 * k < NAV ? wo + k * wstep : wo) + c * 512));
  };
  auto put = [&]() {
#pragma unroll
    for (int k = 0; k < NXT; ++k) {
      const int p = pl + 64 * k;
      if (p < SH * SW) {
        const u16x8 v = (okbits >> k) & 1u ? px[k] : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        *reinterpret_cast<u16x8*>(Xs + p * PS + g8) = v;
      }
    }
#pragma unroll
    for (int k = 0; k < NAT; ++k) {
      const int v = tid + 256 * k;
      if (v < NAV) *reinterpret_cast<u16x8*>(As + v * 8) = pa[k];
    }
  };

  // accumulators start at the bias
  f32x4 acc[TM][TN];
#pragma unroll
  for (int m = 0; m < TM; ++m) {
    f32x4 b0 = f32x4{0.f, 0.f, 0.f, 0.f};
    const int co0 = (cob * TM + m) * 16 + 4 * (lane >> 4);
    if (a.bias && co0 < a.Cout) b0 = *reinterpret_cast<const f32x4*>(a.bias + co0);
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[m][j] = b0;
  }

  fetch(0);
  put();
  __syncthreads();
  for (int c = 0; c < a.nchunk; ++c) {
    const bool more = c + 1 < a.nchunk;
    if (more) fetch(c + 1);
    // pooled inputs are averaged now rather than holding four raw loads across the MFMAs
    if constexpr (MODE == APS_CONV_POOL2) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      __builtin_amdgcn_sched_barrier(0);  // keep one dx step's fragments live at a time
      Frag<uint16_t> A[3][TM];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int m = 0; m < TM; ++m) frag_load(A[dy][m], As + ((m * 9 + dy * 3 + dx) * 64 + lane) * 8);
#pragma unroll
      for (int ir = 0; ir < TN + 2; ++ir) {
        Frag<uint16_t> B;
        frag_load(B, Xs + ((wave * TN + ir) * SW + (lane & 15) + dx) * PS + (lane >> 4) * 8);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const int j = ir - dy;
          if (j >= 0 && j < TN) {
#pragma unroll
            for (int m = 0; m < TM; ++m) acc[m][j] = mma(A[dy][m], B, acc[m][j]);
          }
        }
      }
    }
    if (more) {
      __syncthreads();
      put();
      __syncthreads();
    }
  }
  if constexpr (HEAD) {
    __syncthreads();  // the head's re-layout reuses Xs
    conv_epilogue<uint16_t, uint16_t, TM, TN, HEAD, true>(a, acc, ty0 + wave * TN, tx0, cob, n, lane, wave, Xs);
  } else {
    // bf16 store of 4 channels per lane; ReLU on the rounded bits (round-to-nearest-even keeps
    // the sign, so this equals rounding max(v, 0)).  Cout % 16 == 0 and ldy % 4 == 0 (host).
    // With a.pool, the 2x2 mean of the stored values (rows j, j+1 of this lane; columns of
    // this lane and its neighbour lane ^ 1), summed in the order of the POOL2 input transform,
    // goes to the half-resolution tensor; H, W and the tile origins are even.
    uint16_t* y = static_cast<uint16_t*>(a.y);
    uint16_t* yp = static_cast<uint16_t*>(a.pool);
    const int col = tx0 + (lane & 15);
#pragma unroll
    for (int j0 = 0; j0 < TN; j0 += 2) {
#pragma unroll
      for (int m = 0; m < TM; ++m) {
        const int co = (cob * TM + m) * 16 + 4 * (lane >> 4);
        if (co >= a.Cout) continue;
        s16x4 h[2];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int j = j0 + jj, row = ty0 + wave * TN + j;
          h[jj] = __builtin_bit_cast(s16x4, f2bf4(acc[m][j][0], acc[m][j][1], acc[m][j][2], acc[m][j][3]));
          if (a.relu) h[jj] = __builtin_elementwise_max(h[jj], s16x4{0, 0, 0, 0});
          if (row < a.H && col < a.W)
            *reinterpret_cast<s16x4*>(y + (((size_t)n * a.H + row) * a.W + col) * a.ldy + co) = h[jj];
        }
        if (yp) {
          // neighbour column's values (all lanes take part in the exchange)
          s16x4 nb[2];
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            const uint2 u = __builtin_bit_cast(uint2, h[jj]);
            // DPP quad_perm [1,0,3,2]: lane l reads lane l ^ 1
            nb[jj] = __builtin_bit_cast(
                s16x4, make_uint2((uint32_t)__builtin_amdgcn_update_dpp(0, (int)u.x, 0xB1, 0xF, 0xF, true),
                                  (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u.y, 0xB1, 0xF, 0xF, true)));
          }
          const int row = ty0 + wave * TN + j0;
          if ((lane & 1) == 0 && row < a.H && col < a.W) {
            float r[4];
#pragma unroll
            for (int e = 0; e < 4; ++e)
              r[e] = ((bf2f((uint16_t)h[0][e]) + bf2f((uint16_t)nb[0][e])) +
                      (bf2f((uint16_t)h[1][e]) + bf2f((uint16_t)nb[1][e]))) * 0.25f;
            *reinterpret_cast<u16x4*>(yp + (((size_t)n * (a.H / 2) + row / 2) * (a.W / 2) + col / 2) * a.Cout + co) =
                f2bf4(r[0], r[1], r[2], r[3]);
          }
        }
      }
    }
  }
}

// ---- fp32 3x3 convolution with both MFMA operands in LDS --------------------------------------
// k_conv_lds for fp32 on v_mfma_f32_16x16x4_f32: chunks of 16 input channels (4 per lane per
// fragment, 4 MFMAs per fragment pair), pixel stride 20 floats in LDS (80 B, conflict-free for the
// 16 lanes of a B fragment), weights packed by k_pack_f32c16.  Same tiling, row reuse, prefetch
// and epilogue rules as the bf16 kernel; the pooled copy averages the fp32 outputs in the order of
// the POOL2 input transform.
__device__ inline f32x4 mma4(f32x4 a, f32x4 b, f32x4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
}

// The value of lane l ^ 1 (DPP quad_perm [1,0,3,2]).  By value on purpose: a bit cast applied
// directly to a vector-element subscript was compiled as a read of element 0.
__device__ inline float lane_xor1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, true));
}

template <int TM, int TN>
__device__ inline void lds_epilogue_f32(const ConvArgs& a, f32x4 (&acc)[TM][TN], int row0, int tx0,
                                        int cob, int n, int lane) {
  float* y = static_cast<float*>(a.y);
  float* yp = static_cast<float*>(a.pool);
  const int col = tx0 + (lane & 15);
#pragma unroll
  for (int j0 = 0; j0 < TN; j0 += 2) {
#pragma unroll
    for (int m = 0; m < TM; ++m) {
      const int co = (cob * TM + m) * 16 + 4 * (lane >> 4);
      if (co >= a.Cout) continue;
      f32x4 h[2];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int j = j0 + jj, row = row0 + j;
        f32x4 v = acc[m][j];
        if (a.relu) {
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = fmaxf(v[q], 0.f);
        }
        h[jj] = v;
        if (row < a.H && col < a.W) {
          const float vv[4] = {v[0], v[1], v[2], v[3]};
          store_out<float>(y + (((size_t)n * a.H + row) * a.W + col) * a.ldy, a.ldy, co, a.Cout, vv);
        }
      }
      if (yp) {
        f32x4 nb[2];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
          for (int q = 0; q < 4; ++q) nb[jj][q] = lane_xor1(h[jj][q]);
        const int row = row0 + j0;
        if ((lane & 1) == 0 && row < a.H && col < a.W)
          *reinterpret_cast<f32x4*>(yp + (((size_t)n * (a.H / 2) + row / 2) * (a.W / 2) + col / 2) * a.Cout + co) =
              ((h[0] + nb[0]) + (h[1] + nb[1])) * 0.25f;
      }
    }
  }
}

template <int MODE, int TM, int TN, int HEAD>
__global__ __launch_bounds__(256, 2) void k_conv_lds_f32(ConvArgs a) {
  constexpr int KC = 16, ROWS = 4 * TN, SH = ROWS + 2, SW = 18, PS = 20;
  constexpr int NXV = SH * SW * 4, NXT = (NXV + 255) / 256;  // input 16-B vectors per chunk
  constexpr int NAV = TM * 9 * 64, NAT = (NAV + 255) / 256;  // weight 16-B vectors per chunk
  // the fused head's epilogue reuses Xs (re-layout and output staging regions)
  constexpr int XS_TILE = SH * SW * PS, XS_HEAD = HEAD ? head_lds_elems<float, float, TM, HEAD>() : 0;
  __shared__ __attribute__((aligned(16))) float Xs[XS_TILE > XS_HEAD ? XS_TILE : XS_HEAD];
  __shared__ __attribute__((aligned(16))) float As[NAV * 4];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const TileId tid_ = xcd_tile(blockIdx.x, a.ntiles, a.nco);
  if (tid_.tile >= a.ntiles) return;
  const int tx0 = (tid_.tile % a.ntx) * 16, ty0 = (tid_.tile / a.ntx) * ROWS;
  const int cob = tid_.cob, n = blockIdx.z;
  const float* x = static_cast<const float*>(a.x);
  const float* x2 = static_cast<const float*>(a.x2);
  const float* wp = static_cast<const float*>(a.wp);
  const int Cin = a.Cx + a.C2;
  // This thread stages channel group g (4 channels) of tile pixel 16 w + l % 16 + 64 k, g = l / 16
  // (lane l of wave w; bank-conflict-free writes as in k_conv_lds; offsets in floats).
  const int g4 = ((tid >> 4) & 3) * 4;
  const int pl = (tid >> 6) * 16 + (tid & 15);
  uint32_t xo[NXT], so[MODE == APS_CONV_UP2_CAT ? NXT : 1];
#pragma unroll
  for (int k = 0; k < NXT; ++k) {
    const int p = pl + 64 * k, r = p / SW, col = p - r * SW;
    const int iy = ty0 - 1 + r, ix = tx0 - 1 + col;
    const bool in = p < SH * SW && iy >= 0 && iy < a.H && ix >= 0 && ix < a.W;
    uint32_t o = kNoPixel;
    if (in) {
      if constexpr (MODE == APS_CONV_POOL2)
        o = (uint32_t)((((size_t)n * 2 * a.H + 2 * iy) * (2 * a.W) + 2 * ix) * a.Cx + g4);
      else if constexpr (MODE == APS_CONV_UP2_CAT)
        o = (uint32_t)((((size_t)n * (a.H / 2) + iy / 2) * (a.W / 2) + ix / 2) * a.Cx + g4);
      else
        o = (uint32_t)((((size_t)n * a.H + iy) * a.W + ix) * a.Cx + g4);
    }
    xo[k] = o;
    if constexpr (MODE == APS_CONV_UP2_CAT)
      so[k] = in ? (uint32_t)((((size_t)n * a.H + iy) * a.W + ix) * a.C2 + g4) : kNoPixel;
  }
  const uint32_t wo = (uint32_t)((((size_t)cob * TM * 9 + wave) * a.nchunk) * 256 + lane * 4);
  const uint32_t wstep = (uint32_t)(4 * a.nchunk * 256);

  f32x4 px[NXT], pa[NAT];  // clang vector types: HIP's struct vectors are not promoted here
  uint32_t okbits = 0;
  const f32x4 zero4 = f32x4{0.f, 0.f, 0.f, 0.f};
  auto fetch = [&](int c) {
    const int cb = c * KC;
    const bool in_ch = cb + g4 < Cin;
    okbits = 0;
#pragma unroll
    for (int k = 0; k < NXT; ++k) {
      const bool ok = xo[k] != kNoPixel && in_ch;
      okbits |= (uint32_t)ok << k;
      if constexpr (MODE == APS_CONV_DIRECT) {
        px[k] = *reinterpret_cast<const f32x4*>(x + (ok ? xo[k] + cb : 0u));
      } else if constexpr (MODE == APS_CONV_UP2_CAT) {
        const float* src = cb + g4 < a.Cx ? x + (xo[k] + cb) : x2 + (so[k] + (cb - a.Cx));
        px[k] = *reinterpret_cast<const f32x4*>(ok ? src : x);
      } else {
        f32x4 v = zero4;
        if (ok) {
          if constexpr (MODE == kModeReluMask) {
            const f32x4 gr = *reinterpret_cast<const f32x4*>(x + (xo[k] + cb));
            const f32x4 yv = *reinterpret_cast<const f32x4*>(x2 + (xo[k] + cb));
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = yv[q] > 0.f ? gr[q] : 0.f;
          } else {  // APS_CONV_POOL2
            const uint32_t rs = (uint32_t)(2 * a.W * a.Cx);
            const uint32_t o = xo[k] + cb;
            const f32x4 q0 = *reinterpret_cast<const f32x4*>(x + o);
            const f32x4 q1 = *reinterpret_cast<const f32x4*>(x + (o + a.Cx));
            const f32x4 q2 = *reinterpret_cast<const f32x4*>(x + (o + rs));
            const f32x4 q3 = *reinterpret_cast<const f32x4*>(x + (o + rs + a.Cx));
            v = ((q0 + q1) + (q2 + q3)) * 0.25f;
          }
        }
        px[k] = v;
      }
    }
#pragma unroll
    for (int k = 0; k < NAT; ++k)
      pa[k] = *reinterpret_cast<const f32x4*>(wp + ((tid + 256 * k < NAV ? wo + k * wstep : wo) + c * 256));
  };
  auto put = [&]() {
#pragma unroll
    for (int k = 0; k < NXT; ++k) {
      const int p = pl + 64 * k;
      if (p < SH * SW) *reinterpret_cast<f32x4*>(Xs + p * PS + g4) = (okbits >> k) & 1u ? px[k] : zero4;
    }
#pragma unroll
    for (int k = 0; k < NAT; ++k) {
      const int v = tid + 256 * k;
      if (v < NAV) *reinterpret_cast<f32x4*>(As + v * 4) = pa[k];
    }
  };

  f32x4 acc[TM][TN];
#pragma unroll
  for (int m = 0; m < TM; ++m) {
    f32x4 b0 = f32x4{0.f, 0.f, 0.f, 0.f};
    const int co0 = (cob * TM + m) * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (a.bias && co0 + q < a.Cout) b0[q] = a.bias[co0 + q];
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[m][j] = b0;
  }

  fetch(0);
  put();
  __syncthreads();
  for (int c = 0; c < a.nchunk; ++c) {
    const bool more = c + 1 < a.nchunk;
    if (more) fetch(c + 1);
    if constexpr (MODE == APS_CONV_POOL2 || MODE == kModeReluMask) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      __builtin_amdgcn_sched_barrier(0);
      f32x4 A[3][TM];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int m = 0; m < TM; ++m) A[dy][m] = *reinterpret_cast<const f32x4*>(As + ((m * 9 + dy * 3 + dx) * 64 + lane) * 4);
#pragma unroll
      for (int ir = 0; ir < TN + 2; ++ir) {
        const f32x4 B = *reinterpret_cast<const f32x4*>(Xs + ((wave * TN + ir) * SW + (lane & 15) + dx) * PS + (lane >> 4) * 4);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const int j = ir - dy;
          if (j >= 0 && j < TN) {
#pragma unroll
            for (int m = 0; m < TM; ++m) acc[m][j] = mma4(A[dy][m], B, acc[m][j]);
          }
        }
      }
    }
    if (more) {
      __syncthreads();
      put();
      __syncthreads();
    }
  }
  if constexpr (HEAD) {
    __syncthreads();  // the head's re-layout reuses Xs
    conv_epilogue<float, float, TM, TN, HEAD, true>(a, acc, ty0 + wave * TN, tx0, cob, n, lane, wave, Xs);
  } else {
    lds_epilogue_f32<TM, TN>(a, acc, ty0 + wave * TN, tx0, cob, n, lane);
  }
}

template <int MODE, int HEAD>
void launch_conv_lds_f32_m(const ConvArgs& a, hipStream_t st) {
  ConvArgs b = a;
  b.ntx = (a.W + 15) / 16;
  b.nchunk = (a.Cx + a.C2 + 15) / 16;
  // 8-row blocks (TN = 2) for small problems, and for POOL2 with TM = 4, whose 16-row variant
  // does not fit in 256 VGPRs
  const bool wide = a.Cout > 32;
  const bool tn2 = (size_t)a.N * a.H * a.W < 64 * 64 * 8 || (wide && MODE == APS_CONV_POOL2);
  const int rows = tn2 ? 8 : 16;
  b.ntiles = b.ntx * ((a.H + rows - 1) / rows);
  b.nco = wide ? (a.Cout + 63) / 64 : 1;
  dim3 grid(xcd_grid(b.ntiles, b.nco), 1, a.N);
  if (!wide) {
    if (tn2) k_conv_lds_f32<MODE, 2, 2, HEAD><<<grid, 256, 0, st>>>(b);
    else k_conv_lds_f32<MODE, 2, 4, HEAD><<<grid, 256, 0, st>>>(b);
  } else if (tn2) {
    k_conv_lds_f32<MODE, 4, 2, HEAD><<<grid, 256, 0, st>>>(b);
  } else if constexpr (MODE != APS_CONV_POOL2) {
    k_conv_lds_f32<MODE, 4, 4, HEAD><<<grid, 256, 0, st>>>(b);
  }
}

// Every fp32 3x3 convolution with more than 16 input channels (its weights are packed in
// 16-channel chunks, which only this kernel reads).  false: 32-bit offsets would overflow.
bool launch_conv_sweep_f32(const ConvArgs& a, hipStream_t st);  // the row sweep, below

template <int HEAD>
bool launch_conv_lds_f32(const ConvArgs& a, hipStream_t st) {
  const size_t px = (size_t)a.N * a.H * a.W;
  const size_t ex = a.mode == APS_CONV_POOL2 ? 4 * px * a.Cx
                    : a.mode == APS_CONV_UP2_CAT ? px / 4 * a.Cx : px * a.Cx;
  const size_t e2 = a.mode == APS_CONV_UP2_CAT ? px * a.C2 : 0;
  if ((ex > e2 ? ex : e2) + 16 >= ((size_t)1 << 31)) return false;
  if constexpr (HEAD) {
    if (a.mode != APS_CONV_DIRECT) return false;
    launch_conv_lds_f32_m<APS_CONV_DIRECT, HEAD>(a, st);
    return true;
  } else {
    if (launch_conv_sweep_f32(a, st)) return true;
    switch (a.mode) {
      case APS_CONV_DIRECT: launch_conv_lds_f32_m<APS_CONV_DIRECT, 0>(a, st); return true;
      case APS_CONV_POOL2: launch_conv_lds_f32_m<APS_CONV_POOL2, 0>(a, st); return true;
      case APS_CONV_UP2_CAT: launch_conv_lds_f32_m<APS_CONV_UP2_CAT, 0>(a, st); return true;
      case kModeReluMask: launch_conv_lds_f32_m<kModeReluMask, 0>(a, st); return true;
      default: return false;
    }
  }
}

// Launch k_conv_lds for a bf16 3x3 convolution with bf16 output whose input channels fill
// 32-channel chunks (Cin > 16); TM = 2 for Cout <= 32, else 4 with ceil(Cout / 64) channel
// blocks; 8-row blocks for small problems.
template <int MODE, int HEAD>
void launch_conv_lds_m(const ConvArgs& a, hipStream_t st) {
  ConvArgs b = a;
  b.ntx = (a.W + 15) / 16;
  const bool small = (size_t)a.N * a.H * a.W < 64 * 64 * 8;
  const int rows = small ? 8 : 16;
  b.ntiles = b.ntx * ((a.H + rows - 1) / rows);
  b.nco = a.Cout <= 32 ? 1 : (a.Cout + 63) / 64;
  dim3 grid(xcd_grid(b.ntiles, b.nco), 1, a.N);
  if (a.Cout <= 32) {
    if (small) k_conv_lds<MODE, 2, 2, HEAD><<<grid, 256, 0, st>>>(b);
    else k_conv_lds<MODE, 2, 4, HEAD><<<grid, 256, 0, st>>>(b);
  } else {
    if (small) k_conv_lds<MODE, 4, 2, HEAD><<<grid, 256, 0, st>>>(b);
    else k_conv_lds<MODE, 4, 4, HEAD><<<grid, 256, 0, st>>>(b);
  }
}

// ---- bf16 3x3 convolution with 32 output channels as a per-wave row sweep ----------------
// For the full-resolution 32-channel layers (16 or 32 input channels), and the half-resolution
// 32 -> 64 layer as two such halves, which move far more bytes than they compute: the tiled blocks stage a tile and its weights, compute for a fraction of the
// time and store, with too little work per block to hide the staging behind the other blocks of
// a CU.  Here each wave runs on its own, with no block barrier: it owns a band of 32 output
// columns and R output rows, keeps its weights in registers, and walks down the band one output
// row per step, reading each input row from HBM once (requested four steps before it is staged,
// two with a fused head, through a buffer resource whose out-of-image lanes return zeros) into a
// ring of four LDS rows.  Output row o is summed from input rows o - 1, o, o + 1 in the tiled
// kernel's order — taps dx outer, dy inner, one MFMA per tap over the 32 channels of the chunk
// (zeros above 16 input channels), starting from the bias — so the two kernels agree bit for bit
// and either may serve a layer.  The row is rounded to bf16, rectified on the rounded bits,
// staged in LDS and stored as 16-byte runs; with a pooled output every second row is averaged
// with the one before it in the order of the POOL2 input transform; with a fused 1x1 head (HM
// m-tiles of logits) the staged row is the head's B operand, as in the tiled epilogue.  LDS
// operations of one wave complete in program order, so no block barrier orders the ring or the
// staging rows; wave_lds_sync keeps the compiler from reordering them.
constexpr int kCsCols = 32;      // output columns per band (two 16-pixel n-tiles)
constexpr int kCsPix = 36;       // staged input positions per row: 34 read + 2 zero (pad reads)
constexpr long kCsWaves = 2048;  // waves per launch the band height aims at (two per SIMD)
constexpr int kCsDepth = 4;      // input rows requested ahead, steps per loop iteration (R % 4 == 0)

// Orders this wave's LDS accesses across lanes: a compiler barrier for memory operations (the
// LDS itself completes one wave's operations in program order).  Plain signal fences are not
// enough where the two sides use different vector types, which type-based alias analysis may
// then take as disjoint.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// element offset of 8-channel group g of staged pixel p (CG groups per pixel): 64-byte pixels
// swizzle their chunks on pixel bits 1-2, 32-byte pixels on bit 2
template <int CG>
__device__ inline int cs_off(int p, int g) {
  if constexpr (CG == 4) return p * 32 + ((g ^ ((p >> 1) & 3)) << 3);
  else return p * 16 + ((g ^ ((p >> 2) & 1)) << 3);
}

template <int CG, int HM>
__global__ __launch_bounds__(256) void k_conv_sweep(ConvArgs a, int R, int nseg, int nunit) {
  using T = uint16_t;
  constexpr int XR = kCsPix * CG * 8;          // elements of one ring row
  constexpr int XN = 4 * XR, ON = 2 * kCsCols * 32;
  // a row's staged logits [32 px][hldy <= 16 HM], then the head biases as floats (16 HM)
  constexpr int LN = HM ? kCsCols * 16 * HM + 32 * HM : 0;
  constexpr int NLD = (34 * CG + 63) / 64;     // 16-byte input loads per lane and row
  constexpr int D = HM ? 2 : kCsDepth;         // input rows in flight in registers
  __shared__ __attribute__((aligned(16))) T lds[4][XN + ON + LN];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int unit = blockIdx.x * 4 + wave, n = blockIdx.y;
  if (unit >= nunit) return;  // the whole wave; nothing below synchronises waves
  const int H = a.H, W = a.W;
  // 64 outputs: the two halves of a band segment go to neighbouring waves (units 2 k, 2 k + 1)
  const int mt0 = a.Cout == 64 ? 2 * (unit & 1) : 0, bs = a.Cout == 64 ? unit >> 1 : unit;
  const int x0 = (bs / nseg) * kCsCols, y0 = (bs % nseg) * R;
  T* X = lds[wave];
  T* O = X + XN;  // two output rows, [2][32 px][32 channels], chunks swizzled as cs_off<4>
  T* Ls = O + ON;
  for (int e = lane * 8; e < XN + ON; e += 512) zero8(X + e);

  // weights of the chunk layout: fragment (m-tile mt0 + m, tap), lane l = output channel
  // 16 (mt0 + m) + l % 16, input channels 8 (l / 16) .. + 7
  const T* wp = static_cast<const T*>(a.wp);
  Frag<T> w[2][9];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int t = 0; t < 9; ++t) frag_load(w[m][t], wp + ((size_t)((mt0 + m) * 9 + t) * 64 + lane) * 8);
  f32x4 bias[2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
    bias[m] = *reinterpret_cast<const f32x4*>(a.bias + 16 * (mt0 + m) + 4 * (lane >> 4));
  // fused 1x1 head (HM m-tiles of logits): the packed head weights of the one 32-channel chunk
  // and the head biases, as the tiled kernel's epilogue holds them
  // (biases in LDS, read per row, to keep the weights and the row prefetch in registers)
  Frag<T> hwf[HM ? HM : 1];
  float* Hb = reinterpret_cast<float*>(Ls + kCsCols * 16 * HM);
  if constexpr (HM != 0) {
    const T* hw = static_cast<const T*>(a.hw);
#pragma unroll
    for (int mh = 0; mh < HM; ++mh) {
      hwf[mh].v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (mh * 16 < a.hK) frag_load(hwf[mh], hw + ((size_t)mh * 64 + lane) * 8);
    }
    for (int k = lane; k < 16 * HM; k += 64) Hb[k] = k < a.hK ? a.hb[k] : 0.f;
  }
  // this lane's B operand offset within a ring row (n-tile s, tap column dx); groups beyond the
  // input channels read the zero pad
  int bo[2][3];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
      bo[s][dx] = (lane >> 4) < CG ? cs_off<CG>(16 * s + (lane & 15) + dx, lane >> 4) : cs_off<CG>(34, 0);
  // input rows: chunk c = lane + 64 k of the row is pixel c / CG (column x0 - 1 + c / CG), group c % CG
  const uint32_t img_bytes = (uint32_t)((size_t)H * W * a.Cx * sizeof(T));
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<T*>(static_cast<const T*>(a.x) + (size_t)n * H * W * a.Cx), 0, img_bytes, 0x00020000);
  auto load_row = [&](int iy, u16x8 (&v)[NLD]) {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int c = lane + 64 * k, px = c / CG, g = c % CG, xc = x0 - 1 + px;
      const bool in = c < 34 * CG && iy >= 0 && iy < H && xc >= 0 && xc < W;
      const uint32_t off = in ? (uint32_t)((((size_t)iy * W + xc) * a.Cx + g * 8) * sizeof(T)) : img_bytes;
      v[k] = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
    }
  };
  auto store_row = [&](T* dst, const u16x8 (&v)[NLD]) {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int c = lane + 64 * k;
      if (c < 34 * CG) *reinterpret_cast<u16x8*>(dst + cs_off<CG>(c / CG, c % CG)) = v[k];
    }
  };
  T* y = static_cast<T*>(a.y);
  T* yp = static_cast<T*>(a.pool);
  const int ylast = min(y0 + R, H) - 1;
  // emission of output row o from the accumulators acc[s][m]
  auto emit = [&](const f32x4 (&acc)[2][2], int o) {
    T* Ob = O + (o & 1) * (kCsCols * 32);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        s16x4 h = __builtin_bit_cast(s16x4, f2bf4(acc[s][m][0], acc[s][m][1], acc[s][m][2], acc[s][m][3]));
        if (a.relu) h = __builtin_elementwise_max(h, s16x4{0, 0, 0, 0});
        const int px = 16 * s + (lane & 15), co = 16 * m + 4 * (lane >> 4);
        *reinterpret_cast<s16x4*>(Ob + cs_off<4>(px, co >> 3) + (co & 7)) = h;
      }
    wave_lds_sync();  // other lanes' staged values are read below
    const size_t rowbase = ((size_t)n * H + o) * W;
    if (HM == 0 || a.store_main) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int q = lane + 64 * k, px = q >> 2, g = q & 3;
        if (x0 + px < W)
          *reinterpret_cast<u16x8*>(y + (rowbase + x0 + px) * a.ldy + 16 * mt0 + 8 * g) =
              *reinterpret_cast<const u16x8*>(Ob + cs_off<4>(px, g));
      }
    }
    if constexpr (HM != 0) {
      // the head on the staged (rounded, rectified) row: per 16-pixel n-tile one MFMA per head
      // m-tile, from zero, then the head bias, as the tiled epilogue and the stand-alone 1x1
      // convolution; logits staged as [px][hldy] (zeros in [hK, hldy)) and written as the row's
      // contiguous run, nontemporal (read back only by the filter, after the other heads)
      uint16_t* hy = static_cast<uint16_t*>(a.hy);
      const int hldy = a.hldy, npx = min(kCsCols, W - x0);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        Frag<T> b;
        frag_load(b, Ob + cs_off<4>(16 * s + (lane & 15), lane >> 4));
#pragma unroll
        for (int mh = 0; mh < HM; ++mh) {
          if (mh * 16 >= hldy) break;
          f32x4 h = f32x4{0.f, 0.f, 0.f, 0.f};
          if (mh * 16 < a.hK) h = mma(hwf[mh], b, h);
          const int k0 = mh * 16 + 4 * (lane >> 4);
          const f32x4 hb = *reinterpret_cast<const f32x4*>(Hb + k0);
          float v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = k0 + q < a.hK ? h[q] + hb[q] : 0.f;
          if (k0 < hldy) *reinterpret_cast<u16x4*>(Ls + (16 * s + (lane & 15)) * hldy + k0) = f2bf4(v[0], v[1], v[2], v[3]);
        }
      }
      wave_lds_sync();
      const int nvec = npx * hldy / 8;
      u32x4* dst = reinterpret_cast<u32x4*>(hy + (rowbase + x0) * hldy);
      for (int v = lane; v < nvec; v += 64)
        __builtin_nontemporal_store(__builtin_bit_cast(u32x4, *reinterpret_cast<const u16x8*>(Ls + 8 * v)), dst + v);
      if (a.hside && lane < npx) {
        const uint16_t* op = Ls + lane * hldy + a.hside_off;
        *reinterpret_cast<u16x4*>(static_cast<uint16_t*>(a.hside) + (rowbase + x0 + lane) * 4) =
            u16x4{op[0], op[1], op[2], (uint16_t)0};
      }
    }
    if (yp && ((o - y0) & 1)) {  // rows o - 1 and o: the 2x2 means of 16 pooled pixels
      const T* Oa = O + ((o - 1) & 1) * (kCsCols * 32);
      const int xp = lane >> 2, g = lane & 3;
      if (x0 + 2 * xp < W) {
        const u16x8 a0 = *reinterpret_cast<const u16x8*>(Oa + cs_off<4>(2 * xp, g));
        const u16x8 a1 = *reinterpret_cast<const u16x8*>(Oa + cs_off<4>(2 * xp + 1, g));
        const u16x8 b0 = *reinterpret_cast<const u16x8*>(Ob + cs_off<4>(2 * xp, g));
        const u16x8 b1 = *reinterpret_cast<const u16x8*>(Ob + cs_off<4>(2 * xp + 1, g));
        float r[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
          r[e] = ((bf2f(a0[e]) + bf2f(a1[e])) + (bf2f(b0[e]) + bf2f(b1[e]))) * 0.25f;
        const u16x4 lo = f2bf4(r[0], r[1], r[2], r[3]), hi = f2bf4(r[4], r[5], r[6], r[7]);
        *reinterpret_cast<u16x8*>(yp + (((size_t)n * (H / 2) + o / 2) * (W / 2) + (x0 / 2 + xp)) * a.Cout + 16 * mt0 + 8 * g) =
            u16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      }
    }
  };

  // ring row k (k = input row - (y0 - 1)) sits in slot k % 4; rows 0..2 are staged up front and
  // rows 3..2 + D wait in registers gx[k % D]
  {
    u16x8 v[NLD];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      load_row(y0 - 1 + k, v);
      store_row(X + k * XR, v);
    }
  }
  u16x8 gx[D][NLD];
#pragma unroll
  for (int k = 3; k < 3 + D; ++k) load_row(y0 - 1 + k, gx[k % D]);

  // step i: output row y0 + i from ring rows i, i + 1, i + 2; then ring row i + 3 is staged
  // (its slot held row i - 1, read by the previous step) and row i + 3 + D is requested
  auto step = [&](auto ph, int i) {
    constexpr int G = (decltype(ph)::value + 3) % D;  // == (i + 3) % D
    wave_lds_sync();
    f32x4 acc[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int m = 0; m < 2; ++m) acc[s][m] = bias[m];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      __builtin_amdgcn_sched_barrier(0);  // one tap column's operands live at a time
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const T* row = X + ((i + dy) & 3) * XR;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          Frag<T> b;
          frag_load(b, row + bo[s][dx]);
#pragma unroll
          for (int m = 0; m < 2; ++m) acc[s][m] = mma(w[m][3 * dy + dx], b, acc[s][m]);
        }
      }
    }
    wave_lds_sync();
    const int o = y0 + i;
    if (o <= ylast) emit(acc, o);
    store_row(X + ((i + 3) & 3) * XR, gx[G]);
    load_row(y0 + 2 + i + D, gx[G]);
  };
  static_assert(kCsDepth == 4 && 4 % D == 0, "four steps per iteration cycle the ring and gx");
  for (int i = 0; i < R; i += 4) {  // R % 4 == 0 (host)
    step(std::integral_constant<int, 0>{}, i);
    step(std::integral_constant<int, 1>{}, i + 1);
    step(std::integral_constant<int, 2>{}, i + 2);
    step(std::integral_constant<int, 3>{}, i + 3);
  }
}

// false: not this kernel's configuration: bf16 3x3 direct; 32 outputs from 16 or 32 inputs, or
// 64 outputs from 32 (each wave one half, its neighbour the other); with HM, the fused head (32
// inputs and outputs, logits staged: kstride <= 16 HM, 16-byte rows and base), no pool
template <int HM>
bool launch_conv_sweep(const ConvArgs& a, hipStream_t st) {
  if (a.mode != APS_CONV_DIRECT || a.C2 != 0 || a.nchunk != 1 || !a.bias ||
      !((a.Cout == 32 && (a.Cx == 16 || a.Cx == 32)) || (a.Cout == 64 && a.Cx == 32)))
    return false;
  if constexpr (HM == 0) {
    if (a.hw || a.hside || a.ldy != a.Cout) return false;
    if (a.pool && (a.H % 2 || a.W % 2)) return false;
  } else {
    if (a.Cx != 32 || a.Cout != 32 || a.pool || !a.hw || !a.hb || !a.hy || a.hK > 16 * HM ||
        a.hldy > 16 * HM || (a.hldy * 2) % 16 || (reinterpret_cast<uintptr_t>(a.hy) & 15) ||
        (a.hside && (reinterpret_cast<uintptr_t>(a.hside) & 7)) || (a.store_main && a.ldy != 32))
      return false;
  }
  if ((size_t)a.H * a.W * a.Cx * 2 >= (1ull << 31) || a.N > 65535) return false;
  const long nband = (a.W + kCsCols - 1) / kCsCols, halves = a.Cout / 32;
  // rows per wave: a multiple of the prefetch depth (even, so pooled rows pair up in a segment)
  long R = std::max<long>(8, ((long)a.N * a.H * nband * halves + kCsWaves - 1) / kCsWaves);
  R = (std::min<long>(R, a.H) + kCsDepth - 1) / kCsDepth * kCsDepth;
  const int nseg = (int)((a.H + R - 1) / R);
  const long nunit = nband * nseg * halves;
  if (nunit > (1L << 30) / 4) return false;
  dim3 g((unsigned)((nunit + 3) / 4), a.N);
  if constexpr (HM == 0) {
    if (a.Cx == 32) k_conv_sweep<4, 0><<<g, 256, 0, st>>>(a, (int)R, nseg, (int)nunit);
    else k_conv_sweep<2, 0><<<g, 256, 0, st>>>(a, (int)R, nseg, (int)nunit);
  } else {
    k_conv_sweep<4, HM><<<g, 256, 0, st>>>(a, (int)R, nseg, (int)nunit);
  }
  return true;
}

// ---- fp32 form of the row sweep ------------------------------------------------------------
// The same per-wave sweep for the fp32 networks' 32-channel full-resolution layers (16 or 32
// input channels, 32 outputs, no head) and the half-resolution 32 -> 64 layer.  On the tiled fp32
// kernel these run at 57-70 % of the MFMA peak against 81-87 % for the wider layers, each block
// computing two 16-channel chunks at most for one staged tile.  Here the weights (9 taps x CH
// chunks of 16 channels for MS m-tiles: both with 16 input channels; with 32 one per wave, its
// neighbour waves taking the others, so that two waves fit a SIMD) stay in registers and each
// input row is read from HBM once per band into a ring of three LDS rows, each held as CH planes
// of [36 px][20 floats] (the tiled kernel's 80-byte pixel pitch, so the 16 lanes of a B read hit
// distinct banks).  Output row o is summed in the tiled kernel's order: 16-channel chunks outer,
// then taps dx, dy, four K = 4 MFMAs per tap, from the bias; so the two kernels give the same
// bits.  Epilogue as lds_epilogue_f32: ReLU, 16-byte stores per lane, and with a pooled output
// the 2x2 mean of the previous and the current row (neighbour column by DPP) in the POOL2 order.
// Ring row i + 3 is staged into the slot of row i after this step's reads of it (one wave's LDS
// operations complete in program order).
constexpr int kCsfPS = 20;       // floats per staged pixel of a 16-channel plane

template <int CH, int MS>
__global__ __launch_bounds__(256) void k_conv_sweep_f32(ConvArgs a, int R, int nseg, int nunit) {
  constexpr int PL = kCsPix * kCsfPS;           // floats of one plane of a ring row
  constexpr int XR = CH * PL, XN = 3 * XR;      // ring of three rows
  constexpr int NU = 34 * CH * 4;               // 16-byte units of an input row (34 pixels)
  constexpr int NLD = (NU + 63) / 64;
  constexpr int D = 2;                          // input rows in flight in registers
  __shared__ __attribute__((aligned(16))) float lds[4][XN];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int unit = blockIdx.x * 4 + wave, n = blockIdx.y;
  if (unit >= nunit) return;  // the whole wave; nothing below synchronises waves
  const int H = a.H, W = a.W, Cx = a.Cx;
  // MS = 1: the Cout / 16 m-tiles of a band segment go to neighbouring waves
  const int nm = a.Cout >> 4;
  const int mt0 = MS == 2 ? 0 : unit % nm, bs = MS == 2 ? unit : unit / nm;
  const int x0 = (bs / nseg) * kCsCols, y0 = (bs % nseg) * R;
  float* X = lds[wave];
  for (int e = lane * 4; e < XN; e += 256) *reinterpret_cast<f32x4*>(X + e) = f32x4{0.f, 0.f, 0.f, 0.f};

  // weights (16-channel chunk packing): fragment (m, tap, chunk c), lane l = output channel
  // 16 m + l % 16, input channels 16 c + 4 (l / 16) + [0, 4)
  const float* wp = static_cast<const float*>(a.wp);
  f32x4 w[MS][9][CH];
#pragma unroll
  for (int m = 0; m < MS; ++m)
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int c = 0; c < CH; ++c)
        w[m][t][c] = *reinterpret_cast<const f32x4*>(wp + ((size_t)(((mt0 + m) * 9 + t) * CH + c) * 64 + lane) * 4);
  f32x4 bias[MS];
#pragma unroll
  for (int m = 0; m < MS; ++m) bias[m] = *reinterpret_cast<const f32x4*>(a.bias + 16 * (mt0 + m) + 4 * (lane >> 4));
  int bo[2][3];  // B read offsets within a plane: pixel 16 s + l % 16 + dx, channels 4 (l / 16)
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) bo[s][dx] = (16 * s + (lane & 15) + dx) * kCsfPS + 4 * (lane >> 4);

  // input rows: unit u = lane + 64 k is pixel u / (4 CH) (column x0 - 1 + u / (4 CH)), chunk
  // (u % (4 CH)) / 4, channels 4 (u % 4) .. + 3 of it
  const uint32_t img_bytes = (uint32_t)((size_t)H * W * Cx * sizeof(float));
  const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(static_cast<const float*>(a.x) + (size_t)n * H * W * Cx), 0, img_bytes, 0x00020000);
  auto load_row = [&](int iy, f32x4 (&v)[NLD]) {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int u = lane + 64 * k, px = u / (4 * CH), xc = x0 - 1 + px;
      const bool in = u < NU && iy >= 0 && iy < H && xc >= 0 && xc < W;
      const uint32_t off = in ? (uint32_t)((((size_t)iy * W + xc) * Cx + 4 * (u % (4 * CH))) * sizeof(float)) : img_bytes;
      v[k] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
    }
  };
  auto store_row = [&](float* dst, const f32x4 (&v)[NLD]) {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int u = lane + 64 * k, px = u / (4 * CH), wv = u % (4 * CH);
      if (u < NU) *reinterpret_cast<f32x4*>(dst + (wv >> 2) * PL + px * kCsfPS + 4 * (wv & 3)) = v[k];
    }
  };
  float* y = static_cast<float*>(a.y);
  float* yp = static_cast<float*>(a.pool);
  const int ylast = min(y0 + R, H) - 1;
  f32x4 hprev[2][MS];  // the previous (even) row's outputs, for the pooled copy
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int m = 0; m < MS; ++m) hprev[s][m] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto emit = [&](const f32x4 (&acc)[2][MS], int o) {
    const bool second = (o - y0) & 1;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int col = x0 + 16 * s + (lane & 15);
#pragma unroll
      for (int m = 0; m < MS; ++m) {
        const int co = 16 * (mt0 + m) + 4 * (lane >> 4);
        f32x4 v = acc[s][m];
        if (a.relu) {
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = fmaxf(v[q], 0.f);
        }
        if (col < W) *reinterpret_cast<f32x4*>(y + (((size_t)n * H + o) * W + col) * a.ldy + co) = v;
        if (yp) {
          if (second) {
            f32x4 nb0, nb1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              nb0[q] = lane_xor1(hprev[s][m][q]);
              nb1[q] = lane_xor1(v[q]);
            }
            if ((lane & 1) == 0 && col < W)
              *reinterpret_cast<f32x4*>(yp + (((size_t)n * (H / 2) + o / 2) * (W / 2) + col / 2) * a.Cout + co) =
                  ((hprev[s][m] + nb0) + (v + nb1)) * 0.25f;
          } else {
            hprev[s][m] = v;
          }
        }
      }
    }
  };

  // ring row k (input row y0 - 1 + k) sits in slot k % 3; rows 0..2 are staged up front and rows
  // 3, 4 wait in registers gx[k % 2]
  {
    f32x4 v[NLD];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      load_row(y0 - 1 + k, v);
      store_row(X + k * XR, v);
    }
  }
  f32x4 gx[D][NLD];
#pragma unroll
  for (int k = 3; k < 3 + D; ++k) load_row(y0 - 1 + k, gx[k % D]);

  int s0 = 0;  // slot of ring row i
  auto step = [&](auto ph, int i) {
    constexpr int G = (decltype(ph)::value + 3) % D;  // == (i + 3) % D
    const int s1 = s0 == 2 ? 0 : s0 + 1, s2 = s1 == 2 ? 0 : s1 + 1;
    const float* rows[3] = {X + s0 * XR, X + s1 * XR, X + s2 * XR};
    wave_lds_sync();
    f32x4 acc[2][MS];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int m = 0; m < MS; ++m) acc[s][m] = bias[m];
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        __builtin_amdgcn_sched_barrier(0);  // one tap column's operands live at a time
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const f32x4 b = *reinterpret_cast<const f32x4*>(rows[dy] + c * PL + bo[s][dx]);
#pragma unroll
            for (int m = 0; m < MS; ++m) acc[s][m] = mma4(w[m][3 * dy + dx][c], b, acc[s][m]);
          }
      }
    wave_lds_sync();
    const int o = y0 + i;
    if (o <= ylast) emit(acc, o);
    store_row(X + s0 * XR, gx[G]);  // ring row i + 3 into the slot of row i
    load_row(y0 + 2 + i + D, gx[G]);
    s0 = s1;
  };
  for (int i = 0; i < R; i += 4) {  // R % 4 == 0 (host)
    step(std::integral_constant<int, 0>{}, i);
    step(std::integral_constant<int, 1>{}, i + 1);
    step(std::integral_constant<int, 2>{}, i + 2);
    step(std::integral_constant<int, 3>{}, i + 3);
  }
}

// false: not this kernel's configuration (fp32 3x3 direct, no head: 32 outputs from 16 or 32
// inputs, 64 from 32)
bool launch_conv_sweep_f32(const ConvArgs& a, hipStream_t st) {
  if (a.mode != APS_CONV_DIRECT || a.C2 != 0 || a.ldy != a.Cout || a.hw || a.hside || !a.bias ||
      !((a.Cout == 32 && (a.Cx == 16 || a.Cx == 32)) || (a.Cout == 64 && a.Cx == 32)))
    return false;
  if (a.pool && (a.H % 2 || a.W % 2)) return false;
  if ((size_t)a.H * a.W * a.Cx * 4 >= (1ull << 31) || a.N > 65535) return false;
  const long nband = (a.W + kCsCols - 1) / kCsCols;
  // with 32 input channels each wave takes one m-tile (the weights of two would leave one wave
  // per SIMD), its neighbours the others; the launch aims at about 2048 waves, two per SIMD
  const int wps = a.Cx == 32 ? a.Cout / 16 : 1;  // waves per band segment
  long R = std::max<long>(8, ((long)a.N * a.H * nband * wps + 2047) / 2048);
  R = (std::min<long>(R, a.H) + 3) / 4 * 4;  // four steps per loop iteration
  const int nseg = (int)((a.H + R - 1) / R);
  const long nunit = nband * nseg * wps;
  if (nunit > (1L << 30) / 4) return false;
  dim3 g((unsigned)((nunit + 3) / 4), a.N);
  if (a.Cx == 32) k_conv_sweep_f32<2, 1><<<g, 256, 0, st>>>(a, (int)R, nseg, (int)nunit);
  else k_conv_sweep_f32<1, 2><<<g, 256, 0, st>>>(a, (int)R, nseg, (int)nunit);
  return true;
}

// false: the configuration is not covered (the caller uses k_conv)
template <int HEAD>
bool launch_conv_lds(const ConvArgs& a, hipStream_t st) {
  if (a.Cout <= 16 || a.Cout % 16 || a.ldy % 4) return false;
  // the kernel addresses its inputs with 32-bit element offsets
  const size_t px = (size_t)a.N * a.H * a.W;
  const size_t ex = a.mode == APS_CONV_POOL2 ? 4 * px * a.Cx
                    : a.mode == APS_CONV_UP2_CAT ? px / 4 * a.Cx : px * a.Cx;
  const size_t e2 = a.mode == APS_CONV_UP2_CAT ? px * a.C2 : 0;
  if ((ex > e2 ? ex : e2) + kChunk >= ((size_t)1 << 31)) return false;
  if constexpr (HEAD) {
    if (a.mode != APS_CONV_DIRECT) return false;
    if (launch_conv_sweep<HEAD>(a, st)) return true;
    launch_conv_lds_m<APS_CONV_DIRECT, HEAD>(a, st);
    return true;
  } else {
    if (launch_conv_sweep<0>(a, st)) return true;
    switch (a.mode) {
      case APS_CONV_DIRECT: launch_conv_lds_m<APS_CONV_DIRECT, 0>(a, st); return true;
      case APS_CONV_POOL2: launch_conv_lds_m<APS_CONV_POOL2, 0>(a, st); return true;
      case APS_CONV_UP2_CAT: launch_conv_lds_m<APS_CONV_UP2_CAT, 0>(a, st); return true;
      case kModeReluMask: launch_conv_lds_m<kModeReluMask, 0>(a, st); return true;
      default: return false;
    }
  }
}

// ---- weight packing: OHWI fp32 -> fragment order --------------------------------------
// packed[(((ct * KS*KS + tap) * nchunk + c) * 64 + lane) * 8 + e] =
//     w[co = 16 ct + lane % 16][tap][ci = 32 c + 8 (lane / 16) + e]   (0 outside)
// transpose = 1 packs the data-gradient operator of w: a conv with Cout' = Cin, Cin' = Cout and
//     w'[co'][tap][ci'] = w[ci'][KS*KS - 1 - tap][co']   (channels swapped, taps flipped).
template <typename T>
__global__ void k_pack(const float* __restrict__ w, int Cout, int KS, int Cin, int nchunk,
                       size_t total, T* __restrict__ out, int transpose, int cg) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
  size_t r = i >> 9;
  int ct, tap, ci;
  bool ok = true;
  if (cg < 4) {  // merged (tap, group) pairs: step s, lane group q -> pair 4 s + q
    const int npair = KS * KS * cg, steps = (npair + 3) / 4;
    const int st = (int)(r % steps);
    ct = (int)(r / steps);
    const int p = 4 * st + (lane >> 4);
    ok = p < npair;
    tap = ok ? p / cg : 0;
    ci = (ok ? p % cg : 0) * 8 + e;
  } else {
    const int c = (int)(r % nchunk);
    r /= nchunk;
    tap = (int)(r % (KS * KS));
    ct = (int)(r / (KS * KS));
    ci = c * kChunk + (lane >> 4) * 8 + e;
  }
  const int co = ct * 16 + (lane & 15);
  float v = 0.f;
  if (ok && co < Cout && ci < Cin)
    v = transpose ? w[((size_t)ci * KS * KS + (KS * KS - 1 - tap)) * Cout + co]
                  : w[((size_t)co * KS * KS + tap) * Cin + ci];
  if constexpr (sizeof(T) == 2) out[i] = f2bf(v);
  else out[i] = v;
}

// fp32 3x3 layers with more than 16 input channels (the operand of k_conv_lds_f32), in chunks of
// 16 channels with 4 per lane:
// packed[(((ct * 9 + tap) * nchunk16 + c) * 64 + lane) * 4 + e] =
//     w[co = 16 ct + lane % 16][tap][ci = 16 c + 4 (lane / 16) + e]   (0 outside)
// (transpose as in k_pack).
__global__ void k_pack_f32c16(const float* __restrict__ w, int Cout, int Cin, int nchunk16,
                              size_t total, float* __restrict__ out, int transpose) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int e = (int)(i & 3), lane = (int)((i >> 2) & 63);
  size_t r = i >> 8;
  const int c = (int)(r % nchunk16);
  r /= nchunk16;
  const int tap = (int)(r % 9), ct = (int)(r / 9);
  const int co = ct * 16 + (lane & 15), ci = c * 16 + (lane >> 4) * 4 + e;
  float v = 0.f;
  if (co < Cout && ci < Cin)
    v = transpose ? w[((size_t)ci * 9 + (8 - tap)) * Cout + co] : w[((size_t)co * 9 + tap) * Cin + ci];
  out[i] = v;
}

// fp32 3x3 convolutions with more than 16 input channels run only in k_conv_lds_f32, which
// addresses its inputs with 32-bit element offsets
bool fp32_offsets_fit(int mode, int N, int H, int W, int Cx, int C2) {
  const size_t px = (size_t)N * H * W;
  const size_t ex = mode == APS_CONV_POOL2 ? 4 * px * Cx : mode == APS_CONV_UP2_CAT ? px / 4 * Cx : px * Cx;
  const size_t e2 = mode == APS_CONV_UP2_CAT ? px * C2 : 0;
  return (ex > e2 ? ex : e2) + 16 < ((size_t)1 << 31);
}

// 8-channel groups of the K layout (see k_conv).  4: 32-channel chunks (fp32: the 16-channel
// chunks of k_conv_lds_f32), for 1x1 convolutions, 3x3 with more than 16 input channels, and
// 3x3 with 9..16 input channels whose output channels fill whole 16-channel tiles beyond 16 (the
// U-Net's first layer: it runs in the LDS kernels, in bf16 as one half-filled chunk).  1 or 2:
// merged (tap, group) pairs for the other 3x3 layers with <= 16 input channels (the sampler).
int conv_cg(int KS, int Cin, int Cout) {
  if (KS != 3) return 4;
  const int g = (Cin + 7) / 8;
  if (g == 2 && Cout > 16 && Cout % 16 == 0) return 4;
  return g <= 1 ? 1 : (g <= 2 ? 2 : 4);
}

size_t packed_elems(int Cout, int KS, int Cin) {
  const size_t nct = (size_t)((Cout + 16 * kMaxTM - 1) / (16 * kMaxTM)) * kMaxTM;
  const int cg = conv_cg(KS, Cin, Cout);
  if (cg < 4) return nct * ((KS * KS * cg + 3) / 4) * 512;
  const size_t nchunk = (size_t)(Cin + kChunk - 1) / kChunk;
  return nct * KS * KS * nchunk * 512;
}

template <typename T, typename TO, int KS, int TM, int TN, int CG>
void launch_conv(const ConvArgs& a, hipStream_t st) {
  const int TH = 4 * TN;
  const int ntx = (a.W + 15) / 16, nty = (a.H + TH - 1) / TH;
  ConvArgs b = a;
  b.ntx = ntx;
  b.ntiles = ntx * nty;
  b.nco = (a.Cout + 16 * TM - 1) / (16 * TM);
  dim3 grid(xcd_grid(b.ntiles, b.nco), 1, a.N);
  k_conv<T, TO, KS, TM, TN, CG><<<grid, 256, 0, st>>>(b);
}

// 3x3 conv (Cout = 16 TM, one block covers all of it) with its 1x1 head of HM m-tiles in the
// epilogue.
template <typename T, int TM, int HM>
void launch_conv_head_hm(const ConvArgs& a, hipStream_t st) {
  if constexpr (sizeof(T) == 2) {
    if (launch_conv_lds<HM>(a, st)) return;
  } else {
    if (launch_conv_lds_f32<HM>(a, st)) return;
  }
  const bool big = (size_t)a.H * a.W >= 64 * 64;
  const int TN = big ? 4 : 2, TH = 4 * TN;
  ConvArgs b = a;
  b.ntx = (a.W + 15) / 16;
  b.ntiles = b.ntx * ((a.H + TH - 1) / TH);
  b.nco = 1;
  dim3 grid(xcd_grid(b.ntiles, 1), 1, a.N);
  if (big) k_conv<T, T, 3, TM, 4, 4, HM><<<grid, 256, 0, st>>>(b);
  else k_conv<T, T, 3, TM, 2, 4, HM><<<grid, 256, 0, st>>>(b);
}

// heads of up to 64 logits keep the four-m-tile epilogue (fewer registers); 65..80 take five
template <typename T, int TM>
void launch_conv_head(const ConvArgs& a, hipStream_t st) {
  if (a.hK > 64) launch_conv_head_hm<T, TM, 5>(a, st);
  else launch_conv_head_hm<T, TM, 4>(a, st);
}

// ---- 1x1 convolution for the logit heads -------------------------------------------------------
// One wave per 16 consecutive output pixels and all MT m-tiles (Cout <= 16 MT); no LDS and no
// barriers: each lane loads its B fragments straight from global memory (pixel lane % 16,
// channels 32 c + 8 (lane / 16) + [0, 8) of chunk c, zero past Cin), the A fragments are the
// packed weights (L2-resident).  The heads at the coarse levels have few pixels, so the tiled
// kernel's block-wide chunk loop (stage, barrier, MFMAs, barrier) left most of the chip idle
// and serialised one memory round trip per chunk.  The MFMA sequence and the POOL2 transform
// (2x2 mean of the inputs in fp32, rounded to T) are those of k_conv, so the results are the same
// bit for bit.
template <typename T, typename TO, int MT, bool POOL>
__global__ __launch_bounds__(256) void k_conv1x1(ConvArgs a) {
  constexpr int MAXC = 8;  // Cin <= 256
  const int lane = threadIdx.x & 63;
  const size_t npix = (size_t)a.N * a.H * a.W;
  const size_t p0 = ((size_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (p0 >= npix) return;  // whole waves
  const size_t pix = p0 + (lane & 15);
  const bool inpx = pix < npix;
  const size_t pc = inpx ? pix : p0;  // a valid pixel for the loads of lanes past the end
  const int g8 = 8 * (lane >> 4);
  const T* x = static_cast<const T*>(a.x);
  const T* wp = static_cast<const T*>(a.wp);
  size_t xo;
  if constexpr (POOL) {
    const size_t hw = (size_t)a.H * a.W, n = pc / hw, r = pc - n * hw;
    const size_t yy = r / a.W, xx = r - yy * a.W;
    xo = ((n * 2 * a.H + 2 * yy) * (2 * (size_t)a.W) + 2 * xx) * a.Cx;
  } else {
    xo = pc * a.Cx;
  }
  Frag<T> b[MAXC];
#pragma unroll
  for (int c = 0; c < MAXC; ++c) {
    if (c >= a.nchunk) break;
    const int ci = c * kChunk + g8;
    const bool ok = inpx && ci < a.Cx;
    const size_t o = xo + (ok ? ci : 0);
    if constexpr (POOL) {
      const size_t rs = 2 * (size_t)a.W * a.Cx;
      const V8f q0 = load8(x + o), q1 = load8(x + o + a.Cx), q2 = load8(x + o + rs),
                q3 = load8(x + o + rs + a.Cx);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float r = ((q0.v[e] + q1.v[e]) + (q2.v[e] + q3.v[e])) * 0.25f;
        if constexpr (sizeof(T) == 2) b[c].v[e] = ok ? f2bf(r) : (uint16_t)0;
        else b[c].v[e] = ok ? r : 0.f;
      }
    } else if constexpr (sizeof(T) == 2) {
      const u16x8 v = *reinterpret_cast<const u16x8*>(x + o);
#pragma unroll
      for (int e = 0; e < 8; ++e) b[c].v[e] = ok ? v[e] : (uint16_t)0;
    } else {
      const V8f v = load8(x + o);
#pragma unroll
      for (int e = 0; e < 8; ++e) b[c].v[e] = ok ? v.v[e] : 0.f;
    }
  }
  f32x4 acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < MAXC; ++c) {
    if (c >= a.nchunk) break;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      Frag<T> w;
      frag_load(w, wp + (((size_t)m * a.nchunk + c) * 64 + lane) * 8);
      acc[m] = mma(w, b[c], acc[m]);
    }
  }
  if (!inpx) return;
  TO* py = static_cast<TO*>(a.y) + pix * a.ldy;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int co0 = m * 16 + 4 * (lane >> 4);
    if (co0 >= a.Cout) continue;
    float v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // no bias for the input-gradient convolutions (aps_conv2d_bwd_data passes none)
      const float t = acc[m][q] + (a.bias && co0 + q < a.Cout ? a.bias[co0 + q] : 0.f);
      v[q] = a.relu ? fmaxf(t, 0.f) : t;
    }
    store_out<TO>(py, a.ldy, co0, a.Cout, v);
  }
}

// false: not covered (the caller uses k_conv)
template <typename T, typename TO>
bool launch_conv1x1(const ConvArgs& a, hipStream_t st) {
  if (a.C2 != 0 || a.Cx % 8 || a.nchunk > 8 || a.Cout > 80) return false;
  if (a.mode != APS_CONV_DIRECT && a.mode != APS_CONV_POOL2) return false;
  const size_t npix = (size_t)a.N * a.H * a.W;
  const size_t blocks = (npix + 63) / 64;
  if (blocks > 0x7fffffff) return false;
  const dim3 grid((unsigned)blocks);
  const int mt = (a.Cout + 15) / 16;
  const bool pool = a.mode == APS_CONV_POOL2;
#define APS_C1X1(MT)                                                          \
  if (pool) k_conv1x1<T, TO, MT, true><<<grid, 256, 0, st>>>(a);              \
  else k_conv1x1<T, TO, MT, false><<<grid, 256, 0, st>>>(a);
  if (mt == 1) { APS_C1X1(1) }
  else if (mt == 2) { APS_C1X1(2) }
  else if (mt == 3) { APS_C1X1(3) }
  else if (mt == 4) { APS_C1X1(4) }
  else { APS_C1X1(5) }
#undef APS_C1X1
  return true;
}

template <typename T, typename TO, int KS, int CG>
void dispatch_tiles(const ConvArgs& a, hipStream_t st) {
  if constexpr (KS == 1) {
    if (launch_conv1x1<T, TO>(a, st)) return;
  }
  if constexpr (sizeof(T) == 2 && sizeof(TO) == 2 && KS == 3 && CG == 4) {
    if (launch_conv_lds<false>(a, st)) return;
  }
  if constexpr (sizeof(T) == 4 && KS == 3 && CG == 4) {
    launch_conv_lds_f32<false>(a, st);  // sizes checked by the entry points (fp32_offsets_fit)
    return;
  }
  const bool big = (size_t)a.H * a.W >= 64 * 64;
  if (a.Cout <= 16) {
    if (big) launch_conv<T, TO, KS, 1, 4, CG>(a, st); else launch_conv<T, TO, KS, 1, 2, CG>(a, st);
  } else if (a.Cout <= 32) {
    if (big) launch_conv<T, TO, KS, 2, 4, CG>(a, st); else launch_conv<T, TO, KS, 2, 2, CG>(a, st);
  } else {
    if (big) launch_conv<T, TO, KS, 4, 4, CG>(a, st); else launch_conv<T, TO, KS, 4, 2, CG>(a, st);
  }
}

template <typename T, typename TO>
void dispatch_ks(const ConvArgs& a, int KS, hipStream_t st) {
  if (KS == 3) {
    const int cg = conv_cg(3, a.Cx + a.C2, a.Cout);
    if (cg == 1) dispatch_tiles<T, TO, 3, 1>(a, st);
    else if (cg == 2) dispatch_tiles<T, TO, 3, 2>(a, st);
    else dispatch_tiles<T, TO, 3, 4>(a, st);
  } else {
    dispatch_tiles<T, TO, 1, 4>(a, st);
  }
}

// ======================================================================== backward
// ---- data gradient: transposes of the fused input transforms ----------------------------
// POOL2:    dx[n][2y+a][2x+b][c] (+)= dX[n][y][x][c] / 4
// UP2_CAT:  dx[n][Y][X][c] (+)= sum_{a,b} dX[n][2Y+a][2X+b][c] (c < Cx);
//           dx2[n][y][x][c] (+)= dX[n][y][x][Cx + c]
// DIRECT:   dx (+)= dX
template <typename T>
__global__ __launch_bounds__(256) void k_input_grad(int mode, const T* __restrict__ dX, int N,
                                                    int H, int W, int Cx, int C2,
                                                    T* __restrict__ dx, int acc, T* __restrict__ dx2,
                                                    int acc2) {
  const int Cin = Cx + C2;
  size_t total;
  if (mode == APS_CONV_POOL2) total = (size_t)N * 2 * H * 2 * W * Cx;
  else if (mode == APS_CONV_UP2_CAT) total = (size_t)N * (H / 2) * (W / 2) * Cx + (size_t)N * H * W * C2;
  else total = (size_t)N * H * W * Cx;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  if (mode == APS_CONV_POOL2) {
    const int c = (int)(i % Cx);
    const size_t pf = i / Cx;
    const int xf = (int)(pf % (2 * W)), yf = (int)((pf / (2 * W)) % (2 * H)), n = (int)(pf / ((size_t)4 * H * W));
    const float v = 0.25f * Ld<T>::get(dX, (((size_t)n * H + yf / 2) * W + xf / 2) * Cin + c);
    dx[i] = f2t<T>(acc ? Ld<T>::get(dx, i) + v : v);
  } else if (mode == APS_CONV_UP2_CAT) {
    const size_t n1 = (size_t)N * (H / 2) * (W / 2) * Cx;
    if (i < n1) {
      const int c = (int)(i % Cx);
      const size_t pc = i / Cx;
      const int Wh = W / 2, Hh = H / 2;
      const int X = (int)(pc % Wh), Y = (int)((pc / Wh) % Hh), n = (int)(pc / ((size_t)Wh * Hh));
      float v = 0.f;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          v += Ld<T>::get(dX, (((size_t)n * H + 2 * Y + a) * W + 2 * X + b) * Cin + c);
      dx[i] = f2t<T>(acc ? Ld<T>::get(dx, i) + v : v);
    } else {
      const size_t k = i - n1;
      const int c = (int)(k % C2);
      const size_t p = k / C2;
      const float v = Ld<T>::get(dX, p * Cin + Cx + c);
      dx2[k] = f2t<T>(acc2 ? Ld<T>::get(dx2, k) + v : v);
    }
  } else {
    const float v = Ld<T>::get(dX, i);
    dx[i] = f2t<T>(acc ? Ld<T>::get(dx, i) + v : v);
  }
}

// ---- weight gradient: dW[co][tap][ci] = sum_px dY[px][co] * X[px + d_tap][ci] -------------
// M = cout (16 per MFMA tile), N = cin (16), K = pixels: 2-row x 64-column pixel blocks, the
// block's dY (cout-major) and its input tile with halo (cin-major) staged in LDS.  Pixel blocks
// are split across workgroups; each split writes its partial dW and a second pass sums the
// splits in a fixed order (deterministic).
constexpr int kWgRows = 2, kWgCols = 64;

struct WgradArgs {
  ConvArgs in;          // the forward input (x, x2, N, H, W, Cx, C2, mode)
  const void* dy;       // [N, H, W, ldy]
  const void* ymask;    // post-ReLU output [N, H, W, Cout] or null
  int ldy, Cout, nchunk;
  int nrb, ncb, nblocks, bps;
  int CoutP, CinP;
  float* part;          // [splits][CoutP][KS*KS][CinP]
};

template <typename T>
__device__ inline void frag_load_lds(Frag<T>& f, const T* p);
template <>
__device__ inline void frag_load_lds<float>(Frag<float>& f, const float* p) {
#pragma unroll
  for (int e = 0; e < 8; ++e) f.v[e] = p[e];
}
template <>
__device__ inline void frag_load_lds<uint16_t>(Frag<uint16_t>& f, const uint16_t* p) {
#pragma unroll
  for (int e = 0; e < 8; ++e) f.v[e] = p[e];
}

template <typename T, int KS>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
  constexpr int R = KS / 2;
  constexpr int NP = kWgRows * kWgCols;
  constexpr int XW = kWgCols + 2 * R, XH = kWgRows + 2 * R;
  constexpr int YS = NP + 8;        // per-cout row of dY (elements)
  constexpr int XS = XH * XW + 8;   // per-cin plane of X (elements)
  __shared__ __attribute__((aligned(16))) T dYs[32 * YS];
  __shared__ __attribute__((aligned(16))) T Xs[32 * XS];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int split = blockIdx.x, cot = blockIdx.y, c = blockIdx.z;
  const int m = wave & 1, j = wave >> 1;
  const int H = a.in.H, W = a.in.W;
  const T* dy = static_cast<const T*>(a.dy);
  const T* ym = static_cast<const T*>(a.ymask);

  f32x4 acc[KS * KS];
#pragma unroll
  for (int t = 0; t < KS * KS; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int b1 = min(a.nblocks, (split + 1) * a.bps);
  for (int blk = split * a.bps; blk < b1; ++blk) {
    const int n = blk / (a.nrb * a.ncb), rb = (blk / a.ncb) % a.nrb, cb = blk % a.ncb;
    const int y0 = rb * kWgRows, x0 = cb * kWgCols;
    for (int it = tid; it < NP * 4; it += 256) {
      const int g = it & 3, p = it >> 2;
      const int py = y0 + p / kWgCols, px = x0 + p % kWgCols;
      const int co = cot * 32 + g * 8;
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = 0.f;
      if (py < H && px < W) {
        const size_t pix = ((size_t)n * H + py) * W + px;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (co + e < a.Cout) {
            float g_ = Ld<T>::get(dy, pix * a.ldy + co + e);
            if (ym && !(Ld<T>::get(ym, pix * a.Cout + co + e) > 0.f)) g_ = 0.f;
            v[e] = g_;
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) dYs[(g * 8 + e) * YS + p] = f2t<T>(v[e]);
    }
    for (int it = tid; it < XH * XW * 4; it += 256) {
      const int g = it & 3, p = it >> 2;
      const int r = p / XW, col = p % XW;
      T tmp[8];
      stage8<T>(a.in, n, y0 - R + r, x0 - R + col, c * kChunk + g * 8, tmp);
#pragma unroll
      for (int e = 0; e < 8; ++e) Xs[(g * 8 + e) * XS + p] = tmp[e];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kWgRows; ++r) {
#pragma unroll
      for (int s = 0; s < kWgCols / 32; ++s) {
        Frag<T> af;
        frag_load_lds(af, dYs + (m * 16 + (lane & 15)) * YS + r * kWgCols + 32 * s + 8 * (lane >> 4));
#pragma unroll
        for (int tap = 0; tap < KS * KS; ++tap) {
          const int dyy = tap / KS - R, dxx = tap % KS - R;
          Frag<T> bf;
          frag_load_lds(bf, Xs + (j * 16 + (lane & 15)) * XS + (r + R + dyy) * XW +
                                (32 * s + 8 * (lane >> 4) + R + dxx));
          acc[tap] = mma(af, bf, acc[tap]);
        }
      }
    }
    __syncthreads();
  }
  const int ci = c * kChunk + j * 16 + (lane & 15);
#pragma unroll
  for (int tap = 0; tap < KS * KS; ++tap)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int co = cot * 32 + m * 16 + 4 * (lane >> 4) + q;
      a.part[(((size_t)split * a.CoutP + co) * KS * KS + tap) * a.CinP + ci] = acc[tap][q];
    }
}

// The splits of 32 consecutive dW entries per block: split lane r = t / 32 (8 lanes) sums the
// splits k = r, r + 8, ... in order into two accumulators (k / 8 even and odd), then lane 0 of
// each entry adds the eight lane sums in lane order: a fixed order, eight times the
// parallelism of one thread per entry.
constexpr int kRedLanes = 8;
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int splits,
                                                      int Cout, int KK, int Cin, int CoutP,
                                                      int CinP, float* __restrict__ dw) {
  __shared__ float red[kRedLanes][32];
  const int t = threadIdx.x, e = t & 31, r = t >> 5;
  const size_t i = (size_t)blockIdx.x * 32 + e;
  const bool ok = i < (size_t)Cout * KK * Cin;
  float s0 = 0.f, s1 = 0.f;
  if (ok) {
    const int ci = (int)(i % Cin);
    const int tap = (int)((i / Cin) % KK);
    const int co = (int)(i / ((size_t)Cin * KK));
    const size_t stride = (size_t)CoutP * KK * CinP;
    const float* pp = part + ((size_t)co * KK + tap) * CinP + ci;
    int k = r;
    for (; k + kRedLanes < splits; k += 2 * kRedLanes) {
      s0 += pp[(size_t)k * stride];
      s1 += pp[(size_t)(k + kRedLanes) * stride];
    }
    if (k < splits) s0 += pp[(size_t)k * stride];
  }
  red[r][e] = s0 + s1;
  __syncthreads();
  if (r == 0 && ok) {
    float v = 0.f;
#pragma unroll
    for (int q = 0; q < kRedLanes; ++q) v += red[q][e];
    dw[i] = v;
  }
}

// db[co] = sum_px dY[px][co] (masked), deterministic: block b sums the pixels [b per, (b+1) per).
// Thread t takes channel co = t % Cout and pixel lane r = t / Cout (R = 256 / Cout lanes): pixels
// p0 + r, p0 + r + R, ... in order into four accumulators (independent loads in flight), then the
// lanes of a channel are added in lane order.  The second pass sums the block partials of one
// channel per block: a fixed stride per thread, then a fixed pairwise tree.
template <typename T>
__global__ __launch_bounds__(256) void k_bias_partial(const T* __restrict__ dy,
                                                      const T* __restrict__ ym, int ldy, int Cout,
                                                      size_t npix, size_t per,
                                                      float* __restrict__ part) {
  __shared__ float red[256];
  const int t = threadIdx.x;
  const int R = 256 / Cout;  // Cout <= 256
  const int co = t % Cout, r = t / Cout;
  auto g = [&](size_t p) {
    const float v = Ld<T>::get(dy, p * ldy + co);
    return ym && !(Ld<T>::get(ym, p * Cout + co) > 0.f) ? 0.f : v;
  };
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  if (r < R) {
    const size_t p0 = (size_t)blockIdx.x * per, p1 = min(npix, p0 + per);
    size_t p = p0 + r;
    for (; p + 3 * (size_t)R < p1; p += 4 * (size_t)R) {
      s0 += g(p);
      s1 += g(p + R);
      s2 += g(p + 2 * R);
      s3 += g(p + 3 * R);
    }
    for (; p < p1; p += R) s0 += g(p);
  }
  red[t] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (r == 0) {
    float a = 0.f;
    for (int k = 0; k < R; ++k) a += red[k * Cout + co];
    part[(size_t)blockIdx.x * Cout + co] = a;
  }
}

__global__ __launch_bounds__(256) void k_bias_reduce(const float* __restrict__ part, int nb,
                                                     int Cout, float* __restrict__ db) {
  __shared__ float red[256];
  const int co = blockIdx.x, t = threadIdx.x;
  float s = 0.f;
  for (int b = t; b < nb; b += 256) s += part[(size_t)b * Cout + co];
  red[t] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) db[co] = red[0];
}

struct WgradPlan {
  int nrb, ncb, nblocks, splits, bps, CoutP, CinP, nchunk;
  size_t part_bytes, bias_blocks, bias_per;
};

WgradPlan wgrad_plan(int N, int H, int W, int Cin, int Cout, int KS) {
  WgradPlan p{};
  p.nrb = (H + kWgRows - 1) / kWgRows;
  p.ncb = (W + kWgCols - 1) / kWgCols;
  p.nblocks = N * p.nrb * p.ncb;
  p.nchunk = (Cin + kChunk - 1) / kChunk;
  p.CoutP = (Cout + 31) / 32 * 32;
  p.CinP = p.nchunk * kChunk;
  const int tiles = (p.CoutP / 32) * p.nchunk;
  // about 512 workgroups: enough to fill the chip, few partial sums to write and reduce
  int want = (512 + tiles - 1) / tiles;
  if (want > 256) want = 256;
  if (want < 1) want = 1;
  if (want > p.nblocks) want = p.nblocks;
  p.bps = (p.nblocks + want - 1) / want;
  p.splits = (p.nblocks + p.bps - 1) / p.bps;
  p.part_bytes = (size_t)p.splits * p.CoutP * KS * KS * p.CinP * sizeof(float);
  const size_t npix = (size_t)N * H * W;
  p.bias_per = (size_t)16 * (256 / (Cout < 256 ? Cout : 256));  // 16 pixels per lane
  p.bias_blocks = (npix + p.bias_per - 1) / p.bias_per;
  return p;
}

}  // namespace

extern "C" {

size_t aps_conv_packed_elems(int Cout, int ksize, int Cin) {
  if (Cout <= 0 || Cin <= 0 || (ksize != 1 && ksize != 3)) return 0;
  return packed_elems(Cout, ksize, Cin);
}

static int pack_impl(const float* w, int Cout, int ksize, int Cin, int dtype, void* packed,
                     void* stream, int transpose) {
  if (!w || !packed) return APS_ERR_NULL;
  if (Cout <= 0 || Cin <= 0) return APS_ERR_SHAPE;
  if (ksize != 1 && ksize != 3) return APS_ERR_UNSUPPORTED;
  // the packed operator's sizes
  const int co = transpose ? Cin : Cout, ci = transpose ? Cout : Cin;
  const size_t total = packed_elems(co, ksize, ci);
  const int nchunk = (ci + kChunk - 1) / kChunk;
  const int blocks = (int)((total + 255) / 256);
  hipStream_t st = as_stream(stream);
  if (dtype == APS_F32 && ksize == 3 && conv_cg(3, ci, co) == 4) {
    // 16-channel chunks (fits in the packed_elems allocation, which counts 32-channel chunks)
    const int n16 = (ci + 15) / 16;
    const size_t t16 = (size_t)((co + 16 * kMaxTM - 1) / (16 * kMaxTM)) * kMaxTM * 9 * n16 * 256;
    k_pack_f32c16<<<(int)((t16 + 255) / 256), 256, 0, st>>>(w, co, ci, n16, t16,
                                                            static_cast<float*>(packed), transpose);
  } else if (dtype == APS_F32)
    k_pack<float><<<blocks, 256, 0, st>>>(w, co, ksize, ci, nchunk, total,
                                          static_cast<float*>(packed), transpose, conv_cg(ksize, ci, co));
  else if (dtype == APS_BF16)
    k_pack<uint16_t><<<blocks, 256, 0, st>>>(w, co, ksize, ci, nchunk, total,
                                             static_cast<uint16_t*>(packed), transpose,
                                             conv_cg(ksize, ci, co));
  else
    return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_conv_pack_weights(const float* w, int Cout, int ksize, int Cin, int dtype, void* packed,
                          void* stream) {
  return pack_impl(w, Cout, ksize, Cin, dtype, packed, stream, 0);
}

int aps_conv_pack_weights_dgrad(const float* w, int Cout, int ksize, int Cin, int dtype,
                                void* packed, void* stream) {
  return pack_impl(w, Cout, ksize, Cin, dtype, packed, stream, 1);
}

int aps_conv2d_fwd(const void* x, const void* x2, int N, int H, int W, int Cx, int C2, int mode,
                   const void* packed_w, const float* bias, int Cout, int ksize, int relu,
                   int dtype, void* y, int ldy, int y_dtype, void* stream) {
  if (N < 0 || H < 0 || W < 0 || Cx <= 0 || C2 < 0 || Cout <= 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!x || !packed_w || !bias || !y) return APS_ERR_NULL;
  if (ksize != 1 && ksize != 3) return APS_ERR_UNSUPPORTED;
  if (Cx % 8 || C2 % 8) return APS_ERR_UNSUPPORTED;
  if (ldy < Cout) return APS_ERR_SHAPE;
  if (mode == APS_CONV_UP2_CAT) {
    if (!x2 || C2 <= 0) return APS_ERR_NULL;
    if (H % 2 || W % 2) return APS_ERR_SHAPE;
  } else if (mode == APS_CONV_DIRECT || mode == APS_CONV_POOL2) {
    if (C2 != 0) return APS_ERR_SHAPE;
  } else {
    return APS_ERR_ARG;
  }
  if ((size_t)N * H * W == 0) return APS_OK;
  ConvArgs a{};
  a.x = x;
  a.x2 = x2;
  a.N = N;
  a.H = H;
  a.W = W;
  a.Cx = Cx;
  a.C2 = C2;
  a.mode = mode;
  a.wp = packed_w;
  a.bias = bias;
  a.Cout = Cout;
  a.nchunk = (Cx + C2 + kChunk - 1) / kChunk;
  a.y = y;
  a.ldy = ldy;
  a.relu = relu;
  hipStream_t st = as_stream(stream);
  if (dtype == APS_F32 && ksize == 3 && conv_cg(3, Cx + C2, Cout) == 4 &&
      !fp32_offsets_fit(mode, N, H, W, Cx, C2))
    return APS_ERR_UNSUPPORTED;
  if (dtype == APS_F32 && y_dtype == APS_F32) dispatch_ks<float, float>(a, ksize, st);
  else if (dtype == APS_BF16 && y_dtype == APS_BF16) dispatch_ks<uint16_t, uint16_t>(a, ksize, st);
  else if (dtype == APS_BF16 && y_dtype == APS_F32) dispatch_ks<uint16_t, float>(a, ksize, st);
  else return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

}  // extern "C"

// ======================================================================== backward C ABI
extern "C" {

int aps_conv2d_bwd_data(const void* dy, const void* ymask, int ldy, int N, int H, int W, int Cout,
                        const void* packed_wT, int ksize, int Cin, int dtype, void* dX,
                        void* stream) {
  if (N < 0 || H < 0 || W < 0 || Cout <= 0 || Cin <= 0 || ldy < Cout) return APS_ERR_SHAPE;
  if (ksize != 1 && ksize != 3) return APS_ERR_UNSUPPORTED;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!dy || !packed_wT || !dX) return APS_ERR_NULL;
  const size_t es = dtype == APS_BF16 ? 2 : 4;
  if ((ldy * es) % 16) return APS_ERR_SHAPE;
  if (ymask && ldy != Cout) return APS_ERR_SHAPE;
  ConvArgs a{};
  a.x = dy;
  a.x2 = ymask;
  a.N = N;
  a.H = H;
  a.W = W;
  a.Cx = ldy;
  a.C2 = 0;
  a.mode = ymask ? kModeReluMask : APS_CONV_DIRECT;
  a.wp = packed_wT;
  a.bias = nullptr;
  a.Cout = Cin;
  a.nchunk = (ldy + kChunk - 1) / kChunk;
  // the operator was packed for Cout input channels: the padded stride must give the same layout
  const int kc = dtype == APS_F32 && ksize == 3 && conv_cg(3, ldy, Cin) == 4 ? 16 : kChunk;
  if ((ldy + kc - 1) / kc != (Cout + kc - 1) / kc || conv_cg(ksize, ldy, Cin) != conv_cg(ksize, Cout, Cin))
    return APS_ERR_SHAPE;
  if (dtype == APS_F32 && ksize == 3 && conv_cg(3, ldy, Cin) == 4 &&
      !fp32_offsets_fit(a.mode == kModeReluMask ? APS_CONV_DIRECT : a.mode, N, H, W, ldy, 0))
    return APS_ERR_UNSUPPORTED;
  a.y = dX;
  a.ldy = Cin;
  a.relu = 0;
  hipStream_t st = as_stream(stream);
  if (dtype == APS_F32) dispatch_ks<float, float>(a, ksize, st);
  else if (dtype == APS_BF16) dispatch_ks<uint16_t, uint16_t>(a, ksize, st);
  else return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_conv_input_grad(int mode, const void* dX, int N, int H, int W, int Cx, int C2, int dtype,
                        void* dx, int accumulate, void* dx2, int accumulate2, void* stream) {
  if (N < 0 || H < 0 || W < 0 || Cx <= 0 || C2 < 0) return APS_ERR_SHAPE;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!dX || !dx) return APS_ERR_NULL;
  size_t total;
  if (mode == APS_CONV_POOL2) {
    if (C2) return APS_ERR_SHAPE;
    total = (size_t)N * 4 * H * W * Cx;
  } else if (mode == APS_CONV_UP2_CAT) {
    if (!dx2 || C2 <= 0) return APS_ERR_NULL;
    if (H % 2 || W % 2) return APS_ERR_SHAPE;
    total = (size_t)N * (H / 2) * (W / 2) * Cx + (size_t)N * H * W * C2;
  } else if (mode == APS_CONV_DIRECT) {
    if (C2) return APS_ERR_SHAPE;
    total = (size_t)N * H * W * Cx;
  } else {
    return APS_ERR_ARG;
  }
  const unsigned blocks = (unsigned)((total + 255) / 256);
  hipStream_t st = as_stream(stream);
  if (dtype == APS_F32)
    k_input_grad<float><<<blocks, 256, 0, st>>>(mode, static_cast<const float*>(dX), N, H, W, Cx, C2,
                                                static_cast<float*>(dx), accumulate,
                                                static_cast<float*>(dx2), accumulate2);
  else if (dtype == APS_BF16)
    k_input_grad<uint16_t><<<blocks, 256, 0, st>>>(mode, static_cast<const uint16_t*>(dX), N, H, W,
                                                   Cx, C2, static_cast<uint16_t*>(dx), accumulate,
                                                   static_cast<uint16_t*>(dx2), accumulate2);
  else
    return APS_ERR_UNSUPPORTED;
  APS_LAUNCH_CHECK();
  return APS_OK;
}

size_t aps_conv2d_bwd_weight_workspace_size(int N, int H, int W, int Cx, int C2, int Cout,
                                            int ksize) {
  if (N <= 0 || H <= 0 || W <= 0 || Cout <= 0 || Cx <= 0) return 256;
  const WgradPlan p = wgrad_plan(N, H, W, Cx + C2, Cout, ksize);
  return ((p.part_bytes + 255) / 256) * 256 + p.bias_blocks * Cout * sizeof(float) + 256;
}

int aps_conv2d_bwd_weight(const void* x, const void* x2, int mode, int N, int H, int W, int Cx,
                          int C2, const void* dy, const void* ymask, int ldy, int Cout, int ksize,
                          int dtype, float* dw, float* db, void* ws, size_t ws_bytes,
                          void* stream) {
  if (N < 0 || H < 0 || W < 0 || Cx <= 0 || C2 < 0 || Cout <= 0 || ldy < Cout) return APS_ERR_SHAPE;
  if (ksize != 1 && ksize != 3) return APS_ERR_UNSUPPORTED;
  if (Cx % 8 || C2 % 8 || Cout > 256) return APS_ERR_UNSUPPORTED;
  if (mode == APS_CONV_UP2_CAT) {
    if (!x2 || C2 <= 0) return APS_ERR_NULL;
    if (H % 2 || W % 2) return APS_ERR_SHAPE;
  } else if (mode == APS_CONV_DIRECT || mode == APS_CONV_POOL2) {
    if (C2) return APS_ERR_SHAPE;
  } else {
    return APS_ERR_ARG;
  }
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!x || !dy || !dw) return APS_ERR_NULL;
  if (!ws || ws_bytes < aps_conv2d_bwd_weight_workspace_size(N, H, W, Cx, C2, Cout, ksize))
    return APS_ERR_WORKSPACE;
  const int Cin = Cx + C2;
  const WgradPlan p = wgrad_plan(N, H, W, Cin, Cout, ksize);
  WgradArgs a{};
  a.in.x = x;
  a.in.x2 = x2;
  a.in.N = N;
  a.in.H = H;
  a.in.W = W;
  a.in.Cx = Cx;
  a.in.C2 = C2;
  a.in.mode = mode;
  a.dy = dy;
  a.ymask = ymask;
  a.ldy = ldy;
  a.Cout = Cout;
  a.nchunk = p.nchunk;
  a.nrb = p.nrb;
  a.ncb = p.ncb;
  a.nblocks = p.nblocks;
  a.bps = p.bps;
  a.CoutP = p.CoutP;
  a.CinP = p.CinP;
  a.part = static_cast<float*>(ws);
  float* bpart = reinterpret_cast<float*>(static_cast<char*>(ws) + ((p.part_bytes + 255) / 256) * 256);
  hipStream_t st = as_stream(stream);
  dim3 grid(p.splits, p.CoutP / 32, p.nchunk);
  if (dtype == APS_F32) {
    if (ksize == 3) k_wgrad<float, 3><<<grid, 256, 0, st>>>(a);
    else k_wgrad<float, 1><<<grid, 256, 0, st>>>(a);
  } else if (dtype == APS_BF16) {
    if (ksize == 3) k_wgrad<uint16_t, 3><<<grid, 256, 0, st>>>(a);
    else k_wgrad<uint16_t, 1><<<grid, 256, 0, st>>>(a);
  } else {
    return APS_ERR_UNSUPPORTED;
  }
  const size_t nw = (size_t)Cout * ksize * ksize * Cin;
  k_wgrad_reduce<<<(unsigned)((nw + 31) / 32), 256, 0, st>>>(a.part, p.splits, Cout,
                                                                ksize * ksize, Cin, p.CoutP, p.CinP,
                                                                dw);
  if (db) {
    const size_t npix = (size_t)N * H * W;
    if (dtype == APS_F32)
      k_bias_partial<float><<<(unsigned)p.bias_blocks, 256, 0, st>>>(
          static_cast<const float*>(dy), static_cast<const float*>(ymask), ldy, Cout, npix,
          p.bias_per, bpart);
    else
      k_bias_partial<uint16_t><<<(unsigned)p.bias_blocks, 256, 0, st>>>(
          static_cast<const uint16_t*>(dy), static_cast<const uint16_t*>(ymask), ldy, Cout, npix,
          p.bias_per, bpart);
    k_bias_reduce<<<Cout, 256, 0, st>>>(bpart, (int)p.bias_blocks, Cout, db);
  }
  APS_LAUNCH_CHECK();
  return APS_OK;
}

}  // extern "C"

extern "C" {

int aps_conv2d_fwd_pool(const void* x, const void* x2, int N, int H, int W, int Cx, int C2,
                        int mode, const void* packed_w, const float* bias, int Cout, int relu,
                        int dtype, void* y, void* pooled, void* stream) {
  if (N < 0 || H < 0 || W < 0 || Cx <= 0 || C2 < 0 || Cout <= 0) return APS_ERR_SHAPE;
  if (dtype != APS_BF16 && dtype != APS_F32) return APS_ERR_ARG;
  if (H % 2 || W % 2) return APS_ERR_SHAPE;
  if (mode == APS_CONV_UP2_CAT) {
    if (C2 <= 0) return APS_ERR_SHAPE;
  } else if (mode == APS_CONV_DIRECT || mode == APS_CONV_POOL2) {
    if (C2 != 0) return APS_ERR_SHAPE;
  } else {
    return APS_ERR_ARG;
  }
  if (Cx % 8 || C2 % 8 || conv_cg(3, Cx + C2, Cout) != 4 || Cout % 16 || Cout <= 16)
    return APS_ERR_UNSUPPORTED;
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!x || !packed_w || !bias || !y || !pooled || (mode == APS_CONV_UP2_CAT && !x2))
    return APS_ERR_NULL;
  ConvArgs a{};
  a.x = x;
  a.x2 = x2;
  a.N = N;
  a.H = H;
  a.W = W;
  a.Cx = Cx;
  a.C2 = C2;
  a.mode = mode;
  a.wp = packed_w;
  a.bias = bias;
  a.Cout = Cout;
  a.nchunk = (Cx + C2 + kChunk - 1) / kChunk;
  a.y = y;
  a.ldy = Cout;
  a.relu = relu;
  a.pool = pooled;
  if (dtype == APS_F32) {
    if (!launch_conv_lds_f32<false>(a, as_stream(stream))) return APS_ERR_UNSUPPORTED;
  } else if (!launch_conv_lds<false>(a, as_stream(stream))) {
    return APS_ERR_UNSUPPORTED;
  }
  APS_LAUNCH_CHECK();
  return APS_OK;
}

int aps_conv2d_fwd_head(const void* x, const void* x2, int N, int H, int W, int Cx, int C2,
                        int mode, const void* packed_w, const float* bias, int Cout, int relu,
                        const void* packed_head, const float* head_bias, int K, int dtype,
                        void* y, int ldy, void* logits, int kstride, void* stream) {
  return aps_conv2d_fwd_head_ex(x, x2, N, H, W, Cx, C2, mode, packed_w, bias, Cout, relu,
                                packed_head, head_bias, K, dtype, y, ldy, logits, kstride, nullptr,
                                -1, stream);
}

int aps_conv2d_fwd_head_ex(const void* x, const void* x2, int N, int H, int W, int Cx, int C2,
                           int mode, const void* packed_w, const float* bias, int Cout, int relu,
                           const void* packed_head, const float* head_bias, int K, int dtype,
                           void* y, int ldy, void* logits, int kstride, void* side,
                           int side_offset, void* stream) {
  if (N < 0 || H < 0 || W < 0 || Cx <= 0 || C2 < 0 || K <= 0 || kstride < K) return APS_ERR_SHAPE;
  if (side) {
    if (side_offset < 0 || side_offset + 3 > K) return APS_ERR_SHAPE;
    // the side output is written from the staged logit rows (conv_epilogue)
    const size_t es = dtype == APS_BF16 ? 2 : 4;
    if (kstride > 16 * ((K + 15) / 16 > 4 ? 5 : 4) || (kstride * es) % 16 ||
        (reinterpret_cast<uintptr_t>(logits) & 15) ||
        (reinterpret_cast<uintptr_t>(side) & (4 * es - 1)))
      return APS_ERR_UNSUPPORTED;
  }
  if (Cout != 32 && Cout != 64) return APS_ERR_UNSUPPORTED;
  if (K > 80 || Cx % 8 || C2 % 8 || conv_cg(3, Cx + C2, Cout) != 4) return APS_ERR_UNSUPPORTED;
  if (y && ldy < Cout) return APS_ERR_SHAPE;
  if (mode == APS_CONV_UP2_CAT) {
    if (!x2 || C2 <= 0) return APS_ERR_NULL;
    if (H % 2 || W % 2) return APS_ERR_SHAPE;
  } else if (mode == APS_CONV_DIRECT || mode == APS_CONV_POOL2) {
    if (C2 != 0) return APS_ERR_SHAPE;
  } else {
    return APS_ERR_ARG;
  }
  if ((size_t)N * H * W == 0) return APS_OK;
  if (!x || !packed_w || !bias || !packed_head || !head_bias || !logits) return APS_ERR_NULL;
  ConvArgs a{};
  a.x = x;
  a.x2 = x2;
  a.N = N;
  a.H = H;
  a.W = W;
  a.Cx = Cx;
  a.C2 = C2;
  a.mode = mode;
  a.wp = packed_w;
  a.bias = bias;
  a.Cout = Cout;
  a.nchunk = (Cx + C2 + kChunk - 1) / kChunk;
  a.y = y;
  a.ldy = y ? ldy : Cout;
  a.relu = relu;
  a.hw = packed_head;
  a.hb = head_bias;
  a.hK = K;
  a.hy = logits;
  a.hldy = kstride;
  a.store_main = y != nullptr;
  a.hside = side;
  a.hside_off = side_offset;
  hipStream_t st = as_stream(stream);
  if (dtype == APS_F32 && !fp32_offsets_fit(mode, N, H, W, Cx, C2)) return APS_ERR_UNSUPPORTED;
  if (dtype == APS_F32) {
    if (Cout == 32) launch_conv_head<float, 2>(a, st); else launch_conv_head<float, 4>(a, st);
  } else if (dtype == APS_BF16) {
    if (Cout == 32) launch_conv_head<uint16_t, 2>(a, st); else launch_conv_head<uint16_t, 4>(a, st);
  } else {
    return APS_ERR_UNSUPPORTED;
  }
  APS_LAUNCH_CHECK();
  return APS_OK;
}

}  // extern "C"
