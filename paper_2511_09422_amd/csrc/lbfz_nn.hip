// lbfz_nn.hip -- kernels of the learned surrogate of the LB step (a 3-level
// U-Net of 3x3 convolutions that maps the six fields of a 256^2 crop to their
// change over 64 steps), for gfx950.  C ABI in include/lbfz_nn.h.
//
// Tensors are NHWC bf16 (channels innermost, a multiple of 8), weights
// [out channel][tap][in channel] bf16 with FP32 master copies, accumulation in
// FP32.  Convolutions are implicit GEMMs on the BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16).  Forward and data gradient: a 256-thread block
// computes a 128 x 128, 256 x 64 or 256 x 32 output tile (by the layer's
// width), 64 x 64 or 64 x 32 per wave, with the next K slice prefetched into
// registers during the MFMAs of the current one.  Weight gradient: 64 x 64
// tiles, 2 x 2 waves of 32 x 32, 32-deep K slices.
//   forward        out[p][n]  = sum_{t, c} in[p + o(t)][c] W[n][t][c]   (M = pixels)
//   data gradient  din[p][c]  = sum_{t, n} dz[p - o(t)][n] W[n][t][c]   (same kernel,
//                  weights transposed to Wt[c][t][n], offsets negated)
//   weight grad    dW[n][t][c] = sum_p dz[p][n] in[p + o(t)][c]          (M = out channels,
//                  K = pixels split over blocks, partials reduced in a fixed order)
// with o(t) = (t / 3 - 1, t % 3 - 1) for 3x3 taps (zero padding at the image
// edges) and o = 0 for 1x1.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "../../include/lbfz_nn.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 8;  // LDS rows padded by 16 B

// Buffer descriptor over `bytes` bytes at `base` (raw 32-bit data, no
// swizzle): loads take a 32-bit lane byte offset, and offsets at or past
// `bytes` read zero.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr uint32_t kOut = 0x80000000u;  // an offset past every tensor (< 2^31 bytes)
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ uint4 ld16B(rsrc_t r, uint32_t off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
  return __builtin_bit_cast(uint4, v);
}

// 8-channel (16-byte) groups of bf16 activations: pooling, upsampling and the
// bias gradient move whole groups (channel counts, strides and offsets are
// multiples of 8, checked by the callers).
union V8 {
  uint4 u;
  bf16 h[8];
};

__device__ __forceinline__ V8 ld8(const bf16* p) {
  V8 v;
  v.u = *reinterpret_cast<const uint4*>(p);
  return v;
}

__device__ __forceinline__ void st8(bf16* p, const V8& v) {
  *reinterpret_cast<uint4*>(p) = v.u;
}

__device__ __forceinline__ void tap_offset(int taps, int t, int sign, int& dy, int& dx) {
  if (taps == 1) {
    dy = dx = 0;
  } else {
    dy = sign * (t / 3 - 1);
    dx = sign * (t % 3 - 1);
  }
}

// 16 bytes (8 bf16) of channel data at pixel (b, y, x) shifted by (dy, dx) of
// an H x W image; zero outside the image.  up: the tensor holds the
// (H/2) x (W/2) image that nearest 2x upsampling maps onto H x W.
__device__ __forceinline__ uint4 load_px8(const bf16* __restrict__ t, int cs, int coff, int c,
                                          int b, int y, int x, int dy, int dx, int H, int W,
                                          bool ok, bool up) {
  const int yy = y + dy, xx = x + dx;
  if (!ok || yy < 0 || yy >= H || xx < 0 || xx >= W) return make_uint4(0, 0, 0, 0);
  const size_t px = up ? ((size_t)(b * (H >> 1) + (yy >> 1)) * (W >> 1) + (xx >> 1))
                       : ((size_t)(b * H + yy) * W + xx);
  return *reinterpret_cast<const uint4*>(t + px * cs + coff + c);
}

__device__ __forceinline__ f32x16 mfma_tile(const bf16 (*As)[LDK], const bf16 (*Bs)[LDK], int wm,
                                            int wn, int lane, f32x16 acc) {
#pragma unroll
  for (int kk = 0; kk < BK; kk += 16) {
    // lane: row (lane & 31), 8 consecutive k from 8 * (lane >> 5)
    const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&As[wm + (lane & 31)][kk + 8 * (lane >> 5)]);
    const bf16x8 fb = *reinterpret_cast<const bf16x8*>(&Bs[wn + (lane & 31)][kk + 8 * (lane >> 5)]);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb, acc, 0, 0, 0);
  }
  return acc;
}

// Accumulator element r of a lane sits at row 8 (r / 4) + 4 (lane / 32) + r % 4
// and column lane % 32 of the wave's 32 x 32 tile.
__device__ __forceinline__ int acc_row(int r, int lane) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// Forward / data-gradient convolution (M = pixels, N = a.N, K = taps * a.Cin).
// A block of 4 waves computes a BM x BN output tile; wave w owns a
// (32 FM) x (32 FN) sub-tile (FM x FN accumulators of 32 x 32) at wave
// position (w % WGM, w / WGM).  K advances in slices of KS = 32: each thread
// loads its 16-byte chunks of the next slice (chunk q = tid % 4 of rows
// tid / 4 + 64 j) into registers while the waves run the 2 x FM x FN MFMAs of
// the current slice from LDS, so the global latency hides behind the matrix
// work (a 64-deep slice doubles the LDS per block and measured slower: fewer
// blocks per CU).  Consecutive M tiles go to one XCD (blocks are dealt to the
// 8 XCDs round-robin), so the rows a 3 x 3 stencil re-reads from the
// neighbouring tiles hit the same L2.  The bf16 output tile is staged in LDS
// and written as whole 16-byte channel groups.
constexpr int KS = 32, LDS_K = KS + 8;      // LDS rows padded by 16 B
constexpr int CPR = KS / 8, RPP = 256 / CPR;   // 16-byte chunks per row, rows per pass

template <int FM, int FN, int WGM, int WGN, bool UP>
__global__ __launch_bounds__(256) void k_conv(lbfz_conv_args a) {
  static_assert(WGM * WGN == 4, "4 waves");
  constexpr int BM_ = 32 * FM * WGM, BN_ = 32 * FN * WGN;
  // 16-byte chunks per thread and slice (B: the last pass may be partial)
  constexpr int AR = BM_ / RPP, BR = (BN_ + RPP - 1) / RPP;
  constexpr int A_EL = BM_ * LDS_K, B_EL = BN_ * LDS_K;
  constexpr int OS = BN_;         // row stride of the bf16 output tile staged for the stores
  constexpr int O_EL = BM_ * OS;
  constexpr int SM_EL = (A_EL + B_EL) > O_EL ? (A_EL + B_EL) : O_EL;
  __shared__ __align__(16) bf16 smem[SM_EL];
  bf16 (*As)[LDS_K] = reinterpret_cast<bf16 (*)[LDS_K]>(smem);
  bf16 (*Bs)[LDS_K] = reinterpret_cast<bf16 (*)[LDS_K]>(smem + A_EL);
  const int M = a.B * a.H * a.W, K = a.taps * a.Cin;
  const int nbm = gridDim.x;
  int bx = blockIdx.x;
  if ((nbm & 7) == 0) bx = (bx & 7) * (nbm >> 3) + (bx >> 3);
  const int m0 = bx * BM_, n0 = blockIdx.y * BN_;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave % WGM) * 32 * FM, wn = (wave / WGM) * 32 * FN;
  // operands through buffer descriptors: 32-bit byte offsets, and an offset
  // past the end (kOut) reads zeros -- the halo of the image and the K tail
  // need no branches (the host keeps both tensors under 2^31 bytes)
  const uint32_t in_bytes = (uint32_t)((UP ? (size_t)M / 4 : (size_t)M) * a.in_cs * 2);
  const rsrc_t rin = make_rsrc(a.in, in_bytes);
  const rsrc_t rw = make_rsrc(a.w, (uint32_t)((size_t)a.N * K * 2));
  const int q = tid % CPR, r0 = tid / CPR;
  // per A row (pixel): the byte offset of its own pixel (UP: of its image in
  // the half-resolution tensor) and the set of taps whose source lies inside
  // the image; UP also keeps the half-resolution row / column offsets of the
  // three source rows and columns
  const int cs2 = a.in_cs * 2;
  uint32_t rowb[AR], tapok[AR];
  int ysh[UP ? AR : 1][3], xsh[UP ? AR : 1][3];
#pragma unroll
  for (int j = 0; j < AR; ++j) {
    const int p = m0 + r0 + RPP * j;
    const int img = p / (a.H * a.W), rem = p - img * (a.H * a.W);
    const int py = rem / a.W, px = rem - py * a.W;
    uint32_t ok = 0;
    if (p < M) {
      if (a.taps == 1) {
        ok = 1;
      } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const int yy = py + a.sign * (t / 3 - 1), xx = px + a.sign * (t % 3 - 1);
          if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W) ok |= 1u << t;
        }
      }
    }
    tapok[j] = ok;
    if constexpr (UP) {
      rowb[j] = (uint32_t)(img * (a.H >> 1) * (a.W >> 1)) * cs2;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        ysh[j][d] = ((py + d - 1) >> 1) * (a.W >> 1) * cs2;
        xsh[j][d] = ((px + d - 1) >> 1) * cs2;
      }
    } else {
      rowb[j] = (uint32_t)p * cs2;
    }
  }
  // this thread's K position k = k0 + 8 q as (tap t, channel c), advanced by
  // KS per slice without a division
  int t = (8 * q) / a.Cin, c = 8 * q - t * a.Cin;
  // weight rows of this thread (B operand) and their byte offsets at k
  uint32_t wb[BR];
  bool wok[BR];
#pragma unroll
  for (int j = 0; j < BR; ++j) {
    const int rr = r0 + RPP * j, n = n0 + rr;
    wok[j] = rr < BN_ && n < a.N;
    wb[j] = (uint32_t)(n * K + 8 * q) * 2;
  }
  const uint32_t co2 = (uint32_t)a.in_co * 2;
  auto gload = [&](uint4 (&ra)[AR], uint4 (&rb)[BR]) {
    const bool kok = t < a.taps;
    const int ti = a.taps == 1 ? 4 : t;   // the centre tap for 1 x 1
    const int dyi = ti >= 6 ? 2 : (ti >= 3 ? 1 : 0), dxi = ti - 3 * dyi;
    const uint32_t cb = co2 + (uint32_t)c * 2;
    // non-UP: the tap's shift of the pixel index, in bytes
    const int dsh = (a.sign * (dyi - 1) * a.W + a.sign * (dxi - 1)) * cs2;
#pragma unroll
    for (int j = 0; j < AR; ++j) {
      uint32_t off;
      if constexpr (UP)
        off = rowb[j] + ysh[j][dyi] + xsh[j][dxi] + cb;
      else
        off = rowb[j] + dsh + cb;
      const bool ok = kok && ((tapok[j] >> (a.taps == 1 ? 0 : t)) & 1u);
      ra[j] = ld16B(rin, ok ? off : kOut);
    }
#pragma unroll
    for (int j = 0; j < BR; ++j) rb[j] = ld16B(rw, (kok && wok[j]) ? wb[j] : kOut);
  };
  // advance (t, c) and the weight offsets by one slice
  auto advance = [&]() {
    c += KS;
    while (c >= a.Cin) {
      c -= a.Cin;
      ++t;
    }
#pragma unroll
    for (int j = 0; j < BR; ++j) wb[j] += KS * 2;
  };
  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};
  // one slice: registers -> LDS (after every wave has read the previous one)
  auto stage = [&](const uint4 (&ra)[AR], const uint4 (&rb)[BR]) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < AR; ++j) *reinterpret_cast<uint4*>(&As[r0 + RPP * j][8 * q]) = ra[j];
#pragma unroll
    for (int j = 0; j < BR; ++j)
      if (r0 + RPP * j < BN_) *reinterpret_cast<uint4*>(&Bs[r0 + RPP * j][8 * q]) = rb[j];
    __syncthreads();
  };
  auto compute = [&]() {
#pragma unroll
    for (int kk = 0; kk < KS; kk += 16) {
      bf16x8 fa[FM], fb[FN];
      const int kc = kk + 8 * (lane >> 5);
#pragma unroll
      for (int i = 0; i < FM; ++i)
        fa[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 32 * i + (lane & 31)][kc]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        fb[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 32 * j + (lane & 31)][kc]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
  };
  uint4 ra[AR], rb[BR];
  gload(ra, rb);
  for (int k0 = 0; k0 < K; k0 += KS) {
    stage(ra, rb);
    if (k0 + KS < K) {
      advance();
      gload(ra, rb);
    }
    compute();
  }
  const float* bias = a.bias;
  if (!a.out_f32 && a.N % 8 == 0 && a.out_cs % 8 == 0 && a.out_co % 8 == 0) {
    // stage the bf16 tile in LDS, then write whole 16-byte channel groups
    bf16* Os = smem;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = wn + 32 * j + (lane & 31);
      const float bv = (bias && n0 + col < a.N) ? bias[n0 + col] : 0.0f;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          float v = acc[i][j][r] + bv;
          if (a.relu) v = fmaxf(v, 0.0f);
          Os[(wm + 32 * i + acc_row(r, lane)) * OS + col] = (bf16)v;
        }
    }
    __syncthreads();
    constexpr int GPR = BN_ / 8;  // 16-byte groups per tile row
    for (int g = tid; g < BM_ * GPR; g += 256) {
      const int row = g / GPR, cg = g - row * GPR;
      const int pm = m0 + row, cn = n0 + 8 * cg;
      if (pm < M && cn < a.N)
        *reinterpret_cast<uint4*>(static_cast<bf16*>(a.out) + (size_t)pm * a.out_cs + a.out_co +
                                  cn) = *reinterpret_cast<const uint4*>(&Os[row * OS + 8 * cg]);
    }
    return;
  }
  // FP32 output or unaligned channels: direct stores
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int cn = n0 + wn + 32 * j + (lane & 31);
    if (cn >= a.N) continue;
    const float bv = bias ? bias[cn] : 0.0f;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int pm = m0 + wm + 32 * i + acc_row(r, lane);
        if (pm >= M) continue;
        float v = acc[i][j][r] + bv;
        if (a.relu) v = fmaxf(v, 0.0f);
        const size_t o = (size_t)pm * a.out_cs + a.out_co + cn;
        if (a.out_f32)
          static_cast<float*>(a.out)[o] = v;
        else
          static_cast<bf16*>(a.out)[o] = (bf16)v;
      }
    }
  }
}

// Direct 3 x 3 convolution (forward, data gradient, and the forward through
// 2x upsampling): a block computes a (4 RPW) x 64 tile of output pixels of
// one image for BN = 32 FN output channels.  Per input-channel chunk of CC
// (32, or 16) it stages the (4 RPW + 2) x 66 haloed input tile and the chunk's
// weights [n][tap][c] in LDS once, then every wave (RPW output rows, 2 RPW x
// FN accumulators of 32 x 32) runs the nine taps' MFMAs reading its A
// fragments from the tile at the tap's shift -- each input byte is loaded
// from memory 1.3 - 1.6 times instead of nine (the implicit GEMM above
// re-gathers it per tap).  Tap shifts are compile-time (SIGN), so fragment addresses are one
// per-lane base plus immediates.  The next chunk's loads are issued before
// the current chunk's MFMAs.
constexpr int TW = 64, TH = 4, HWD = TW + 2, HHT = TH + 2;

// CC: input channels per chunk (32, or 16 for layers whose channel count is
// not a multiple of 32, e.g. the 16-channel input layer)
//
// TAIL (inference, lbfz_nn_conv_tail): after the block's output tile is staged
// in LDS, the 1 x 1 head and the prediction of the tile's pixels follow in
// the same block (the 32 channels of every pixel are in the tile).
template <int FN, bool UP, int SIGN, int CC, int RPW, bool TAIL>
__device__ __forceinline__ void conv_direct(const lbfz_conv_args& a, const lbfz_tail_args& tl) {
  constexpr int BN_ = 32 * FN;
  constexpr int TH_ = 4 * RPW, HH_ = TH_ + 2;  // tile rows (RPW per wave), halo rows
  constexpr int FM = 2 * RPW;                  // A fragments per wave (32 pixels each)
  constexpr int HPS = CC + 8;            // LDS pixel stride (bf16), padded by 16 B
  constexpr int CPX = CC / 8;            // 16-byte chunks per pixel and chunk
  constexpr int H_EL = HH_ * HWD * HPS;  // haloed input tile [pixel][c]
  constexpr int W_EL = BN_ * 9 * HPS;    // weights [n][tap][c]
  constexpr int O_EL = TH_ * TW * BN_;   // bf16 output tile for the stores
  constexpr int SM_EL = (H_EL + W_EL) > O_EL ? (H_EL + W_EL) : O_EL;
  constexpr int HE = HH_ * HWD * CPX, HJ = (HE + 255) / 256;  // halo 16-byte chunks
  constexpr int WE = BN_ * 9 * CPX, WJ = (WE + 255) / 256;    // weight 16-byte chunks
  __shared__ __align__(16) bf16 smem[SM_EL];
  bf16* Hs = smem;
  bf16* Ws = smem + H_EL;
  const int tiles_x = (a.W + TW - 1) / TW, tiles_y = (a.H + TH_ - 1) / TH_;
  const int nt = gridDim.x;
  int bx = blockIdx.x;
  if ((nt & 7) == 0) bx = (bx & 7) * (nt >> 3) + (bx >> 3);  // neighbouring tiles on one XCD
  const int b = bx / (tiles_y * tiles_x), rt = bx - b * (tiles_y * tiles_x);
  const int y0 = (rt / tiles_x) * TH_, x0 = (rt % tiles_x) * TW;
  const int n0 = blockIdx.y * BN_;
  const int M = a.B * a.H * a.W, K = 9 * a.Cin;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint32_t in_bytes = (uint32_t)((UP ? (size_t)M / 4 : (size_t)M) * a.in_cs * 2);
  const rsrc_t rin = make_rsrc(a.in, in_bytes);
  const rsrc_t rw = make_rsrc(a.w, (uint32_t)((size_t)a.N * K * 2));
  // this thread's halo chunks: byte offset at channel 0 of the layer input
  // (kOut outside the image) and the chunk's channel offset q * 8
  uint32_t hoff[HJ];
  int hq[HJ];
#pragma unroll
  for (int j = 0; j < HJ; ++j) {
    const int e = tid + 256 * j, hp = e / CPX;
    hq[j] = 8 * (e % CPX);
    const int yy = y0 + hp / HWD - 1, xx = x0 + hp % HWD - 1;
    hoff[j] = kOut;
    if (e < HE && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W) {
      const int src = UP ? (b * (a.H >> 1) + (yy >> 1)) * (a.W >> 1) + (xx >> 1)
                         : (b * a.H + yy) * a.W + xx;
      hoff[j] = ((uint32_t)src * a.in_cs + a.in_co + hq[j]) * 2;
    }
  }
  uint32_t woff[WJ];
  int wq[WJ];
#pragma unroll
  for (int j = 0; j < WJ; ++j) {
    const int e = tid + 256 * j, n = e / (9 * CPX), rem = e - n * (9 * CPX);
    wq[j] = 8 * (rem % CPX);
    woff[j] = (e < WE && n0 + n < a.N) ? ((uint32_t)(n0 + n) * K + (rem / CPX) * a.Cin + wq[j]) * 2
                                      : kOut;
  }
  uint4 hv[HJ], wv[WJ];
  auto gload = [&](int c0) {
#pragma unroll
    for (int j = 0; j < HJ; ++j)
      hv[j] = ld16B(rin, (hoff[j] != kOut && c0 + hq[j] < a.Cin) ? hoff[j] + 2 * c0 : kOut);
#pragma unroll
    for (int j = 0; j < WJ; ++j)
      wv[j] = ld16B(rw, (woff[j] != kOut && c0 + wq[j] < a.Cin) ? woff[j] + 2 * c0 : kOut);
  };
  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};
  // fragment bases: A at halo pixel (RPW wave, lane % 32) -- the (-1, -1)
  // shift of output pixel (RPW wave, lane % 32) -- and B at weight row
  // lane % 32; the k half 8 (lane / 32).  A fragment i covers output row
  // RPW wave + i / 2, columns 32 (i % 2) ...
  const bf16* abase = Hs + (RPW * wave * HWD + (lane & 31)) * HPS + 8 * (lane >> 5);
  const bf16* bbase = Ws + (lane & 31) * 9 * HPS + 8 * (lane >> 5);
  gload(0);
  for (int c0 = 0; c0 < a.Cin; c0 += CC) {
    __syncthreads();  // the previous chunk's fragments have been read
#pragma unroll
    for (int j = 0; j < HJ; ++j) {
      const int e = tid + 256 * j;
      if (e < HE) *reinterpret_cast<uint4*>(Hs + (e / CPX) * HPS + 8 * (e % CPX)) = hv[j];
    }
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      const int e = tid + 256 * j;
      if (e < WE) {
        const int n = e / (9 * CPX), rem = e - n * (9 * CPX);
        *reinterpret_cast<uint4*>(Ws + (n * 9 + rem / CPX) * HPS + 8 * (rem % CPX)) = wv[j];
      }
    }
    __syncthreads();
    if (c0 + CC < a.Cin) gload(c0 + CC);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      // tap t reads input pixel (y + SIGN (t / 3 - 1), x + SIGN (t % 3 - 1));
      // relative to the (-1, -1) base that is row 1 + SIGN (t / 3 - 1), column
      // 1 + SIGN (t % 3 - 1) of the halo tile
      const int hy = 1 + SIGN * (t / 3 - 1), hx = 1 + SIGN * (t % 3 - 1);
#pragma unroll
      for (int kk = 0; kk < CC; kk += 16) {
        bf16x8 fa[FM], fb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
          fa[i] = *reinterpret_cast<const bf16x8*>(
              abase + ((hy + i / 2) * HWD + hx + 32 * (i % 2)) * HPS + kk);
#pragma unroll
        for (int j = 0; j < FN; ++j)
          fb[j] = *reinterpret_cast<const bf16x8*>(bbase + (32 * j * 9 + t) * HPS + kk);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
      }
    }
  }
  // epilogue: output pixel (y0 + RPW wave + i / 2, x0 + 32 (i % 2) + row)
  // and channel n0 + 32 j + lane % 32 of accumulator element r (row =
  // acc_row(r, lane))
  const float* bias = a.bias;
  if (TAIL || (!a.out_f32 && a.N % 8 == 0 && a.out_cs % 8 == 0 && a.out_co % 8 == 0)) {
    bf16* Os = smem;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = 32 * j + (lane & 31);
      const float bv = (bias && n0 + col < a.N) ? bias[n0 + col] : 0.0f;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          float v = acc[i][j][r] + bv;
          if (a.relu) v = fmaxf(v, 0.0f);
          Os[((RPW * wave + i / 2) * TW + 32 * (i % 2) + acc_row(r, lane)) * BN_ + col] = (bf16)v;
        }
    }
    // tail: the head's weights and bias as FP32 behind the output tile
    float* hw = reinterpret_cast<float*>(smem + O_EL);
    if constexpr (TAIL) {
      static_assert(FN == 1 && 2 * O_EL + 4 * 32 * 33 <= 2 * SM_EL, "tail LDS");
      for (int e = tid; e < tl.nh * 32; e += 256)
        hw[e] = (float)static_cast<const bf16*>(tl.head_w)[e];
      if (tid < tl.nh) hw[32 * 32 + tid] = tl.head_b ? tl.head_b[tid] : 0.0f;
    }
    __syncthreads();
    constexpr int GPR = BN_ / 8;
    if (!TAIL || a.out) {
      for (int g = tid; g < TH_ * TW * GPR; g += 256) {
        const int m = g / GPR, cg = g - m * GPR;
        const int yy = y0 + m / TW, xx = x0 + m % TW, cn = n0 + 8 * cg;
        if (yy < a.H && xx < a.W && cn < a.N)
          *reinterpret_cast<uint4*>(static_cast<bf16*>(a.out) +
                                    ((size_t)(b * a.H + yy) * a.W + xx) * a.out_cs + a.out_co +
                                    cn) = *reinterpret_cast<const uint4*>(&Os[m * BN_ + 8 * cg]);
      }
    }
    if constexpr (TAIL) {
      // head and prediction, one pixel per thread and pass (consecutive
      // threads take consecutive columns of a row: coalesced plane accesses)
      const long npx = (long)a.H * a.W;
      for (int m = tid; m < TH_ * TW; m += 256) {
        const int yy = y0 + m / TW, xx = x0 + m % TW;
        if (yy >= a.H || xx >= a.W) continue;
        float v[32];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          V8 c8;
          c8.u = *reinterpret_cast<const uint4*>(&Os[m * BN_ + 8 * q]);
#pragma unroll
          for (int e = 0; e < 8; ++e) v[8 * q + e] = (float)c8.h[e];
        }
        const long px = (long)yy * a.W + xx;
        const float* bsrc = tl.before + b * tl.before_stride + px;
        float* pdst = tl.pred + b * tl.pred_stride + px;
        for (int f = 0; f < tl.nf; ++f) {
          float o = hw[32 * 32 + f];
#pragma unroll
          for (int c = 0; c < 32; ++c) o = fmaf(hw[32 * f + c], v[c], o);
          pdst[f * npx] = tl.resid[f] * bsrc[f * npx] + o / tl.scale[f] + tl.shift[f];
        }
      }
      return;
    }
    if (a.pool) {
      // fused 2 x 2 max pooling of the stored (bf16) output: the tile's rows
      // and columns start even, so every window lies inside it
      const int Ho = a.H >> 1, Wo = a.W >> 1;
      for (int g = tid; g < (TH_ / 2) * (TW / 2) * GPR; g += 256) {
        const int m = g / GPR, cg = g - m * GPR;
        const int py = m / (TW / 2), px = m % (TW / 2);
        const int yo = (y0 >> 1) + py, xo = (x0 >> 1) + px, cn = n0 + 8 * cg;
        if (yo >= Ho || xo >= Wo || cn >= a.N) continue;
        const int m00 = (2 * py) * TW + 2 * px;
        V8 v0, v1, v2, v3, r;
        v0.u = *reinterpret_cast<const uint4*>(&Os[m00 * BN_ + 8 * cg]);
        v1.u = *reinterpret_cast<const uint4*>(&Os[(m00 + 1) * BN_ + 8 * cg]);
        v2.u = *reinterpret_cast<const uint4*>(&Os[(m00 + TW) * BN_ + 8 * cg]);
        v3.u = *reinterpret_cast<const uint4*>(&Os[(m00 + TW + 1) * BN_ + 8 * cg]);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          r.h[e] = (bf16)fmaxf(fmaxf((float)v0.h[e], (float)v1.h[e]),
                               fmaxf((float)v2.h[e], (float)v3.h[e]));
        *reinterpret_cast<uint4*>(static_cast<bf16*>(a.pool) +
                                  ((size_t)(b * Ho + yo) * Wo + xo) * a.pool_cs + a.pool_co + cn) = r.u;
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int cn = n0 + 32 * j + (lane & 31);
    if (cn >= a.N) continue;
    const float bv = bias ? bias[cn] : 0.0f;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int y = y0 + RPW * wave + i / 2;
      if (y >= a.H) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int x = x0 + 32 * (i % 2) + acc_row(r, lane);
        if (x >= a.W) continue;
        float v = acc[i][j][r] + bv;
        if (a.relu) v = fmaxf(v, 0.0f);
        const size_t o = ((size_t)(b * a.H + y) * a.W + x) * a.out_cs + a.out_co + cn;
        if (a.out_f32)
          static_cast<float*>(a.out)[o] = v;
        else
          static_cast<bf16*>(a.out)[o] = (bf16)v;
      }
    }
  }
}

template <int FN, bool UP, int SIGN, int CC = 32, int RPW = 1>
__global__ __launch_bounds__(256) void k_conv_direct(lbfz_conv_args a) {
  conv_direct<FN, UP, SIGN, CC, RPW, false>(a, lbfz_tail_args{});
}

__global__ __launch_bounds__(256) void k_conv_tail(lbfz_conv_args a, lbfz_tail_args t) {
  conv_direct<1, false, 1, 32, 2, true>(a, t);
}

// Weight gradient of a 3 x 3 convolution, direct form: dW[n][t][c] = sum_p
// dz[p][n] x[p + o(t)][c].  A block owns 32 output channels n0.. and 32 input
// channels c0.. and walks the 4 x 64 pixel tiles split, split + gridDim.x, ...
// For each tile it stages dz transposed, dzT[n][pixel], and the haloed input
// transposed in three copies shifted by the tap column, X[s][c][row][col] =
// x(row - 1, col + s - 1), so that the MFMA fragments -- 8 consecutive
// pixels of one channel per lane -- are aligned 16-byte LDS reads for every
// tap.  Wave w reduces over output row w of the tile and keeps the nine
// taps' 32 x 32 accumulators; the block adds its four waves' sums (fixed
// order) into partial row `split`, and the partial rows are summed in a
// fixed order (deterministic).
constexpr int DZS = TH * TW + 8;  // dzT row stride (bf16)
constexpr int XRS = TW + 8;       // X row stride (bf16)

template <bool UP>
__global__ __launch_bounds__(256) void k_conv_wgrad_direct(lbfz_conv_args a,
                                                           float* __restrict__ part) {
  constexpr int DZ_EL = 32 * DZS, X_EL = 3 * 32 * HHT * XRS;
  constexpr int DJ = TH * TW * 4 / 256;                  // dz 16-byte chunks per thread
  constexpr int XE = HHT * HWD * 4, XJ = (XE + 255) / 256;  // halo chunks
  __shared__ __align__(16) bf16 smem[DZ_EL + X_EL];
  bf16* dzT = smem;
  bf16* Xs = smem + DZ_EL;
  const int tiles_x = (a.W + TW - 1) / TW, tiles_y = (a.H + TH - 1) / TH;
  const int ntiles = a.B * tiles_y * tiles_x;
  const int n0 = blockIdx.y * 32, c0 = blockIdx.z * 32;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int M = a.B * a.H * a.W;
  const rsrc_t rin = make_rsrc(a.in, (uint32_t)((UP ? (size_t)M / 4 : (size_t)M) * a.in_cs * 2));
  const rsrc_t rdz = make_rsrc(a.w, (uint32_t)((size_t)M * a.dz_cs * 2));
  uint4 dv[DJ], xv[XJ];
  // loads of tile `tile` into registers: dz chunk j of this thread is pixel
  // (tid + 256 j) % 256 of the tile, channel group (tid + 256 j) / 256; halo
  // chunk j is halo pixel e % (HHT HWD), channel group e / (HHT HWD)
  auto gload = [&](int tile) {
    const int b = tile / (tiles_y * tiles_x), rt = tile - b * (tiles_y * tiles_x);
    const int y0 = (rt / tiles_x) * TH, x0 = (rt % tiles_x) * TW;
#pragma unroll
    for (int j = 0; j < DJ; ++j) {
      const int e = tid + 256 * j, px = e % (TH * TW), g = e / (TH * TW);
      const int y = y0 + px / TW, x = x0 + px % TW;
      const bool ok = y < a.H && x < a.W && n0 + 8 * g < a.N;
      dv[j] = ld16B(rdz, ok ? ((uint32_t)((b * a.H + y) * a.W + x) * a.dz_cs + n0 + 8 * g) * 2
                            : kOut);
    }
#pragma unroll
    for (int j = 0; j < XJ; ++j) {
      const int e = tid + 256 * j, hp = e % (HHT * HWD), g = e / (HHT * HWD);
      const int yy = y0 + hp / HWD - 1, xx = x0 + hp % HWD - 1;
      uint32_t off = kOut;
      if (e < XE && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W && c0 + 8 * g < a.Cin) {
        const int src = UP ? (b * (a.H >> 1) + (yy >> 1)) * (a.W >> 1) + (xx >> 1)
                           : (b * a.H + yy) * a.W + xx;
        off = ((uint32_t)src * a.in_cs + a.in_co + c0 + 8 * g) * 2;
      }
      xv[j] = ld16B(rin, off);
    }
  };
  f32x16 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = f32x16{};
  const int split = blockIdx.x;
  if (split < ntiles) gload(split);
  for (int tile = split; tile < ntiles; tile += gridDim.x) {
    __syncthreads();  // the previous tile's fragments have been read
#pragma unroll
    for (int j = 0; j < DJ; ++j) {
      const int e = tid + 256 * j, px = e % (TH * TW), g = e / (TH * TW);
      V8 v;
      v.u = dv[j];
#pragma unroll
      for (int k = 0; k < 8; ++k) dzT[(8 * g + k) * DZS + px] = v.h[k];
    }
#pragma unroll
    for (int j = 0; j < XJ; ++j) {
      const int e = tid + 256 * j;
      if (e >= XE) continue;
      const int hp = e % (HHT * HWD), g = e / (HHT * HWD);
      const int hy = hp / HWD, hx = hp % HWD;
      V8 v;
      v.u = xv[j];
#pragma unroll
      for (int sft = 0; sft < 3; ++sft) {
        const int tx = hx - sft;
        if (tx >= 0 && tx < TW) {
#pragma unroll
          for (int k = 0; k < 8; ++k) Xs[((sft * 32 + 8 * g + k) * HHT + hy) * XRS + tx] = v.h[k];
        }
      }
    }
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) gload(tile + gridDim.x);
    // wave w: output row w of the tile, 4 k-steps of 16 pixels per tap
    const bf16* abase = dzT + (lane & 31) * DZS + wave * TW + 8 * (lane >> 5);
    const bf16* bbase = Xs + (lane & 31) * HHT * XRS + 8 * (lane >> 5);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int sft = t % 3, hy = wave + t / 3;  // copy dx + 1, halo row y + dy + 1
#pragma unroll
      for (int kk = 0; kk < TW; kk += 16) {
        const bf16x8 fa = *reinterpret_cast<const bf16x8*>(abase + kk);
        const bf16x8 fb =
            *reinterpret_cast<const bf16x8*>(bbase + (sft * 32 * HHT + hy) * XRS + kk);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb, acc[t], 0, 0, 0);
      }
    }
  }
  // the four waves' sums, added in LDS in a fixed order, one tap at a time,
  // into partial row `split`: element r of tap t is dW[n0 + acc_row][t][c0 +
  // lane % 32]
  const size_t NW = (size_t)9 * a.Cin;
  float* prow = part + (size_t)split * a.N * NW;
  float* red = reinterpret_cast<float*>(smem);  // 4 x 32 x 32 floats
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wave * 1024 + acc_row(r, lane) * 32 + (lane & 31)] = acc[t][r];
    __syncthreads();
    for (int i = tid; i < 1024; i += 256) {
      const float v = ((red[i] + red[1024 + i]) + red[2048 + i]) + red[3072 + i];
      const int n = n0 + i / 32, c = c0 + i % 32;
      if (n < a.N && c < a.Cin) prow[(size_t)n * NW + t * a.Cin + c] = v;
    }
  }
}

// Weight gradient: partial[s][n][t * Cin + c] over the pixel range of split s
// (M = out channels a.N, N = taps * a.Cin, K = pixels).  a.in: the layer's
// input, a.w: dz (gradient at the layer's pre-activation, a.N channels at
// channel stride a.dz_cs).
__global__ __launch_bounds__(256) void k_conv_wgrad(lbfz_conv_args a, float* __restrict__ part,
                                                    int kper) {
  __shared__ __align__(16) bf16 As[BM][LDK];
  __shared__ __align__(16) bf16 Bs[BN][LDK];
  const int P = a.B * a.H * a.W, NW = a.taps * a.Cin;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN, s = blockIdx.z;
  const int kb = s * kper, ke = min(kb + kper, P);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const bf16* __restrict__ in = static_cast<const bf16*>(a.in);
  const bf16* __restrict__ dz = static_cast<const bf16*>(a.w);
  // loader slot: pixel lp of the 32-pixel K slice, 8 channels from lq
  const int lp = tid >> 3, lq = (tid & 7) * 8;
  const int am = m0 + lq;            // out channels am .. am + 7
  const int bn = n0 + lq;            // (tap, in channel) columns bn .. bn + 7
  const int bt = bn / a.Cin, bc = bn - bt * a.Cin;
  int bdy, bdx;
  tap_offset(a.taps, bt, 1, bdy, bdx);
  f32x16 acc = {};
  for (int k0 = kb; k0 < ke; k0 += BK) {
    const int p = k0 + lp;
    const bool pok = p < ke;
    const int px = p % a.W, py = (p / a.W) % a.H, pb = p / (a.W * a.H);
    uint4 va = make_uint4(0, 0, 0, 0), vb = make_uint4(0, 0, 0, 0);
    if (pok && am < a.N)
      va = *reinterpret_cast<const uint4*>(dz + (size_t)p * a.dz_cs + am);
    if (bn < NW)
      vb = load_px8(in, a.in_cs, a.in_co, bc, pb, py, px, bdy, bdx, a.H, a.W, pok, a.up != 0);
    __syncthreads();
    const bf16* ea = reinterpret_cast<const bf16*>(&va);
    const bf16* eb = reinterpret_cast<const bf16*>(&vb);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      As[lq + j][lp] = ea[j];
      Bs[lq + j][lp] = eb[j];
    }
    __syncthreads();
    acc = mfma_tile(As, Bs, wm, wn, lane, acc);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int mm = m0 + wm + acc_row(r, lane), nn = n0 + wn + (lane & 31);
    if (mm < a.N && nn < NW) part[((size_t)s * a.N + mm) * NW + nn] = acc[r];
  }
}


// dst[i] = sum over s of part[s][i] (fixed order).
__global__ void k_sum_splits(const float* __restrict__ part, int nsplit, long n,
                             float* __restrict__ dst) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    float v = 0.0f;
    for (int s = 0; s < nsplit; ++s) v += part[(size_t)s * n + i];
    dst[i] = v;
  }
}

// dst[i] = sum over s of part[s][i] for a short vector (n small, many
// splits): one block per element, the splits strided over the threads, then
// a tree over the block (a fixed order).
__global__ __launch_bounds__(256) void k_sum_splits_small(const float* __restrict__ part,
                                                          int nsplit, int n,
                                                          float* __restrict__ dst) {
  __shared__ float red[256];
  const int i = blockIdx.x;
  float v = 0.0f;
  for (int s = threadIdx.x; s < nsplit; s += 256) v += part[(size_t)s * n + i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dst[i] = red[0];
}

// Bias gradient partials: part[blk][c] = sum over the block's pixels of
// dz[p][c].  Thread t takes the 8-channel group t % G (G = C / 8) of pixels
// pb + t / G, pb + t / G + 256 / G, ... (16-byte loads); the 256 / G lanes of
// a group are then summed in LDS in a fixed order.
__global__ __launch_bounds__(256) void k_bias_grad(const bf16* __restrict__ dz, int P, int cs,
                                                   int C, int pper, float* __restrict__ part) {
  __shared__ float red[256 * 8];
  const int G = C / 8, R = 256 / G;
  const int t = threadIdx.x, g = t % G, r = t / G;
  const int pb = blockIdx.x * pper, pe = min(pb + pper, P);
  float v[8] = {};
  if (r < R)
    for (int p = pb + r; p < pe; p += R) {
      const V8 a = ld8(dz + (size_t)p * cs + 8 * g);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] += (float)a.h[e];
    }
#pragma unroll
  for (int e = 0; e < 8; ++e) red[t * 8 + e] = (r < R) ? v[e] : 0.0f;
  __syncthreads();
  if (t < C) {
    const int gg = t / 8, e = t % 8;
    float s = 0.0f;
    for (int rr = 0; rr < R; ++rr) s += red[(rr * G + gg) * 8 + e];
    part[(size_t)blockIdx.x * C + t] = s;
  }
}

// dz = dy where y > 0, else 0 (ReLU backward; y: the activated output).
__global__ void k_relu_bwd(const bf16* __restrict__ dy, int dy_cs, int dy_co,
                           const bf16* __restrict__ y, int y_cs, int y_co, bf16* __restrict__ dz,
                           int dz_cs, long P, int C) {
  const long n = P * C;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const long p = i / C;
    const int c = (int)(i - p * C);
    const float yv = (float)y[p * y_cs + y_co + c];
    dz[p * dz_cs + c] = yv > 0.0f ? dy[p * dy_cs + dy_co + c] : (bf16)0.0f;
  }
}

// 2x2 max pooling (stride 2) and its gradient (to the first maximum).
// Pooling and upsampling: thread i takes group i % (C / 8) of output pixel
// i / (C / 8).
// 2x2 max pooling, stride 2.
__global__ void k_maxpool2(const bf16* __restrict__ x, int x_cs, int x_co, bf16* __restrict__ y,
                           int y_cs, int B, int H, int W, int C) {
  const int Ho = H / 2, Wo = W / 2, G = C / 8;
  const int n = B * Ho * Wo * G;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int g = i % G, q = i / G;
    const int xo = q % Wo, t = q / Wo, yo = t % Ho, b = t / Ho;
    const size_t p0 = (size_t)(b * H + 2 * yo) * W + 2 * xo;
    const size_t px[4] = {p0, p0 + 1, p0 + W, p0 + W + 1};
    float m[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) m[e] = -3.0e38f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const V8 v = ld8(x + px[j] * x_cs + x_co + 8 * g);
#pragma unroll
      for (int e = 0; e < 8; ++e) m[e] = fmaxf(m[e], (float)v.h[e]);
    }
    V8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o.h[e] = (bf16)m[e];
    st8(y + (size_t)q * y_cs + 8 * g, o);
  }
}

// Its gradient: each window's gradient goes to its first maximum.
__global__ void k_maxpool2_bwd(const bf16* __restrict__ x, int x_cs, int x_co,
                               const bf16* __restrict__ dy, int dy_cs, bf16* __restrict__ dx,
                               int dx_cs, int dx_co, int accumulate, int B, int H, int W, int C) {
  const int Ho = H / 2, Wo = W / 2, G = C / 8;
  const int n = B * Ho * Wo * G;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int g = i % G, q = i / G;
    const int xo = q % Wo, t = q / Wo, yo = t % Ho, b = t / Ho;
    const size_t p0 = (size_t)(b * H + 2 * yo) * W + 2 * xo;
    const size_t px[4] = {p0, p0 + 1, p0 + W, p0 + W + 1};
    float m[8];
    int arg[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      m[e] = -3.0e38f;
      arg[e] = 0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const V8 v = ld8(x + px[j] * x_cs + x_co + 8 * g);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float f = (float)v.h[e];
        if (f > m[e]) {
          m[e] = f;
          arg[e] = j;
        }
      }
    }
    const V8 gv = ld8(dy + (size_t)q * dy_cs + 8 * g);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bf16* d = dx + px[j] * dx_cs + dx_co + 8 * g;
      V8 o = accumulate ? ld8(d) : V8{};
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float add = arg[e] == j ? (float)gv.h[e] : 0.0f;
        o.h[e] = (bf16)(accumulate ? (float)o.h[e] + add : add);
      }
      st8(d, o);
    }
  }
}

// Nearest 2x upsampling of a dense H x W x C image and its gradient (the sum
// of the four children).
__global__ void k_upsample2(const bf16* __restrict__ x, int B, int H, int W, int C,
                            bf16* __restrict__ y) {
  const int Ho = 2 * H, Wo = 2 * W, G = C / 8;
  const int n = B * Ho * Wo * G;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int g = i % G, q = i / G;
    const int xo = q % Wo, t = q / Wo, yo = t % Ho, b = t / Ho;
    st8(y + (size_t)q * C + 8 * g, ld8(x + ((size_t)(b * H + yo / 2) * W + xo / 2) * C + 8 * g));
  }
}

__global__ void k_upsample2_bwd(const bf16* __restrict__ dy, int B, int H, int W, int C,
                                bf16* __restrict__ dx) {
  const int G = C / 8;
  const int n = B * H * W * G;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int g = i % G, q = i / G;
    const int x = q % W, t = q / W, y = t % H, b = t / H;
    const size_t p0 = (size_t)(b * 2 * H + 2 * y) * (2 * W) + 2 * x;
    const size_t px[4] = {p0, p0 + 1, p0 + 2 * W, p0 + 2 * W + 1};
    float v[8] = {};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const V8 a = ld8(dy + px[j] * C + 8 * g);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] += (float)a.h[e];
    }
    V8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o.h[e] = (bf16)v[e];
    st8(dx + (size_t)q * C + 8 * g, o);
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, long n, uint32_t v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    p[i] = v;
}

// Mean squared error over the first C channels of out (FP32, channel stride
// out_cs) against target (FP32, C channels), channel c weighted by wch[c] (or
// 1); dout = d loss / d out (bf16, channel stride out_cs, zero beyond C);
// per-block loss partials in FP64.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out, int out_cs,
                                             const float* __restrict__ tgt, long P, int C,
                                             const float* __restrict__ wch,
                                             bf16* __restrict__ dout, double* __restrict__ part) {
  __shared__ double red[256];
  const double inv = 1.0 / ((double)P * C);
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < P * out_cs;
       i += (long)gridDim.x * blockDim.x) {
    const long p = i / out_cs;
    const int c = (int)(i - p * out_cs);
    float g = 0.0f;
    if (c < C) {
      const float wc = wch ? wch[c] : 1.0f;
      const float d = out[i] - tgt[p * C + c];
      acc += (double)wc * d * d;
      g = (float)(2.0 * inv) * wc * d;
    }
    if (dout) dout[i] = (bf16)g;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] * inv;
}

__global__ void k_sum_f64(const double* __restrict__ part, int n, double* __restrict__ dst) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *dst = s;
  }
}

// Sum of each of nplanes FP32 planes (plane k at src + k * stride, n values),
// one block per plane, FP64 in a fixed order (per-thread strided sums, then a
// tree over the block).
__global__ __launch_bounds__(256) void k_plane_sums(const float* __restrict__ src, long n,
                                                    long stride, double* __restrict__ out) {
  __shared__ double red[256];
  const float* p = src + blockIdx.x * stride;
  // four independent accumulators over 16-byte loads (the plane start is
  // 16-byte aligned when stride is a multiple of 4), then the scalar tail
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const bool vec = ((uintptr_t)p & 15) == 0;
  const long n4 = vec ? n / 4 : 0;
  const float4* p4 = reinterpret_cast<const float4*>(p);
#pragma unroll 4
  for (long i = threadIdx.x; i < n4; i += 256) {
    const float4 v = p4[i];
    a0 += (double)v.x;
    a1 += (double)v.y;
    a2 += (double)v.z;
    a3 += (double)v.w;
  }
  for (long i = 4 * n4 + threadIdx.x; i < n; i += 256) a0 += (double)p[i];
  red[threadIdx.x] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Phase-field budget term of a grid's state: the sum over its nodes of
// phi div u, with div u the isotropic D2Q9 stencil divergence that the step
// uses for the phase-field source (Sec. 3.1; stencil weights at the end of
// Sec. 3.4), x periodic, y periodic or closed by no-slip walls (ghost rows
// are the negated mirrors of the first and last rows).  Grid g's planes sit
// at planes + g * img_stride, plane f at f * nx * ny.  Block (p, g) sums the
// rows p, p + nparts, ... of grid g into part[g * nparts + p]; a second pass
// adds a grid's parts in order (FP64 throughout, fixed order).
__global__ __launch_bounds__(256) void k_phi_div_parts(const float* __restrict__ planes,
                                                       long img_stride, int nx, int ny, int walls,
                                                       int f_phi, int f_ux, int f_uy,
                                                       double* __restrict__ part) {
  __shared__ double red[256];
  const int nparts = gridDim.x, p = blockIdx.x, g = blockIdx.y;
  const long np = (long)nx * ny;
  const float* base = planes + (long)g * img_stride;
  const float* phi = base + (long)f_phi * np;
  const float* ux = base + (long)f_ux * np;
  const float* uy = base + (long)f_uy * np;
  double acc = 0.0;
  for (int y = p; y < ny; y += nparts) {
    // the rows below / above and the sign of their velocity (a ghost row
    // beyond a no-slip wall carries -u of the row it mirrors)
    int ym = y - 1, yp = y + 1;
    double sm = 1.0, sp = 1.0;
    if (y == 0) {
      ym = walls ? 0 : ny - 1;
      sm = walls ? -1.0 : 1.0;
    }
    if (y == ny - 1) {
      yp = walls ? ny - 1 : 0;
      sp = walls ? -1.0 : 1.0;
    }
    const long rm = (long)ym * nx, r0 = (long)y * nx, rp = (long)yp * nx;
    for (int x = threadIdx.x; x < nx; x += 256) {
      const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
      const double dux = (1.0 / 3.0) * ((double)ux[r0 + xp] - (double)ux[r0 + xm]) +
                         (1.0 / 12.0) * (sp * ux[rp + xp] + sm * ux[rm + xp] - sp * ux[rp + xm] -
                                         sm * ux[rm + xm]);
      const double duy = (1.0 / 3.0) * (sp * uy[rp + x] - sm * uy[rm + x]) +
                         (1.0 / 12.0) * (sp * uy[rp + xp] + sp * uy[rp + xm] - sm * uy[rm + xp] -
                                         sm * uy[rm + xm]);
      acc += (double)phi[r0 + x] * (dux + duy);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long)g * nparts + p] = red[0];
}

// out[g] = the nparts parts of grid g added in order (one thread per grid).
__global__ void k_sum_parts(const double* __restrict__ part, int nparts, int nimg,
                            double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nimg) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(long)g * nparts + p];
  out[g] = s;
}

// Plane `plane` of image i (at planes + i * img_stride + plane * n) times
// n / sums[i] (inverse = 0: the values over their mean) or sums[i] / n
// (inverse = 1: back), in place.
__global__ void k_scale_planes(float* __restrict__ planes, int nimg, long img_stride, int plane,
                               long n, const double* __restrict__ sums, int inverse) {
  const long total = (long)nimg * n;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total;
       k += (long)gridDim.x * blockDim.x) {
    const long i = k / n, j = k - i * n;
    const double s = sums[i];
    const float f = (float)(inverse ? s / (double)n : (double)n / s);
    float* v = planes + i * img_stride + (long)plane * n + j;
    *v = *v * f;
  }
}

// Adam on FP32 master weights (bias-corrected), then the bf16 copy.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, bf16* __restrict__ wb, long n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = (bf16)wi;
  }
}

__global__ void k_to_bf16(const float* __restrict__ s, bf16* __restrict__ d, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    d[i] = (bf16)s[i];
}

// Wt[c][t][n] = W[n][t][c]
__global__ void k_transpose_w(const bf16* __restrict__ w, int N, int taps, int C,
                              bf16* __restrict__ wt) {
  const long total = (long)N * taps * C;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const long r = i / C;
    const int t = (int)(r % taps), n = (int)(r / taps);
    wt[((long)c * taps + t) * N + n] = w[i];
  }
}

// Crop of FP32 field planes (nf planes of ny x nx, row-major) at (x0, y0),
// size S, normalised (v - shift[f]) * scale[f] into a bf16 NHWC tile of cs
// channels (channels nf .. cs-1 zero) for image b.  Periodic in x, clamped
// in y (the crops stay inside the grid in y).
__global__ void k_pack_fields(const float* __restrict__ planes, int nf, int nx, int ny, int x0,
                              int y0, int S, const float* __restrict__ shift,
                              const float* __restrict__ scale, bf16* __restrict__ dst, int cs,
                              int b) {
  const long n = (long)S * S;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const int x = (int)(i % S), y = (int)(i / S);
    const int gx = (x0 + x) % nx, gy = min(max(y0 + y, 0), ny - 1);
    bf16* d = dst + ((long)b * n + i) * cs;
    for (int f = 0; f < cs; ++f)
      d[f] = f < nf ? (bf16)((planes[(long)f * nx * ny + (long)gy * nx + gx] - shift[f]) * scale[f])
                    : (bf16)0.0f;
  }
}

// Target of a crop: ((after - resid[f] before) - shift[f]) * scale[f], FP32
// [S*S][nf] for image b (resid 1: the change is learned, 0: the new value).
__global__ void k_pack_delta(const float* __restrict__ after, const float* __restrict__ before,
                             int nf, int nx, int ny, int x0, int y0, int S,
                             const float* __restrict__ shift, const float* __restrict__ scale,
                             const float* __restrict__ resid, float* __restrict__ dst, int b) {
  const long n = (long)S * S;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const int x = (int)(i % S), y = (int)(i / S);
    const int gx = (x0 + x) % nx, gy = min(max(y0 + y, 0), ny - 1);
    for (int f = 0; f < nf; ++f) {
      const long o = (long)f * nx * ny + (long)gy * nx + gx;
      dst[((long)b * n + i) * nf + f] = ((after[o] - resid[f] * before[o]) - shift[f]) * scale[f];
    }
  }
}

// Prediction of a whole grid from the network output of image b (FP32,
// channel stride out_cs): pred[f] = resid[f] before[f] + out[f] / scale[f] +
// shift[f].
__global__ void k_apply_delta(const float* __restrict__ out, int out_cs,
                              const float* __restrict__ before, int nf, int nx, int ny,
                              const float* __restrict__ shift, const float* __restrict__ scale,
                              const float* __restrict__ resid, float* __restrict__ pred, int b) {
  const long n = (long)nx * ny;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    for (int f = 0; f < nf; ++f)
      pred[(long)f * n + i] = resid[f] * before[(long)f * n + i] +
                              out[((long)b * n + i) * out_cs + f] / scale[f] + shift[f];
}

// Whole S x S grids as network input, nimg at once: image i's nf FP32 planes
// at planes + i * img_stride (plane stride S * S), normalised, into image i
// of the bf16 NHWC tensor dst (cs channels, nf .. cs - 1 zero); one thread
// per pixel writes its cs channels as 16-byte groups.
__global__ void k_pack_images(const float* __restrict__ planes, int nimg, long img_stride, int nf,
                              int S, const float* __restrict__ shift,
                              const float* __restrict__ scale, bf16* __restrict__ dst, int cs) {
  const long npx = (long)S * S, n = npx * nimg;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const long img = i / npx, px = i - img * npx;
    const float* src = planes + img * img_stride + px;
    bf16* d = dst + i * cs;
    for (int g = 0; g < cs; g += 8) {
      V8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int f = g + e;
        v.h[e] = f < nf ? (bf16)((src[(long)f * npx] - shift[f]) * scale[f]) : (bf16)0.0f;
      }
      st8(d + g, v);
    }
  }
}

// Predictions of nimg whole grids from the network output: pred_i[f] =
// resid[f] before_i[f] + out_i[f] / scale[f] + shift[f] (planes of S * S at
// before + i * before_stride, pred + i * pred_stride).
__global__ void k_apply_images(const float* __restrict__ out, int out_cs,
                               const float* __restrict__ before, int nimg, long before_stride,
                               int nf, int S, const float* __restrict__ shift,
                               const float* __restrict__ scale, const float* __restrict__ resid,
                               float* __restrict__ pred, long pred_stride) {
  const long npx = (long)S * S, n = npx * nimg;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const long img = i / npx, px = i - img * npx;
    const float* o = out + i * out_cs;
    const float* bsrc = before + img * before_stride + px;
    float* p = pred + img * pred_stride + px;
    for (int f = 0; f < nf; ++f) p[(long)f * npx] = resid[f] * bsrc[(long)f * npx] + o[f] / scale[f] + shift[f];
  }
}

int grid_for(long n) { return (int)std::min<long>((n + 255) / 256, 16384); }

// 8-channel groups: C, the channel stride and the offset multiples of 8
bool groups_ok(int C, int cs, int co) {
  return C > 0 && C % 8 == 0 && cs % 8 == 0 && co % 8 == 0 && co + C <= cs;
}

}  // namespace

extern "C" {

#define HCHK()                                                \
  do {                                                        \
    return hipGetLastError() == hipSuccess ? 0 : LBFZ_NN_EHIP; \
  } while (0)

static bool conv_ok(const lbfz_conv_args* a) {
  return a && a->in && a->w && a->B > 0 && a->H > 0 && a->W > 0 && (a->taps == 1 || a->taps == 9) &&
         a->Cin > 0 && a->Cin % 8 == 0 && a->N > 0 && a->in_cs % 8 == 0 && a->in_co % 8 == 0 &&
         (a->up == 0 || (a->up == 1 && a->H % 2 == 0 && a->W % 2 == 0));
}

int lbfz_nn_conv_tail(const lbfz_conv_args* a, const lbfz_tail_args* t, void* stream) {
  if (!conv_ok(a) || !t || a->taps != 9 || a->sign != 1 || a->up || a->pool || a->out_f32 ||
      a->N != 32 || a->Cin % 32 != 0)
    return LBFZ_NN_EINVAL;
  if (a->out && (a->out_cs % 8 || a->out_co % 8 || a->out_co + a->N > a->out_cs))
    return LBFZ_NN_EINVAL;
  if (!t->head_w || !t->before || !t->shift || !t->scale || !t->resid || !t->pred ||
      t->nf < 1 || t->nf > t->nh || t->nh > 32)
    return LBFZ_NN_EINVAL;
  const long M = (long)a->B * a->H * a->W, npx = (long)a->H * a->W;
  if (M >= (1L << 30) || M * a->in_cs * 2 >= (1L << 31) || (long)a->N * 9 * a->Cin * 2 >= (1L << 31) ||
      t->before_stride < t->nf * npx || t->pred_stride < t->nf * npx)
    return LBFZ_NN_EINVAL;
  const long ty8 = (a->H + 7) / 8, tx = (a->W + TW - 1) / TW;
  hipLaunchKernelGGL(k_conv_tail, dim3((unsigned)(a->B * ty8 * tx)), dim3(256), 0,
                     (hipStream_t)stream, *a, *t);
  HCHK();
}

int lbfz_nn_conv(const lbfz_conv_args* a, void* stream) {
  if (!conv_ok(a) || !a->out || (a->sign != 1 && a->sign != -1) || (a->up && a->sign != 1))
    return LBFZ_NN_EINVAL;
  // fused pooling: 3 x 3, bf16 output written whole 16-byte groups, even sizes
  if (a->pool && (a->taps != 9 || a->out_f32 || a->N % 8 || a->out_cs % 8 || a->out_co % 8 ||
                  a->pool_cs % 8 || a->pool_co % 8 || a->pool_co + a->N > a->pool_cs ||
                  a->H % 2 || a->W % 2))
    return LBFZ_NN_EINVAL;
  const long M = (long)a->B * a->H * a->W;
  // operands are addressed with 32-bit byte offsets below 2^31
  if (M >= (1L << 30) || (a->up ? M / 4 : M) * a->in_cs * 2 >= (1L << 31) ||
      (long)a->N * a->taps * a->Cin * 2 >= (1L << 31))
    return LBFZ_NN_EINVAL;
  const hipStream_t st = (hipStream_t)stream;
  if (a->taps == 9) {
    // direct convolution: 64 output channels per block over 4 x 64 pixel
    // tiles when N is a multiple of 64; else 32 channels over 8 x 64 tiles
    // (two output rows per wave: one weight fragment serves four pixel
    // fragments)
    const long nb = a->B, ty4 = (a->H + 3) / 4, ty8 = (a->H + 7) / 8, tx = (a->W + TW - 1) / TW;
    const dim3 g64((unsigned)(nb * ty4 * tx), (unsigned)(a->N / 64));
    const dim3 g32((unsigned)(nb * ty8 * tx), (unsigned)((a->N + 31) / 32));
    const dim3 g32r1((unsigned)(nb * ty4 * tx), (unsigned)((a->N + 31) / 32));
    if (a->Cin % 32 != 0 && !a->up && a->sign == 1) {
      // 16-channel chunks: no half-empty chunk for e.g. a 16-channel input
      if (a->N % 64 == 0)
        hipLaunchKernelGGL((k_conv_direct<2, false, 1, 16>), g64, dim3(256), 0, st, *a);
      else
        hipLaunchKernelGGL((k_conv_direct<1, false, 1, 16>), g32r1, dim3(256), 0, st, *a);
    } else if (a->N % 64 == 0) {
      if (a->up)
        hipLaunchKernelGGL((k_conv_direct<2, true, 1>), g64, dim3(256), 0, st, *a);
      else if (a->sign == 1)
        hipLaunchKernelGGL((k_conv_direct<2, false, 1>), g64, dim3(256), 0, st, *a);
      else
        hipLaunchKernelGGL((k_conv_direct<2, false, -1>), g64, dim3(256), 0, st, *a);
    } else {
      if (a->up)
        hipLaunchKernelGGL((k_conv_direct<1, true, 1, 32, 2>), g32, dim3(256), 0, st, *a);
      else if (a->sign == 1)
        hipLaunchKernelGGL((k_conv_direct<1, false, 1, 32, 2>), g32, dim3(256), 0, st, *a);
      else
        hipLaunchKernelGGL((k_conv_direct<1, false, -1, 32, 2>), g32, dim3(256), 0, st, *a);
    }
    HCHK();
  }
  // 1 x 1: implicit GEMM, tile shape by output width: 128 x 128 (N a
  // multiple of 128), 256 x 64 (a multiple of 64), else 256 x 32
  if (a->N % 128 == 0) {
    const dim3 grid((unsigned)((M + 127) / 128), (unsigned)(a->N / 128));
    if (a->up)
      hipLaunchKernelGGL((k_conv<2, 2, 2, 2, true>), grid, dim3(256), 0, st, *a);
    else
      hipLaunchKernelGGL((k_conv<2, 2, 2, 2, false>), grid, dim3(256), 0, st, *a);
  } else if (a->N % 64 == 0) {
    const dim3 grid((unsigned)((M + 255) / 256), (unsigned)(a->N / 64));
    if (a->up)
      hipLaunchKernelGGL((k_conv<2, 2, 4, 1, true>), grid, dim3(256), 0, st, *a);
    else
      hipLaunchKernelGGL((k_conv<2, 2, 4, 1, false>), grid, dim3(256), 0, st, *a);
  } else {
    const dim3 grid((unsigned)((M + 255) / 256), (unsigned)((a->N + 31) / 32));
    if (a->up)
      hipLaunchKernelGGL((k_conv<2, 1, 4, 1, true>), grid, dim3(256), 0, st, *a);
    else
      hipLaunchKernelGGL((k_conv<2, 1, 4, 1, false>), grid, dim3(256), 0, st, *a);
  }
  HCHK();
}

int lbfz_nn_conv_wgrad(const lbfz_conv_args* a, float* part, int nsplit, float* dw,
                       void* stream) {
  if (!conv_ok(a) || !part || !dw || nsplit <= 0 || a->dz_cs % 8 != 0 || a->N % 8 != 0)
    return LBFZ_NN_EINVAL;
  const long P = (long)a->B * a->H * a->W;
  const int NW = a->taps * a->Cin;
  if (a->taps == 9) {
    if ((a->up ? P / 4 : P) * a->in_cs * 2 >= (1L << 31) || P * a->dz_cs * 2 >= (1L << 31))
      return LBFZ_NN_EINVAL;
    // direct form: blocks of 32 output x 32 input channels, each walking a
    // share of the pixel tiles (about 512 blocks in all, at most nsplit
    // shares: one partial row per share)
    const long tiles = (long)a->B * ((a->H + TH - 1) / TH) * ((a->W + TW - 1) / TW);
    const long cblk = (long)((a->N + 31) / 32) * ((a->Cin + 31) / 32);
    const int splits = (int)std::max<long>(
        1, std::min<long>(std::min<long>(nsplit, tiles), (512 + cblk - 1) / cblk));
    const dim3 grid((unsigned)splits, (unsigned)((a->N + 31) / 32),
                    (unsigned)((a->Cin + 31) / 32));
    if (a->up)
      hipLaunchKernelGGL((k_conv_wgrad_direct<true>), grid, dim3(256), 0, (hipStream_t)stream,
                         *a, part);
    else
      hipLaunchKernelGGL((k_conv_wgrad_direct<false>), grid, dim3(256), 0, (hipStream_t)stream,
                         *a, part);
    if (hipGetLastError() != hipSuccess) return LBFZ_NN_EHIP;
    const long n = (long)a->N * NW;
    const int rows = splits;
    if (n <= 16384)
      hipLaunchKernelGGL(k_sum_splits_small, dim3((unsigned)n), dim3(256), 0,
                         (hipStream_t)stream, part, rows, (int)n, dw);
    else
      hipLaunchKernelGGL(k_sum_splits, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                         part, rows, n, dw);
    HCHK();
  }
  long kper = (P + nsplit - 1) / nsplit;
  kper = (kper + BK - 1) / BK * BK;
  const int ns = (int)((P + kper - 1) / kper);
  const dim3 grid((unsigned)((a->N + BM - 1) / BM), (unsigned)((NW + BN - 1) / BN),
                  (unsigned)ns);
  hipLaunchKernelGGL(k_conv_wgrad, grid, dim3(256), 0, (hipStream_t)stream, *a, part, (int)kper);
  if (hipGetLastError() != hipSuccess) return LBFZ_NN_EHIP;
  const long n = (long)a->N * NW;
  if (n <= 16384)
    hipLaunchKernelGGL(k_sum_splits_small, dim3((unsigned)n), dim3(256), 0, (hipStream_t)stream,
                       part, ns, (int)n, dw);
  else
    hipLaunchKernelGGL(k_sum_splits, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, part,
                       ns, n, dw);
  HCHK();
}

int lbfz_nn_bias_grad(const void* dz, long P, int cs, int C, float* part, int nblocks, float* db,
                      void* stream) {
  if (!dz || !part || !db || !groups_ok(C, cs, 0) || C > 256 || nblocks <= 0 || P <= 0 ||
      P >= (1L << 31))
    return LBFZ_NN_EINVAL;
  const int pper = (int)((P + nblocks - 1) / nblocks);
  hipLaunchKernelGGL(k_bias_grad, dim3(nblocks), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(dz), (int)P, cs, C, pper, part);
  if (hipGetLastError() != hipSuccess) return LBFZ_NN_EHIP;
  hipLaunchKernelGGL(k_sum_splits_small, dim3(C), dim3(256), 0, (hipStream_t)stream, part,
                     nblocks, C, db);
  HCHK();
}

int lbfz_nn_relu_bwd(const void* dy, int dy_cs, int dy_co, const void* y, int y_cs, int y_co,
                     void* dz, int dz_cs, long P, int C, void* stream) {
  if (!dy || !y || !dz || P <= 0 || C <= 0) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_relu_bwd, dim3(grid_for(P * C)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(dy), dy_cs, dy_co, static_cast<const bf16*>(y),
                     y_cs, y_co, static_cast<bf16*>(dz), dz_cs, P, C);
  HCHK();
}

int lbfz_nn_maxpool2(const void* x, int x_cs, int x_co, void* y, int y_cs, int B, int H, int W,
                     int C, void* stream) {
  if (!x || !y || H % 2 || W % 2 || !groups_ok(C, x_cs, x_co) || !groups_ok(C, y_cs, 0))
    return LBFZ_NN_EINVAL;
  const long n = (long)B * (H / 2) * (W / 2) * (C / 8);
  if (n >= (1L << 31) || (long)B * H * W >= (1L << 31)) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_maxpool2, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(x), x_cs, x_co, static_cast<bf16*>(y), y_cs, B, H,
                     W, C);
  HCHK();
}

int lbfz_nn_maxpool2_bwd(const void* x, int x_cs, int x_co, const void* dy, int dy_cs, void* dx,
                         int dx_cs, int dx_co, int accumulate, int B, int H, int W, int C,
                         void* stream) {
  if (!x || !dy || !dx || H % 2 || W % 2 || !groups_ok(C, x_cs, x_co) ||
      !groups_ok(C, dy_cs, 0) || !groups_ok(C, dx_cs, dx_co))
    return LBFZ_NN_EINVAL;
  const long n = (long)B * (H / 2) * (W / 2) * (C / 8);
  if (n >= (1L << 31) || (long)B * H * W >= (1L << 31)) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_maxpool2_bwd, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(x), x_cs, x_co, static_cast<const bf16*>(dy), dy_cs,
                     static_cast<bf16*>(dx), dx_cs, dx_co, accumulate, B, H, W, C);
  HCHK();
}

int lbfz_nn_upsample2(const void* x, int B, int H, int W, int C, void* y, void* stream) {
  if (!x || !y || !groups_ok(C, C, 0)) return LBFZ_NN_EINVAL;
  const long n = (long)B * 4 * H * W * (C / 8);
  if (n >= (1L << 31) || (long)B * 4 * H * W >= (1L << 31)) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_upsample2, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(x), B, H, W, C, static_cast<bf16*>(y));
  HCHK();
}

int lbfz_nn_upsample2_bwd(const void* dy, int B, int H, int W, int C, void* dx, void* stream) {
  if (!dy || !dx || !groups_ok(C, C, 0)) return LBFZ_NN_EINVAL;
  const long n = (long)B * H * W * (C / 8);
  if (n >= (1L << 31) || (long)B * 4 * H * W >= (1L << 31)) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_upsample2_bwd, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(dy), B, H, W, C, static_cast<bf16*>(dx));
  HCHK();
}

int lbfz_nn_fill_u32(void* p, long n, uint32_t v, void* stream) {
  if (!p || n < 0) return LBFZ_NN_EINVAL;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<uint32_t*>(p), n, v);
  HCHK();
}

int lbfz_nn_mse(const float* out, int out_cs, const float* tgt, long P, int C, const float* wch,
                void* dout, double* part, int nblocks, double* loss, void* stream) {
  if (!out || !tgt || !part || !loss || C <= 0 || C > out_cs || nblocks <= 0)
    return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(256), 0, (hipStream_t)stream, out, out_cs, tgt, P,
                     C, wch, static_cast<bf16*>(dout), part);
  if (hipGetLastError() != hipSuccess) return LBFZ_NN_EHIP;
  hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(64), 0, (hipStream_t)stream, part, nblocks, loss);
  HCHK();
}

// Per-block partial sums of lbfz_nn_mse_noalloc: a fixed device array, so
// that the call needs no workspace from its caller.  In host code `scratch`
// is only a stand-in symbol; kernels get the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[LBFZ_NN_MSE_NOALLOC_MAX_BLOCKS];

// Device address of `scratch`, looked up once per device with that device
// current; nullptr when the lookup fails.
static double* scratch_ptr_for_current_device(int* err) {
  static std::mutex mu;
  static double* ptrs[256] = {};
  static bool looked[256] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 256) {
    *err = LBFZ_NN_EHIP;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!looked[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      *err = LBFZ_NN_EHIP;
      return nullptr;
    }
    ptrs[dev] = static_cast<double*>(p);
    looked[dev] = true;
  }
  return ptrs[dev];
}

int lbfz_nn_mse_noalloc(const float* out, int out_cs, const float* tgt, long P, int C,
                        const float* wch, void* dout, int nblocks, double* loss, void* stream) {
  if (!out || !tgt || !loss || C <= 0 || C > out_cs || nblocks <= 0)
    return LBFZ_NN_EINVAL;
  if (nblocks > LBFZ_NN_MSE_NOALLOC_MAX_BLOCKS) return LBFZ_NN_EINVAL;
  int err = 0;
  double* part = scratch_ptr_for_current_device(&err);
  if (!part) return err;
  // every one of the nblocks partial slots is written by k_mse before
  // k_sum_f64 reads it, so the array needs no clearing between calls
  hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(256), 0, (hipStream_t)stream, out, out_cs, tgt, P,
                     C, wch, static_cast<bf16*>(dout), part);
  if (hipGetLastError() != hipSuccess) return LBFZ_NN_EHIP;
  hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(64), 0, (hipStream_t)stream, part, nblocks, loss);
  HCHK();
}

int lbfz_nn_pack_images(const float* planes, int nimg, long img_stride, int nf, int S,
                        const float* shift, const float* scale, void* dst, int cs, void* stream) {
  if (!planes || !shift || !scale || !dst || nimg <= 0 || S <= 0 || nf <= 0 || nf > cs ||
      cs % 8 != 0 || img_stride < (long)nf * S * S)
    return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_pack_images, dim3(grid_for((long)nimg * S * S)), dim3(256), 0,
                     (hipStream_t)stream, planes, nimg, img_stride, nf, S, shift, scale,
                     static_cast<bf16*>(dst), cs);
  HCHK();
}

int lbfz_nn_apply_images(const float* out, int out_cs, const float* before, int nimg,
                         long before_stride, int nf, int S, const float* shift,
                         const float* scale, const float* resid, float* pred, long pred_stride,
                         void* stream) {
  if (!out || !before || !shift || !scale || !resid || !pred || nimg <= 0 || S <= 0 ||
      nf <= 0 || nf > out_cs || before_stride < (long)nf * S * S ||
      pred_stride < (long)nf * S * S)
    return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_apply_images, dim3(grid_for((long)nimg * S * S)), dim3(256), 0,
                     (hipStream_t)stream, out, out_cs, before, nimg, before_stride, nf, S, shift,
                     scale, resid, pred, pred_stride);
  HCHK();
}

int lbfz_nn_plane_sums(const float* src, int nplanes, long n, long stride, double* out,
                       void* stream) {
  if (!src || !out || nplanes <= 0 || n <= 0 || stride < n) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_plane_sums, dim3(nplanes), dim3(256), 0, (hipStream_t)stream, src, n,
                     stride, out);
  HCHK();
}

int lbfz_nn_phi_div_sums(const float* planes, int nimg, long img_stride, int nx, int ny,
                         int walls, int f_phi, int f_ux, int f_uy, double* parts, int nparts,
                         double* out, void* stream) {
  if (!planes || !parts || !out || nimg <= 0 || nx < 2 || ny < 2 || f_phi < 0 || f_ux < 0 ||
      f_uy < 0 || nparts < 1 || nparts > ny || nimg > 65535)
    return LBFZ_NN_EINVAL;
  const long np = (long)nx * ny;
  const int fmax = f_phi > f_ux ? (f_phi > f_uy ? f_phi : f_uy) : (f_ux > f_uy ? f_ux : f_uy);
  if (img_stride < (long)(fmax + 1) * np) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_phi_div_parts, dim3(nparts, nimg), dim3(256), 0, (hipStream_t)stream,
                     planes, img_stride, nx, ny, walls ? 1 : 0, f_phi, f_ux, f_uy, parts);
  hipLaunchKernelGGL(k_sum_parts, dim3((nimg + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     parts, nparts, nimg, out);
  HCHK();
}

int lbfz_nn_scale_planes(float* planes, int nimg, long img_stride, int plane, long n,
                         const double* sums, int inverse, void* stream) {
  if (!planes || !sums || nimg <= 0 || n <= 0 || plane < 0 ||
      (nimg > 1 && img_stride < (long)(plane + 1) * n))
    return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_scale_planes, dim3(grid_for((long)nimg * n)), dim3(256), 0,
                     (hipStream_t)stream, planes, nimg, img_stride, plane, n, sums,
                     inverse ? 1 : 0);
  HCHK();
}

int lbfz_nn_adam(float* w, const float* g, float* m, float* v, void* wb, long n, float lr,
                 float b1, float b2, float eps, int step, void* stream) {
  if (!w || !g || !m || !v || n <= 0 || step <= 0) return LBFZ_NN_EINVAL;
  const float c1 = 1.0f / (1.0f - powf(b1, (float)step));
  const float c2 = 1.0f / (1.0f - powf(b2, (float)step));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, w, g, m, v,
                     static_cast<bf16*>(wb), n, lr, b1, b2, eps, c1, c2);
  HCHK();
}

int lbfz_nn_to_bf16(const float* src, void* dst, long n, void* stream) {
  if (!src || !dst || n <= 0) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, src,
                     static_cast<bf16*>(dst), n);
  HCHK();
}

int lbfz_nn_transpose_w(const void* w, int N, int taps, int C, void* wt, void* stream) {
  if (!w || !wt || N <= 0 || C <= 0) return LBFZ_NN_EINVAL;
  const long n = (long)N * taps * C;
  hipLaunchKernelGGL(k_transpose_w, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(w), N, taps, C, static_cast<bf16*>(wt));
  HCHK();
}

int lbfz_nn_pack_fields(const float* planes, int nf, int nx, int ny, int x0, int y0, int S,
                        const float* shift, const float* scale, void* dst, int cs, int b,
                        void* stream) {
  if (!planes || !shift || !scale || !dst || nf > cs || S <= 0) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_pack_fields, dim3(grid_for((long)S * S)), dim3(256), 0,
                     (hipStream_t)stream, planes, nf, nx, ny, x0, y0, S, shift, scale,
                     static_cast<bf16*>(dst), cs, b);
  HCHK();
}

int lbfz_nn_pack_delta(const float* after, const float* before, int nf, int nx, int ny, int x0,
                       int y0, int S, const float* shift, const float* scale, const float* resid,
                       float* dst, int b, void* stream) {
  if (!after || !before || !shift || !scale || !resid || !dst || S <= 0) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_pack_delta, dim3(grid_for((long)S * S)), dim3(256), 0,
                     (hipStream_t)stream, after, before, nf, nx, ny, x0, y0, S, shift, scale,
                     resid, dst, b);
  HCHK();
}

int lbfz_nn_apply_delta(const float* out, int out_cs, const float* before, int nf, int nx, int ny,
                        const float* shift, const float* scale, const float* resid, float* pred,
                        int b, void* stream) {
  if (!out || !before || !shift || !scale || !resid || !pred) return LBFZ_NN_EINVAL;
  hipLaunchKernelGGL(k_apply_delta, dim3(grid_for((long)nx * ny)), dim3(256), 0,
                     (hipStream_t)stream, out, out_cs, before, nf, nx, ny, shift, scale, resid,
                     pred, b);
  HCHK();
}

}  // extern "C"
