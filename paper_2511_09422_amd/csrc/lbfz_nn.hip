// lbfz_nn.hip -- kernels of the learned surrogate of the LB step (a 3-level
// U-Net of 3x3 convolutions that maps the six fields of a 256^2 crop to their
// change over 64 steps), for gfx950.  C ABI in include/lbfz_nn.h.
//
// Tensors are NHWC bf16 (channels innermost, a multiple of 8), weights
// [out channel][tap][in channel] bf16 with FP32 master copies, accumulation in
// FP32.  Convolutions are implicit GEMMs on the BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16): a 256-thread block computes a 64 x 64 output
// tile as 2 x 2 waves of 32 x 32, staging 64 x 32 slices of both operands in
// LDS per K step.
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

#include "../../include/lbfz_nn.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 8;  // LDS rows padded by 16 B

__device__ __forceinline__ void tap_offset(int taps, int t, int sign, int& dy, int& dx) {
  if (taps == 1) {
    dy = dx = 0;
  } else {
    dy = sign * (t / 3 - 1);
    dx = sign * (t % 3 - 1);
  }
}

// 16 bytes (8 bf16) of channel data at pixel (b, y, x) shifted by (dy, dx);
// zero outside the image.
__device__ __forceinline__ uint4 load_px8(const bf16* __restrict__ t, int cs, int coff, int c,
                                          int b, int y, int x, int dy, int dx, int H, int W,
                                          bool ok) {
  const int yy = y + dy, xx = x + dx;
  if (!ok || yy < 0 || yy >= H || xx < 0 || xx >= W) return make_uint4(0, 0, 0, 0);
  const size_t o = ((size_t)(b * H + yy) * W + xx) * cs + coff + c;
  return *reinterpret_cast<const uint4*>(t + o);
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
__global__ __launch_bounds__(256) void k_conv(lbfz_conv_args a) {
  __shared__ __align__(16) bf16 As[BM][LDK];
  __shared__ __align__(16) bf16 Bs[BN][LDK];
  const int M = a.B * a.H * a.W, K = a.taps * a.Cin;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const bf16* __restrict__ in = static_cast<const bf16*>(a.in);
  const bf16* __restrict__ wt = static_cast<const bf16*>(a.w);
  // this thread's loader slot: tile row lr, 8 k values from lk
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  const int p = m0 + lr;
  const bool pok = p < M;
  const int px = p % a.W, py = (p / a.W) % a.H, pb = p / (a.W * a.H);
  const int n = n0 + lr;
  const bool nok = n < a.N;
  f32x16 acc = {};
  for (int k0 = 0; k0 < K; k0 += BK) {
    const int k = k0 + lk;
    uint4 va = make_uint4(0, 0, 0, 0), vb = make_uint4(0, 0, 0, 0);
    if (k < K) {
      const int t = k / a.Cin, c = k - t * a.Cin;
      int dy, dx;
      tap_offset(a.taps, t, a.sign, dy, dx);
      va = load_px8(in, a.in_cs, a.in_co, c, pb, py, px, dy, dx, a.H, a.W, pok);
      if (nok) vb = *reinterpret_cast<const uint4*>(wt + (size_t)n * K + k);
    }
    __syncthreads();
    *reinterpret_cast<uint4*>(&As[lr][lk]) = va;
    *reinterpret_cast<uint4*>(&Bs[lr][lk]) = vb;
    __syncthreads();
    acc = mfma_tile(As, Bs, wm, wn, lane, acc);
  }
  const float* bias = a.bias;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int pm = m0 + wm + acc_row(r, lane), cn = n0 + wn + (lane & 31);
    if (pm < M && cn < a.N) {
      float v = acc[r];
      if (bias) v += bias[cn];
      if (a.relu) v = fmaxf(v, 0.0f);
      const size_t o = (size_t)pm * a.out_cs + a.out_co + cn;
      if (a.out_f32)
        static_cast<float*>(a.out)[o] = v;
      else
        static_cast<bf16*>(a.out)[o] = (bf16)v;
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
    if (bn < NW) vb = load_px8(in, a.in_cs, a.in_co, bc, pb, py, px, bdy, bdx, a.H, a.W, pok);
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

// dst[i] = sum over s of part[s][i] (fixed order), optionally scaled.
__global__ void k_sum_splits(const float* __restrict__ part, int nsplit, long n,
                             float* __restrict__ dst) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    float v = 0.0f;
    for (int s = 0; s < nsplit; ++s) v += part[(size_t)s * n + i];
    dst[i] = v;
  }
}

// Bias gradient partials: part[blk][c] = sum over the block's pixels of dz[p][c].
__global__ __launch_bounds__(256) void k_bias_grad(const bf16* __restrict__ dz, int P, int cs,
                                                   int C, int pper, float* __restrict__ part) {
  const int c = threadIdx.x;
  if (c >= C) return;
  const int pb = blockIdx.x * pper, pe = min(pb + pper, P);
  float v = 0.0f;
  for (int p = pb; p < pe; ++p) v += (float)dz[(size_t)p * cs + c];
  part[(size_t)blockIdx.x * C + c] = v;
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
__global__ void k_maxpool2(const bf16* __restrict__ x, int x_cs, int x_co, bf16* __restrict__ y,
                           int y_cs, int B, int H, int W, int C) {
  const int Ho = H / 2, Wo = W / 2;
  const long n = (long)B * Ho * Wo * C;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const long q = i / C;
    const int xo = (int)(q % Wo), yo = (int)((q / Wo) % Ho), b = (int)(q / ((long)Wo * Ho));
    float m = -3.0e38f;
    for (int j = 0; j < 4; ++j) {
      const long px = ((long)(b * H + 2 * yo + (j >> 1)) * W + 2 * xo + (j & 1));
      m = fmaxf(m, (float)x[px * x_cs + x_co + c]);
    }
    y[q * y_cs + c] = (bf16)m;
  }
}

__global__ void k_maxpool2_bwd(const bf16* __restrict__ x, int x_cs, int x_co,
                               const bf16* __restrict__ dy, int dy_cs, bf16* __restrict__ dx,
                               int dx_cs, int dx_co, int accumulate, int B, int H, int W, int C) {
  const int Ho = H / 2, Wo = W / 2;
  const long n = (long)B * Ho * Wo * C;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const long q = i / C;
    const int xo = (int)(q % Wo), yo = (int)((q / Wo) % Ho), b = (int)(q / ((long)Wo * Ho));
    long px[4];
    int arg = 0;
    float m = -3.0e38f;
    for (int j = 0; j < 4; ++j) {
      px[j] = ((long)(b * H + 2 * yo + (j >> 1)) * W + 2 * xo + (j & 1));
      const float v = (float)x[px[j] * x_cs + x_co + c];
      if (v > m) {
        m = v;
        arg = j;
      }
    }
    const float g = (float)dy[q * dy_cs + c];
    for (int j = 0; j < 4; ++j) {
      bf16* d = dx + px[j] * dx_cs + dx_co + c;
      const float add = j == arg ? g : 0.0f;
      *d = (bf16)(accumulate ? (float)*d + add : add);
    }
  }
}

// Nearest 2x upsampling and its gradient (sum of the four children).
__global__ void k_upsample2(const bf16* __restrict__ x, int B, int H, int W, int C,
                            bf16* __restrict__ y) {
  const int Ho = 2 * H, Wo = 2 * W;
  const long n = (long)B * Ho * Wo * C;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const long q = i / C;
    const int xo = (int)(q % Wo), yo = (int)((q / Wo) % Ho), b = (int)(q / ((long)Wo * Ho));
    y[i] = x[((long)(b * H + yo / 2) * W + xo / 2) * C + c];
  }
}

__global__ void k_upsample2_bwd(const bf16* __restrict__ dy, int B, int H, int W, int C,
                                bf16* __restrict__ dx) {
  const long n = (long)B * H * W * C;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const long q = i / C;
    const int x = (int)(q % W), y = (int)((q / W) % H), b = (int)(q / ((long)W * H));
    float v = 0.0f;
    for (int j = 0; j < 4; ++j)
      v += (float)dy[((long)(b * 2 * H + 2 * y + (j >> 1)) * (2 * W) + 2 * x + (j & 1)) * C + c];
    dx[i] = (bf16)v;
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

int grid_for(long n) { return (int)std::min<long>((n + 255) / 256, 16384); }

}  // namespace

extern "C" {

#define HCHK()                                                \
  do {                                                        \
    return hipGetLastError() == hipSuccess ? 0 : LBFZ_NN_EHIP; \
  } while (0)

static bool conv_ok(const lbfz_conv_args* a) {
  return a && a->in && a->w && a->B > 0 && a->H > 0 && a->W > 0 && (a->taps == 1 || a->taps == 9) &&
         a->Cin > 0 && a->Cin % 8 == 0 && a->N > 0 && a->in_cs % 8 == 0 && a->in_co % 8 == 0;
}

int lbfz_nn_conv(const lbfz_conv_args* a, void* stream) {
  if (!conv_ok(a) || !a->out || (a->sign != 1 && a->sign != -1)) return LBFZ_NN_EINVAL;
  const long M = (long)a->B * a->H * a->W;
  const dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((a->N + BN - 1) / BN));
  hipLaunchKernelGGL(k_conv, grid, dim3(256), 0, (hipStream_t)stream, *a);
  HCHK();
}

int lbfz_nn_conv_wgrad(const lbfz_conv_args* a, float* part, int nsplit, float* dw,
                       void* stream) {
  if (!conv_ok(a) || !part || !dw || nsplit <= 0 || a->dz_cs % 8 != 0 || a->N % 8 != 0)
    return LBFZ_NN_EINVAL;
  const long P = (long)a->B * a->H * a->W;
  const int NW = a->taps * a->Cin;
  long kper = (P + nsplit - 1) / nsplit;
  kper = (kper + BK - 1) / BK * BK;
  const int ns = (int)((P + kper - 1) / kper);
  const dim3 grid((unsigned)((a->N + BM - 1) / BM), (unsigned)((NW + BN - 1) / BN),
                  (unsigned)ns);
  hipLaunchKernelGGL(k_conv_wgrad, grid, dim3(256), 0, (hipStream_t)stream, *a, part, (int)kper);
  if (hipGetLastError() != hipSuccess) return LBFZ_NN_EHIP;
  const long n = (long)a->N * NW;
  hipLaunchKernelGGL(k_sum_splits, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, part,
                     ns, n, dw);
  HCHK();
}

int lbfz_nn_bias_grad(const void* dz, long P, int cs, int C, float* part, int nblocks, float* db,
                      void* stream) {
  if (!dz || !part || !db || C <= 0 || C > 256 || nblocks <= 0) return LBFZ_NN_EINVAL;
  const int pper = (int)((P + nblocks - 1) / nblocks);
  hipLaunchKernelGGL(k_bias_grad, dim3(nblocks), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(dz), (int)P, cs, C, pper, part);
  if (hipGetLastError() != hipSuccess) return LBFZ_NN_EHIP;
  hipLaunchKernelGGL(k_sum_splits, dim3(1), dim3(256), 0, (hipStream_t)stream, part, nblocks,
                     (long)C, db);
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
  if (!x || !y || H % 2 || W % 2 || C <= 0) return LBFZ_NN_EINVAL;
  const long n = (long)B * (H / 2) * (W / 2) * C;
  hipLaunchKernelGGL(k_maxpool2, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(x), x_cs, x_co, static_cast<bf16*>(y), y_cs, B, H,
                     W, C);
  HCHK();
}

int lbfz_nn_maxpool2_bwd(const void* x, int x_cs, int x_co, const void* dy, int dy_cs, void* dx,
                         int dx_cs, int dx_co, int accumulate, int B, int H, int W, int C,
                         void* stream) {
  if (!x || !dy || !dx || H % 2 || W % 2 || C <= 0) return LBFZ_NN_EINVAL;
  const long n = (long)B * (H / 2) * (W / 2) * C;
  hipLaunchKernelGGL(k_maxpool2_bwd, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(x), x_cs, x_co, static_cast<const bf16*>(dy), dy_cs,
                     static_cast<bf16*>(dx), dx_cs, dx_co, accumulate, B, H, W, C);
  HCHK();
}

int lbfz_nn_upsample2(const void* x, int B, int H, int W, int C, void* y, void* stream) {
  if (!x || !y || C <= 0) return LBFZ_NN_EINVAL;
  const long n = (long)B * 4 * H * W * C;
  hipLaunchKernelGGL(k_upsample2, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const bf16*>(x), B, H, W, C, static_cast<bf16*>(y));
  HCHK();
}

int lbfz_nn_upsample2_bwd(const void* dy, int B, int H, int W, int C, void* dx, void* stream) {
  if (!dy || !dx || C <= 0) return LBFZ_NN_EINVAL;
  const long n = (long)B * H * W * C;
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
