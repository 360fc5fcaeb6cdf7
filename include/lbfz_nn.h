/*
 * lbfz_nn.h -- C ABI of the kernels of the learned surrogate of the coupled
 * LB freezing step (arXiv 2511.09422): a 3-level U-Net of 3x3 convolutions
 * (32 / 64 / 128 channels, ReLU, 2x2 max pooling, nearest 2x upsampling,
 * skip connections by channel concatenation, a 1x1 head) that maps the six
 * fields phi, f_l, T, C, u_x, u_y of a crop of the 2D step to their change
 * over 64 steps.  The paper itself has no learned component; the surrogate
 * screens parameter sweeps of its model, with the LB step as the reference.
 *
 * Conventions (all calls):
 *   - Activations and gradients: bf16, NHWC (pixel-major, channels
 *     innermost), images B x H x W.  A tensor argument is (pointer, channel
 *     stride cs, channel offset co): channels co .. co + C - 1 of every pixel,
 *     pixels cs elements apart.  Channel counts, strides and offsets of
 *     convolution operands are multiples of 8; pointers are 16-byte aligned.
 *   - Weights: bf16 [N][taps][Cin] (taps 9: a 3x3 stencil with zero padding,
 *     tap t at offset (t / 3 - 1, t % 3 - 1); taps 1: a 1x1 convolution); FP32
 *     master weights, gradients and optimiser state.  Accumulation in FP32 on
 *     the BF16 matrix cores.
 *   - Device pointers only; the library allocates nothing.  Every call is
 *     asynchronous on `stream` (a hipStream_t, NULL = default stream) and
 *     returns 0 or a negative code: LBFZ_NN_EINVAL for an invalid argument,
 *     LBFZ_NN_EHIP when a launch fails.
 */
#ifndef LBFZ_NN_H
#define LBFZ_NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LBFZ_NN_OK = 0, LBFZ_NN_EINVAL = -1, LBFZ_NN_EHIP = -3 };

/* Operands of a convolution. */
typedef struct lbfz_conv_args {
  const void* in;          /* forward: the layer input x; data gradient: dz (gradient at the
                              layer's pre-activation); weight gradient: the layer input x   */
  int32_t in_cs, in_co;    /* channel stride / offset of `in`                              */
  int32_t Cin;             /* channels contracted per tap (forward / weight gradient: the
                              layer's input channels; data gradient: its output channels) */
  const void* w;           /* forward: W [N][taps][Cin]; data gradient: the transposed
                              weights Wt [N][taps][Cin] (lbfz_nn_transpose_w); weight
                              gradient: dz (N channels, channel stride dz_cs)             */
  int32_t dz_cs;           /* weight gradient only                                         */
  int32_t N;               /* output channels (weight gradient: the layer's outputs)       */
  const float* bias;       /* forward: bias [N] or NULL; else NULL                         */
  void* out;               /* forward / data gradient output (bf16, or FP32 if out_f32)    */
  int32_t out_cs, out_co, out_f32;
  int32_t relu;            /* forward: apply max(., 0) after the bias                      */
  int32_t sign;            /* +1 forward (x at p + o(t)), -1 data gradient (dz at p - o(t)) */
  int32_t B, H, W, taps;
  int32_t up;              /* forward / weight gradient: 1 = `in` is a B x (H/2) x (W/2)
                              image read through nearest 2x upsampling (pixel (y, x) takes
                              (y/2, x/2); H, W even), 0 = `in` is B x H x W.  Must be 0 for
                              the data gradient                                             */
  void* pool;              /* 3 x 3 forward / data gradient with bf16 output: if not NULL,
                              also write the 2x2 max pooling (stride 2) of the stored output
                              here, a B x (H/2) x (W/2) image of N channels at channel
                              stride pool_cs, offset pool_co (H, W even; as lbfz_nn_maxpool2
                              of `out`, bit for bit)                                          */
  int32_t pool_cs, pool_co;
} lbfz_conv_args;

/* Forward: out[p][n] = act(sum_{t,c} in[p + o(t)][c] W[n][t][c] + bias[n]);
 * data gradient (sign -1, w = Wt): out[p][c'] = sum_{t,n} dz[p - o(t)][n]
 * W[n][t][c'].  Implicit GEMM, M = pixels, N = a->N, K = taps * Cin. */
int lbfz_nn_conv(const lbfz_conv_args* a, void* stream);

/* The network's tail at inference, fused into one launch: the last 3 x 3
 * convolution `a` (forward, bias, ReLU, bf16 activations, a->N == 32 output
 * channels, a->Cin a multiple of 32, no upsampling, no pooling), the 1 x 1
 * head over its 32 outputs, and the prediction of whole grids as
 * lbfz_nn_apply_images computes it, without writing the head's input or
 * output to memory (a->out may be NULL; if not, the convolution's output is
 * stored as lbfz_nn_conv stores it).  The head's input is the convolution's
 * output rounded to bf16, as the unfused network stores it; the head's dot
 * products are FP32 in channel order (the unfused head's matrix-core sums
 * round differently, by about 1e-7 of the largest term).  Image i of the
 * convolution is grid i: its nf FP32 planes at before + i * before_stride,
 * its prediction at pred + i * pred_stride (a->H x a->W values per plane). */
typedef struct lbfz_tail_args {
  const void* head_w;      /* bf16 [nh][32]: the head's weights over the 32 channels */
  const float* head_b;     /* [nh] or NULL */
  int32_t nh;              /* head outputs (nf <= nh <= 32); outputs nf .. nh - 1 unused */
  int32_t nf;              /* fields predicted                                           */
  const float* before;     /* fields of the grids before the stride                      */
  int64_t before_stride;
  const float* shift;      /* device arrays of nf floats: pred[f] = resid[f] before[f] +  */
  const float* scale;      /*   head[f] / scale[f] + shift[f]                             */
  const float* resid;
  float* pred;
  int64_t pred_stride;
} lbfz_tail_args;
int lbfz_nn_conv_tail(const lbfz_conv_args* a, const lbfz_tail_args* t, void* stream);

/* Weight gradient dw[n][t][c] = sum_p dz[p][n] x[p + o(t)][c], FP32.  The
 * pixel sum is split into at most nsplit partial rows in part (nsplit * N *
 * taps * Cin floats; 3 x 3: up to about 512 / (ceil(N/32) ceil(Cin/32))
 * rows are used, 1 x 1: nsplit), then summed in a fixed order
 * (deterministic). */
int lbfz_nn_conv_wgrad(const lbfz_conv_args* a, float* part, int nsplit, float* dw, void* stream);

/* Bias gradient db[c] = sum_p dz[p][c] (C <= 256 channels at stride cs, both
 * multiples of 8), via nblocks partial rows in part (nblocks * C floats),
 * summed in a fixed order. */
int lbfz_nn_bias_grad(const void* dz, long P, int cs, int C, float* part, int nblocks, float* db,
                      void* stream);

/* ReLU backward: dz = dy where y > 0 else 0 (y: the activated output). */
int lbfz_nn_relu_bwd(const void* dy, int dy_cs, int dy_co, const void* y, int y_cs, int y_co,
                     void* dz, int dz_cs, long P, int C, void* stream);

/* 2x2 max pooling (stride 2) and its gradient (to the first maximum of each
 * window; accumulate != 0 adds into dx instead of overwriting).  C, channel
 * strides and offsets multiples of 8; H, W even. */
int lbfz_nn_maxpool2(const void* x, int x_cs, int x_co, void* y, int y_cs, int B, int H, int W,
                     int C, void* stream);
int lbfz_nn_maxpool2_bwd(const void* x, int x_cs, int x_co, const void* dy, int dy_cs, void* dx,
                         int dx_cs, int dx_co, int accumulate, int B, int H, int W, int C,
                         void* stream);

/* Nearest 2x upsampling of a dense B x H x W x C tensor (to 2H x 2W) and its
 * gradient (the sum over each 2x2 block); C a multiple of 8. */
int lbfz_nn_upsample2(const void* x, int B, int H, int W, int C, void* y, void* stream);
int lbfz_nn_upsample2_bwd(const void* dy, int B, int H, int W, int C, void* dx, void* stream);

/* n 32-bit words of p set to v (clears buffers without a runtime memset). */
int lbfz_nn_fill_u32(void* p, long n, uint32_t v, void* stream);

/* Mean squared error over the first C channels of out (FP32, stride out_cs)
 * against tgt (FP32, C channels per pixel), channel c weighted by wch[c]
 * (device array, or NULL for 1), into *loss (FP64, via nblocks partials in
 * part); dout (bf16, stride out_cs, or NULL) = d loss / d out. */
int lbfz_nn_mse(const float* out, int out_cs, const float* tgt, long P, int C, const float* wch,
                void* dout, double* part, int nblocks, double* loss, void* stream);

/* lbfz_nn_mse without a caller-provided partial-sum buffer, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops
 * that forbid hipMalloc).  The nblocks FP64 partials live in a fixed array of
 * LBFZ_NN_MSE_NOALLOC_MAX_BLOCKS doubles (32 KiB) inside the library, one per
 * GPU, held until the process ends; the call allocates nothing.  Results are
 * those of lbfz_nn_mse with the same nblocks.  Errors: LBFZ_NN_EINVAL for
 * nblocks outside 1 .. LBFZ_NN_MSE_NOALLOC_MAX_BLOCKS or the arguments
 * lbfz_nn_mse rejects; LBFZ_NN_EHIP if the array's device address cannot be
 * found or a launch fails.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (different streams, or host threads) race
 * and must be serialised by the caller. */
#define LBFZ_NN_MSE_NOALLOC_MAX_BLOCKS 4096
int lbfz_nn_mse_noalloc(const float* out, int out_cs, const float* tgt, long P, int C,
                        const float* wch, void* dout, int nblocks, double* loss, void* stream);

/* One Adam step (bias-corrected with the 1-based step number) on n FP32
 * weights w with gradients g and moments m, v; wb (bf16, or NULL) receives
 * the updated weights. */
int lbfz_nn_adam(float* w, const float* g, float* m, float* v, void* wb, long n, float lr,
                 float b1, float b2, float eps, int step, void* stream);

int lbfz_nn_to_bf16(const float* src, void* dst, long n, void* stream);

/* Network input from nimg whole S x S grids at once: image i's nf FP32
 * planes at planes + i * img_stride (each S * S values), normalised as in
 * lbfz_nn_pack_fields, into images 0 .. nimg - 1 of dst (cs channels, a
 * multiple of 8). */
int lbfz_nn_pack_images(const float* planes, int nimg, long img_stride, int nf, int S,
                        const float* shift, const float* scale, void* dst, int cs, void* stream);

/* Predictions of nimg whole grids (as lbfz_nn_apply_delta for each image):
 * before / pred planes of grid i at before + i * before_stride and pred + i *
 * pred_stride. */
int lbfz_nn_apply_images(const float* out, int out_cs, const float* before, int nimg,
                         long before_stride, int nf, int S, const float* shift,
                         const float* scale, const float* resid, float* pred, long pred_stride,
                         void* stream);

/* out[k] = sum of the n FP32 values of plane k (at src + k * stride), k <
 * nplanes, accumulated in FP64 in a fixed order (the per-grid sums of the
 * screening check). */
int lbfz_nn_plane_sums(const float* src, int nplanes, long n, long stride, double* out,
                       void* stream);

/* Phase-field budget term of nimg grids of nx x ny nodes: out[g] = sum over
 * the nodes of phi * div u (FP64, fixed order), with div u the isotropic
 * D2Q9 stencil divergence the step uses for the phase-field source (Sec. 3.1;
 * stencil weights at the end of Sec. 3.4).  Grid g's FP32 planes at planes +
 * g * img_stride, plane f at f * nx * ny: phi is plane f_phi, u_x plane f_ux,
 * u_y plane f_uy.  x periodic; y periodic (walls = 0) or closed by no-slip
 * walls (walls != 0: the ghost rows carry -u of the rows they mirror).  The
 * screening check integrates it over a stride (trapezoid rule) to predict
 * the change of sum phi.  Each grid is summed in nparts interleaved row sets
 * into the caller's parts buffer (nimg * nparts doubles, overwritten), then
 * the parts are added in order.  Device pointers; out holds nimg doubles.
 * EINVAL for null pointers, nimg outside 1 .. 65535, a side below 2, nparts
 * outside 1 .. ny, a negative plane index or img_stride shorter than the
 * highest plane used. */
int lbfz_nn_phi_div_sums(const float* planes, int nimg, long img_stride, int nx, int ny,
                         int walls, int f_phi, int f_ux, int f_uy, double* parts, int nparts,
                         double* out, void* stream);

/* In place, plane `plane` of image i (n FP32 values at planes + i *
 * img_stride + plane * n) times n / sums[i] (inverse = 0: the values over
 * their mean, with sums[i] the plane's sum) or sums[i] / n (inverse != 0:
 * back), for i < nimg.  The surrogate keeps a grid's solute over its mean
 * (the step conserves the solute, Sec. 3.4, so the mean is the grid's own
 * constant): the network then sees every grid's solute on one scale.
 * Device pointers (sums: nimg doubles).  EINVAL for null pointers, nimg < 1,
 * n < 1, a negative plane or, with more than one image, img_stride shorter
 * than the planes up to `plane`. */
int lbfz_nn_scale_planes(float* planes, int nimg, long img_stride, int plane, long n,
                         const double* sums, int inverse, void* stream);

/* Wt[c][t][n] = W[n][t][c] (weights of the data-gradient convolution). */
int lbfz_nn_transpose_w(const void* w, int N, int taps, int C, void* wt, void* stream);

/* Network input from solver fields: nf FP32 planes of ny x nx (row-major),
 * the S x S crop at (x0, y0) (periodic in x, clamped in y), normalised as
 * (v - shift[f]) * scale[f], into image b of a bf16 NHWC tensor of cs
 * channels (channels nf .. cs - 1 zero). */
int lbfz_nn_pack_fields(const float* planes, int nf, int nx, int ny, int x0, int y0, int S,
                        const float* shift, const float* scale, void* dst, int cs, int b,
                        void* stream);

/* Training target of the same crop: ((after - resid[f] before) - shift[f]) *
 * scale[f], FP32 [S * S][nf] for image b; resid[f] = 1 learns the change of
 * field f, 0 its new value (device arrays of nf floats). */
int lbfz_nn_pack_delta(const float* after, const float* before, int nf, int nx, int ny, int x0,
                       int y0, int S, const float* shift, const float* scale, const float* resid,
                       float* dst, int b, void* stream);

/* Prediction of a whole grid from image b of the network output (FP32, stride
 * out_cs, the grid itself as the image): pred[f] = resid[f] before[f] +
 * out[f] / scale[f] + shift[f], nf planes. */
int lbfz_nn_apply_delta(const float* out, int out_cs, const float* before, int nf, int nx, int ny,
                        const float* shift, const float* scale, const float* resid, float* pred,
                        int b, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBFZ_NN_H */
