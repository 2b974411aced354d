/*
 * eik_unet.h -- C ABI of the learned warm start's kernels (gfx950, BF16 MFMA).
 *
 * The warm start is a component added to the method (not in the paper): a small
 * U-Net maps per-node inputs (metric, drift, Euclidean distance to the nearest
 * source) to a prediction of T that replaces the +inf initialisation of the
 * forward solve (eik_forward's T_init; the sweep overwrites, so the prediction
 * needs no upper-bound property), and the cold start remains the fallback.
 *
 * Tensors are NHWC with the batch folded into the pixel index: pixel
 * p = (b H + y) W + x, element (p, c) at p * cs + co + c, where cs is the
 * buffer's channel stride and co a channel offset. A concatenation of two
 * producers' outputs is either two disjoint channel ranges of one buffer, or
 * two buffers read by the _cat forms below (each producer then writes whole
 * pixels, which interleaved channel ranges of one buffer do not). Activations and
 * weights are bfloat16 (raw uint16 bits); accumulation is FP32; weight and bias
 * gradients are FP32 and are accumulated (callers zero them first).
 * All pointers are device memory owned by the caller; calls enqueue on the
 * stream and return 0, or -1 for an invalid argument (nothing launched).
 *
 * Convolution modes (the GEMM "pixel grid" is B x H x W in every mode):
 *   EIKU_CONV3  3x3, stride 1, zero padding 1: y(p) = sum_{tap, ci} x(p + d_tap) W[tap][co][ci]
 *               with d_tap = (tap/3 - 1, tap%3 - 1) in (y, x);
 *   EIKU_UP2    2x2 transposed convolution, stride 2: input grid B x H x W, output
 *               grid B x 2H x 2W, y(2y+a, 2x+c) = sum_ci x(y, x) W[2a+c][co][ci];
 *   EIKU_DOWN2  the data-gradient of EIKU_UP2: input grid B x 2H x 2W, output grid
 *               B x H x W, y(p) = sum_{a, c, ci} x(2y+a, 2x+c) W[2a+c][co][ci].
 * Cin and Cout must be multiples of 16 (pad channels with zeros). The
 * convolutions and the 3x3 weight gradient move 8 channels per 16-byte
 * access: x (and dy) channel strides and offsets must be multiples of 8 and
 * x, w (dy) 16-byte aligned; y strides and offsets multiples of 4 and y
 * 8-byte aligned. Other layouts are rejected with -1.
 */
#ifndef EIK_UNET_H
#define EIK_UNET_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { EIKU_CONV3 = 0, EIKU_UP2 = 1, EIKU_DOWN2 = 2 };

/* y = act(conv(x) + bias); act = ReLU when relu != 0; bias may be NULL. */
int eiku_conv_fwd(int32_t mode, int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t x_cs, int32_t x_co,
                  int32_t Cin, const uint16_t *w, const float *bias, int32_t relu, uint16_t *y, int32_t y_cs,
                  int32_t y_co, int32_t Cout, hipStream_t stream);

/* dW[tap][co][ci] += sum_p dy(p_out, co) x(p_in, ci) for EIKU_CONV3 / EIKU_UP2
 * (the pixel pairs of the forward mode); dw is FP32. */
int eiku_conv_wgrad(int32_t mode, int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t x_cs, int32_t x_co,
                    int32_t Cin, const uint16_t *dy, int32_t dy_cs, int32_t dy_co, int32_t Cout, float *dw,
                    hipStream_t stream);

/* EIKU_CONV3 of the concatenation [xa | xb]: input channels 0 .. Ca-1 are
 * xa's (channel xa_co + c of a pixel), Ca .. Ca+Cb-1 are xb's (channel
 * xb_co + c - Ca); w is [9][Cout][Ca+Cb] as for eiku_conv_fwd, and the result
 * is that of eiku_conv_fwd on one buffer holding the concatenation. Ca and Cb
 * are multiples of 16; both sources follow x's stride, offset and alignment
 * rules. */
int eiku_conv_fwd_cat(int32_t B, int32_t H, int32_t W, const uint16_t *xa, int32_t xa_cs, int32_t xa_co, int32_t Ca,
                      const uint16_t *xb, int32_t xb_cs, int32_t xb_co, int32_t Cb, const uint16_t *w,
                      const float *bias, int32_t relu, uint16_t *y, int32_t y_cs, int32_t y_co, int32_t Cout,
                      hipStream_t stream);

/* The EIKU_CONV3 weight gradient with x the concatenation [xa | xb], as in
 * eiku_conv_fwd_cat; dw is [9][Cout][Ca+Cb], FP32, accumulated. */
int eiku_conv_wgrad_cat(int32_t B, int32_t H, int32_t W, const uint16_t *xa, int32_t xa_cs, int32_t xa_co,
                        int32_t Ca, const uint16_t *xb, int32_t xb_cs, int32_t xb_co, int32_t Cb, const uint16_t *dy,
                        int32_t dy_cs, int32_t dy_co, int32_t Cout, float *dw, hipStream_t stream);

/* db[c] += sum_p dy(p, c) over npix pixels. */
int eiku_bias_grad(int64_t npix, const uint16_t *dy, int32_t cs, int32_t co, int32_t C, float *db,
                   hipStream_t stream);

/* In place: g(p, c) = 0 where y(p, c) <= 0 (ReLU backward). */
int eiku_relu_mask(int64_t npix, const uint16_t *y, int32_t y_cs, int32_t y_co, uint16_t *g, int32_t g_cs,
                   int32_t g_co, int32_t C, hipStream_t stream);

/* a(p, c) += b(p, c). */
int eiku_add(int64_t npix, uint16_t *a, int32_t a_cs, int32_t a_co, const uint16_t *b, int32_t b_cs, int32_t b_co,
             int32_t C, hipStream_t stream);

/* 2x2 max pooling: input B x 2H x 2W, output B x H x W; backward writes every
 * input gradient (the position of the maximum receives dy, the others 0). */
int eiku_maxpool_fwd(int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t x_cs, int32_t x_co, uint16_t *y,
                     int32_t y_cs, int32_t y_co, int32_t C, hipStream_t stream);
int eiku_maxpool_bwd(int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t x_cs, int32_t x_co,
                     const uint16_t *dy, int32_t dy_cs, int32_t dy_co, uint16_t *dx, int32_t dx_cs, int32_t dx_co,
                     int32_t C, hipStream_t stream);

/* 1x1 output head: out(p) = b + sum_c w[c] x(p, c) in FP32; backward:
 * dx(p, c) = w[c] g(p), dw[c] += sum_p g(p) x(p, c), db += sum_p g(p). */
int eiku_head_fwd(int64_t npix, const uint16_t *x, int32_t cs, int32_t co, int32_t C, const float *w, const float *b,
                  float *out, hipStream_t stream);
int eiku_head_bwd(int64_t npix, const uint16_t *x, int32_t cs, int32_t co, int32_t C, const float *w, const float *g,
                  uint16_t *dx, int32_t dx_cs, int32_t dx_co, float *dw, float *db, hipStream_t stream);

/* Network inputs for B grids of H x W nodes (spacing h[b]): channels m11, m12,
 * m22, bx, by, Euclidean distance to the nearest source, zeros up to cs = 16.
 * M [B][3][H][W] and omega [B][2][H][W] are FP32; src [B][max_src] holds flat
 * node indices, negative entries unused; x is 16-byte aligned. */
int eiku_features(int32_t B, int32_t H, int32_t W, const float *M, const float *omega, const int32_t *src,
                  int32_t max_src, const float *h, uint16_t *x, float *dist, hipStream_t stream);

/* Mean squared error over n values: loss[0] += mean((p - t)^2), grad = 2 (p - t) / n. */
int eiku_mse(int64_t n, const float *pred, const float *target, float *loss, float *grad, hipStream_t stream);

/* Adam step on n FP32 parameters (bias-corrected with step t >= 1); the
 * gradient is cleared afterwards. */
int eiku_adam(int64_t n, float *param, float *grad, float *m, float *v, float lr, float beta1, float beta2, float eps,
              int32_t t, hipStream_t stream);

/* FP32 master weights [taps][Cout][cin_real] -> BF16 forward weights
 * [taps][Cout][Cin] (channels cin_real..Cin-1 zero) and the weights of the
 * data-gradient pass: EIKU_CONV3 -> [9][Cin][Cout] with the taps mirrored,
 * EIKU_UP2 -> [4][Cin][Cout] (for EIKU_DOWN2). wbwd may be NULL. */
int eiku_prep_weights(int32_t mode, int32_t taps, int32_t Cout, int32_t Cin, int32_t cin_real, const float *w32,
                      uint16_t *wfwd, uint16_t *wbwd, hipStream_t stream);

/* FP32 <-> BF16 conversion of n values. */
int eiku_to_bf16(int64_t n, const float *x, uint16_t *y, hipStream_t stream);
int eiku_to_f32(int64_t n, const uint16_t *x, float *y, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* EIK_UNET_H */
