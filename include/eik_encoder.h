/*
 * eik_encoder.h -- C ABI of the covariate encoder's own kernels (Sec. 6,
 * encoder architecture; App. wildfire experiments, training protocol): the
 * global pathway's dense layers and the combination of the global baseline
 * with the spatial residuals,
 *   G(x) = G0 + alpha G_local(x),  b(x) = b0 + alpha b_local(x),
 * before the feasibility projection (eik_project). The spatial pathway (3x3
 * convolutions, ReLU, 1x1 heads) runs in the BF16 MFMA kernels of
 * eik_unet.h; the solve and the implicit gradient of the data term in
 * eik_forward / eik_backward.
 *
 * All pointers are device memory owned by the caller; every call enqueues
 * work on `stream`, never synchronises and never allocates. Dense layers are
 * FP32 with FP32 accumulation in a fixed order; the reductions of
 * eik_enc_combine_backward are deterministic (fixed blocks, fixed-order tree,
 * accumulated in double). Errors: EIK_EINVAL (bad sizes, NULL pointers),
 * EIK_EDEVICE (launch failure).
 */
#ifndef EIK_ENCODER_H
#define EIK_ENCODER_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Dense layer of the global pathway on B rows: x [B][Cin], W [Cout][Cin],
 * b [Cout] (may be NULL), y [B][Cout]:
 *   y[r][o] = act( b[o] + sum_i W[o][i] x[r][i] ),  act = ReLU when relu != 0.
 * The sum runs over i in increasing order with fused multiply-adds. */
int eik_enc_dense(int32_t B, int32_t Cin, int32_t Cout, const float *x, const float *W, const float *b, int32_t relu,
                  float *y, hipStream_t stream);

/* Backward of eik_enc_dense given its output y and the gradient dy:
 *   g[r][o] = dy[r][o] (times [y[r][o] > 0] when relu != 0),
 *   dx[r][i] = sum_o W[o][i] g[r][o]           (written; dx may be NULL),
 *   dW[o][i] += sum_r g[r][o] x[r][i],  db[o] += sum_r g[r][o]  (accumulated). */
int eik_enc_dense_backward(int32_t B, int32_t Cin, int32_t Cout, const float *x, const float *W, const float *y,
                           int32_t relu, const float *dy, float *dx, float *dW, float *db, hipStream_t stream);

/* Combination, for B scenes of n nodes each, of the global baselines
 * base [B][5] (per scene g11, g12, g22, b1, b2) with the spatial residual
 * planes local [5][B][n] (FP32; the layout 1x1 heads write over the B n
 * pixels of a batch) into the metric planes M [B][3][n] and drift planes
 * omega [B][2][n] of type dtype (EIK_F32 / EIK_F64; the packing of the
 * batched solve):
 *   M[b][c][k] = base[b][c] + alpha local[c][b][k],
 *   omega[b][c][k] = base[b][3 + c] + alpha local[3 + c][b][k],
 * evaluated in double and rounded once to dtype. 1 <= B <= 4096. */
int eik_enc_combine(int32_t B, int64_t n, int32_t dtype, double alpha, const float *base, const float *local,
                    void *M, void *omega, hipStream_t stream);

/* Bytes of scratch eik_enc_combine_backward needs for B scenes (independent
 * of n; 0 for B outside 1..4096). */
size_t eik_enc_scratch_bytes(int32_t B);

/* Backward of eik_enc_combine given dM [B][3][n] and domega [B][2][n] (dtype):
 *   dlocal[c][b][k] = alpha d[b][c][k]  (written, FP32),
 *   dbase[b][c] += sum_k d[b][c][k]      (accumulated; the sum in double, fixed order),
 * with d = (dM, domega) stacked as five planes per scene. scratch holds at
 * least eik_enc_scratch_bytes(B) bytes of device memory. */
int eik_enc_combine_backward(int32_t B, int64_t n, int32_t dtype, double alpha, const void *dM, const void *domega,
                             float *dlocal, float *dbase, void *scratch, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* EIK_ENCODER_H */
