/*
 * eik_inverse.h -- C ABI of the inverse-problem kernels of the MI355X
 * (gfx950) Randers-Finsler eikonal library: the pieces that, with eik_forward,
 * eik_backward and eik_project, make one iteration of the regularised
 * least-squares recovery of the metric and the drift from observed arrival
 * times (Sec. 5, Eq. inverse_problem; App. learning details, "Total
 * Variation Regularization"; App. inverse problem experiments, optimiser).
 *
 * Fields are laid out as in eik.h: planes [C][ny][nx] of real numbers (float
 * for EIK_F32, double for EIK_F64), device memory owned by the caller; every
 * call enqueues work on `stream` and never synchronises or allocates.
 * Reductions are deterministic: each block writes a partial sum into the
 * caller's scratch (eik_inv_scratch_bytes), one block adds the partials in a
 * fixed order, and the result stays in device memory (a double).
 * Errors: EIK_EINVAL (bad sizes, NULL pointers), EIK_EDEVICE (launch failure).
 */
#ifndef EIK_INVERSE_H
#define EIK_INVERSE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Bytes of scratch every reducing call below needs (independent of sizes). */
size_t eik_inv_scratch_bytes(void);

/* Total variation of a field of C planes with per-plane weights (App.
 * learning details): with forward differences in grid units, zero across the
 * last column / row,
 *   n_ij = sqrt( sum_c w_c [ (F_c(i+1,j) - F_c(i,j))^2 + (F_c(i,j+1) - F_c(i,j))^2 ] ),
 *   R = sum_ij n_ij.
 * The metric uses C = 3 planes (m11, m12, m22) with w = (1, 2, 1) (Frobenius
 * norm of the symmetric tensor's gradient); the drift C = 2 planes with
 * w = (1, 1) (Euclidean norm). Writes scale * R to *value (device double) and
 * adds scale * dR/dF to grad (same layout as F); where n_ij = 0 the
 * subgradient 0 is taken for its term. C is 1..4. */
int eik_tv(int32_t nx, int32_t ny, int32_t n_planes, int32_t dtype, const void *F, const double *weights,
           double scale, void *grad, double *value, void *scratch, hipStream_t stream);

/* Log-Euclidean TV of a metric field (App. learning details, Total
 * Variation Regularization): R = sum_ij |grad log G_ij|_F, with log G the
 * matrix logarithm of each SPD 2x2 metric in closed form through its
 * eigen-decomposition, and the norm that of eik_tv on the planes
 * (p11, p12, p22) of log G with weights (1, 2, 1). Unlike the Frobenius
 * variant it is invariant under a rotation of all metrics and under a common
 * scale. M [3][ny][nx] must be SPD everywhere (m11 > 0, det > 0; not checked).
 * Writes scale * R to *value (device double) and adds scale * dR/dM (with
 * respect to the stored m11, m12, m22) to grad [3][ny][nx]. work: device
 * memory of eik_tv_log_euclid_work_bytes bytes (log G and its gradient);
 * scratch as for eik_tv. */
size_t eik_tv_log_euclid_work_bytes(int32_t nx, int32_t ny, int32_t dtype);
int eik_tv_log_euclid(int32_t nx, int32_t ny, int32_t dtype, const void *M, double scale, void *grad,
                      double *value, void *work, void *scratch, hipStream_t stream);

/* Data term of Eq. inverse_problem over the observed nodes: with mask w_i in
 * {0, 1} (uint8, nonzero = observed), r_i = T_i - That_i,
 *   L = 1/2 sum_i w_i r_i^2,  dL/dT_i = w_i r_i (0 where T or That is not finite).
 * Writes L to *value (device double) and dL/dT to dLdT. */
int eik_obs_loss(int64_t n, int32_t dtype, const void *T, const void *T_obs, const uint8_t *mask, void *dLdT,
                 double *value, void *scratch, hipStream_t stream);

/* Sum of squares of n elements of a real array, added to *acc (device
 * double): for the global gradient norm of clipping. */
int eik_sum_sq(int64_t n, int32_t dtype, const void *x, double *acc, void *scratch, hipStream_t stream);

/* One optimiser step on n parameters p with gradient g (in place), the
 * gradient first scaled by min(1, max_norm / sqrt(*grad_sq)) when max_norm > 0
 * (global-norm clipping; grad_sq is the device double that eik_sum_sq filled
 * over all parameter groups). method 0: projected gradient descent,
 * p -= lr g. method 1: Adam with bias correction at step t >= 1,
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
 * m and v (same type and size as p) are the caller's state, zero at t = 1.
 * The feasibility projection (eik_project) is a separate call. */
int eik_param_step(int64_t n, int32_t dtype, int32_t method, void *p, const void *g, void *m, void *v, double lr,
                   double beta1, double beta2, double eps, int32_t t, double max_norm, const double *grad_sq,
                   hipStream_t stream);

/* Projection of n nodes of metric planes M [3][n] onto isotropic metrics
 * G = g I, in place: m11 = m22 = (m11 + m22) / 2, m12 = 0 (the Frobenius-
 * nearest isotropic tensor; the constraint of the isotropic recovery of
 * Sec. 5). */
int eik_tie_isotropic(int64_t n, int32_t dtype, void *M, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* EIK_INVERSE_H */
