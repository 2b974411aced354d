// eik_inverse.hip -- kernels of one iteration of the regularised
// least-squares recovery of metric and drift (Sec. 5, Eq. inverse_problem):
// total variation of a field and its gradient (App. learning details), the
// data term over observed nodes, sums of squares for global-norm clipping,
// and the parameter step (projected gradient descent or Adam, App. inverse
// problem experiments).
//
// All are elementwise or stencil passes over HBM-resident planes, so they are
// bandwidth-bound; the TV gradient is a gather (each node recomputes the
// three gradient norms it enters), so no atomics are needed. Reductions are
// deterministic: a fixed grid of kInvBlocks blocks writes one double partial
// per block (shared-memory tree in a fixed order), and one block adds the
// partials in a fixed order.
#include <math.h>

#include "eik_internal.h"

namespace eik {

constexpr int kInvThreads = 256;

// Fixed-order sum of the 256 values of a block; returns the total in thread 0.
__device__ __forceinline__ double block_sum(double x, double *sh)
{
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int s = kInvThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// *out = (add ? *out : 0) + sum of the kInvBlocks partials, in a fixed order.
__global__ __launch_bounds__(kInvThreads) void k_finish_sum(const double *__restrict__ partial, double *out, int add)
{
    __shared__ double sh[kInvThreads];
    double x = 0.0;
    for (int b = threadIdx.x; b < kInvBlocks; b += kInvThreads) x += partial[b];
    const double s = block_sum(x, sh);
    if (threadIdx.x == 0) *out = (add ? *out : 0.0) + s;
}

struct TvWeights {
    double w[4];
};

// Gradient norm of node (i, j): forward differences, zero across the last
// column / row.
template <typename R>
__device__ __forceinline__ R tv_norm(const R *F, int64_t plane, int nx, int ny, int C, const TvWeights &w, int i, int j)
{
    const int64_t c0 = (int64_t)j * nx + i;
    R s = R(0);
    for (int c = 0; c < C; ++c) {
        const R *Fc = F + c * plane;
        const R f = Fc[c0];
        const R dx = i + 1 < nx ? Fc[c0 + 1] - f : R(0);
        const R dy = j + 1 < ny ? Fc[c0 + nx] - f : R(0);
        s += R(w.w[c]) * (dx * dx + dy * dy);
    }
    return sqrt(s);
}

template <typename R>
__global__ __launch_bounds__(kInvThreads) void k_tv(int nx, int ny, int C, const R *__restrict__ F, TvWeights w,
                                                    R scale, R *__restrict__ grad, double *__restrict__ partial)
{
    __shared__ double sh[kInvThreads];
    const int64_t plane = (int64_t)nx * ny;
    double acc = 0.0;
    for (int64_t idx = blockIdx.x * (int64_t)kInvThreads + threadIdx.x; idx < plane;
         idx += (int64_t)kInvBlocks * kInvThreads) {
        const int j = (int)(idx / nx), i = (int)(idx - (int64_t)j * nx);
        const R n0 = tv_norm<R>(F, plane, nx, ny, C, w, i, j);
        const R n1 = i > 0 ? tv_norm<R>(F, plane, nx, ny, C, w, i - 1, j) : R(0);
        const R n2 = j > 0 ? tv_norm<R>(F, plane, nx, ny, C, w, i, j - 1) : R(0);
        acc += (double)n0;
        for (int c = 0; c < C; ++c) {
            const R *Fc = F + c * plane;
            const R f = Fc[idx];
            R g = R(0);
            // the subgradient 0 is taken for a term whose norm is 0
            if (n0 > R(0)) {
                const R dx = i + 1 < nx ? Fc[idx + 1] - f : R(0);
                const R dy = j + 1 < ny ? Fc[idx + nx] - f : R(0);
                g -= (dx + dy) / n0;
            }
            if (n1 > R(0)) g += (f - Fc[idx - 1]) / n1;
            if (n2 > R(0)) g += (f - Fc[idx - nx]) / n2;
            grad[c * plane + idx] += scale * R(w.w[c]) * g;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = (double)scale * s;
}

template <typename R>
__global__ __launch_bounds__(kInvThreads) void k_obs_loss(int64_t n, const R *__restrict__ T, const R *__restrict__ To,
                                                          const uint8_t *__restrict__ mask, R *__restrict__ g,
                                                          double *__restrict__ partial)
{
    __shared__ double sh[kInvThreads];
    double acc = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)kInvThreads + threadIdx.x; k < n; k += (int64_t)kInvBlocks * kInvThreads) {
        const R t = T[k], o = To[k];
        const bool use = mask[k] != 0 && isfinite(t) && isfinite(o);
        const R r = use ? t - o : R(0);
        g[k] = r;
        acc += 0.5 * (double)r * (double)r;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename R>
__global__ __launch_bounds__(kInvThreads) void k_sum_sq(int64_t n, const R *__restrict__ x,
                                                        double *__restrict__ partial)
{
    __shared__ double sh[kInvThreads];
    double acc = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)kInvThreads + threadIdx.x; k < n; k += (int64_t)kInvBlocks * kInvThreads) {
        const double v = (double)x[k];
        acc += v * v;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename R>
__global__ __launch_bounds__(kInvThreads) void k_param_step(int64_t n, int method, R *__restrict__ p,
                                                            const R *__restrict__ g, R *__restrict__ m,
                                                            R *__restrict__ v, R lr, R b1, R b2, R eps, R bc1, R bc2,
                                                            double max_norm, const double *__restrict__ grad_sq)
{
    // global-norm clipping factor, from the device sum of squares
    R cs = R(1);
    if (max_norm > 0.0) {
        const double nrm = sqrt(*grad_sq);
        if (nrm > max_norm) cs = R(max_norm / nrm);
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const R gk = cs * g[k];
        if (method == 0) {
            p[k] -= lr * gk;
        } else {
            const R mk = b1 * m[k] + (R(1) - b1) * gk;
            const R vk = b2 * v[k] + (R(1) - b2) * gk * gk;
            m[k] = mk;
            v[k] = vk;
            p[k] -= lr * (mk / bc1) / (sqrt(vk / bc2) + eps);
        }
    }
}

template <typename R>
__global__ void k_tie_isotropic(int64_t n, R *__restrict__ M)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const R g = R(0.5) * (M[k] + M[2 * n + k]);
        M[k] = g;
        M[n + k] = R(0);
        M[2 * n + k] = g;
    }
}

// ---------------------------------------------------------------------------
// Log-Euclidean TV (App. learning details, Total Variation Regularization):
// the TV of the planes of log G, with log G in closed form through the
// eigen-decomposition of each 2x2 metric, G = Q diag(l1, l2) Q^T with Q the
// rotation by theta = atan2(2 m12, m11 - m22) / 2:
//   log G = Q diag(log l1, log l2) Q^T.
// Its derivative in direction E (a symmetric matrix) is
//   Q (F o (Q^T E Q)) Q^T,  F11 = 1/l1, F22 = 1/l2,
//   F12 = F21 = (log l1 - log l2) / (l1 - l2),
// a self-adjoint map under the Frobenius product, so the gradient with
// respect to G is the same map applied to the gradient with respect to log G.
// With t = (l1 + l2)/2 and d = (l1 - l2)/2 the divided difference is
// atanh(d/t)/d, which tends to 1/t where the eigenvalues meet (series below
// d/t = 1e-3).
template <typename R>
struct Eig2 {
    R c, s, l1, l2, L1, L2, f12;
};

template <typename R>
__device__ __forceinline__ Eig2<R> eig2(R m11, R m12, R m22)
{
    Eig2<R> e;
    const R t = R(0.5) * (m11 + m22), hd = R(0.5) * (m11 - m22);
    const R d = sqrt(hd * hd + m12 * m12);
    e.l1 = t + d;
    e.l2 = (m11 * m22 - m12 * m12) / e.l1; // the smaller eigenvalue, free of cancellation
    const R th = R(0.5) * atan2(m12, hd);
    e.c = cos(th);
    e.s = sin(th);
    e.L1 = log(e.l1);
    e.L2 = log(e.l2);
    const R x = d / t;
    e.f12 = x < R(1e-3) ? (R(1) + x * x * (R(1) / R(3) + x * x * R(0.2))) / t : atanh(x) / d;
    return e;
}

// P[3][n] = planes (p11, p12, p22) of log G.
template <typename R>
__global__ void k_logm(int64_t n, const R *__restrict__ M, R *__restrict__ P)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const Eig2<R> e = eig2<R>(M[k], M[n + k], M[2 * n + k]);
        const R cc = e.c * e.c, ss = e.s * e.s, cs = e.c * e.s;
        P[k] = cc * e.L1 + ss * e.L2;
        P[n + k] = cs * (e.L1 - e.L2);
        P[2 * n + k] = ss * e.L1 + cc * e.L2;
    }
}

// grad[3][n] += d(R)/d(m11, m12, m22) given gP = dR/d(p11, p12, p22); the
// stored m12 and p12 stand for both off-diagonal entries.
template <typename R>
__global__ void k_logm_vjp(int64_t n, const R *__restrict__ M, const R *__restrict__ gP, R *__restrict__ grad)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const Eig2<R> e = eig2<R>(M[k], M[n + k], M[2 * n + k]);
        const R cc = e.c * e.c, ss = e.s * e.s, cs = e.c * e.s, dcs = cc - ss;
        // the symmetric gradient with respect to log G
        const R a11 = gP[k], a12 = R(0.5) * gP[n + k], a22 = gP[2 * n + k];
        // rotated into the eigenbasis, scaled by F, rotated back
        const R A11 = cc * a11 + R(2) * cs * a12 + ss * a22;
        const R A22 = ss * a11 - R(2) * cs * a12 + cc * a22;
        const R A12 = cs * (a22 - a11) + dcs * a12;
        const R B11 = A11 / e.l1, B22 = A22 / e.l2, B12 = e.f12 * A12;
        grad[k] += cc * B11 - R(2) * cs * B12 + ss * B22;
        grad[n + k] += R(2) * (cs * (B11 - B22) + dcs * B12);
        grad[2 * n + k] += ss * B11 + R(2) * cs * B12 + cc * B22;
    }
}

template <typename R>
void launch_tv_log_euclid(int nx, int ny, const void *M, double scale, void *grad, double *value, void *work,
                          double *partial, hipStream_t st)
{
    const int64_t n = (int64_t)nx * ny;
    R *P = (R *)work, *gP = P + 3 * n;
    hipLaunchKernelGGL(k_logm<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, (const R *)M, P);
    launch_fill_i32((int32_t *)gP, 3 * n * (int64_t)(sizeof(R) / 4), 0, st); // +0.0
    const double w[3] = {1.0, 2.0, 1.0};
    launch_tv<R>(nx, ny, 3, P, w, scale, gP, value, partial, st);
    hipLaunchKernelGGL(k_logm_vjp<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, (const R *)M, gP, (R *)grad);
}

// ---------------------------------------------------------------------------
template <typename R>
void launch_tie_isotropic(int64_t n, void *M, hipStream_t st)
{
    hipLaunchKernelGGL(k_tie_isotropic<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, (R *)M);
}

template <typename R>
void launch_tv(int nx, int ny, int C, const void *F, const double *weights, double scale, void *grad,
               double *value, double *partial, hipStream_t st)
{
    TvWeights w = {{0.0, 0.0, 0.0, 0.0}};
    for (int c = 0; c < C; ++c) w.w[c] = weights[c];
    hipLaunchKernelGGL(k_tv<R>, dim3(kInvBlocks), dim3(kInvThreads), 0, st, nx, ny, C, (const R *)F, w, R(scale),
                       (R *)grad, partial);
    hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(kInvThreads), 0, st, partial, value, 0);
}

template <typename R>
void launch_obs_loss(int64_t n, const void *T, const void *To, const uint8_t *mask, void *g, double *value,
                     double *partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_obs_loss<R>, dim3(kInvBlocks), dim3(kInvThreads), 0, st, n, (const R *)T, (const R *)To,
                       mask, (R *)g, partial);
    hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(kInvThreads), 0, st, partial, value, 0);
}

template <typename R>
void launch_sum_sq(int64_t n, const void *x, double *acc, double *partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_sq<R>, dim3(kInvBlocks), dim3(kInvThreads), 0, st, n, (const R *)x, partial);
    hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(kInvThreads), 0, st, partial, acc, 1);
}

template <typename R>
void launch_param_step(int64_t n, int method, void *p, const void *g, void *m, void *v, double lr, double b1,
                       double b2, double eps, int t, double max_norm, const double *grad_sq, hipStream_t st)
{
    const double bc1 = 1.0 - pow(b1, (double)t), bc2 = 1.0 - pow(b2, (double)t);
    hipLaunchKernelGGL(k_param_step<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, method, (R *)p, (const R *)g,
                       (R *)m, (R *)v, R(lr), R(b1), R(b2), R(eps), R(bc1), R(bc2), max_norm, grad_sq);
}

#define EIK_INV_INSTANTIATE(R)                                                                                   \
    template void launch_tv<R>(int, int, int, const void *, const double *, double, void *, double *, double *, \
                               hipStream_t);                                                                     \
    template void launch_obs_loss<R>(int64_t, const void *, const void *, const uint8_t *, void *, double *,     \
                                     double *, hipStream_t);                                                     \
    template void launch_sum_sq<R>(int64_t, const void *, double *, double *, hipStream_t);                      \
    template void launch_param_step<R>(int64_t, int, void *, const void *, void *, void *, double, double,       \
                                       double, double, int, double, const double *, hipStream_t);               \
    template void launch_tie_isotropic<R>(int64_t, void *, hipStream_t);                                     \
    template void launch_tv_log_euclid<R>(int, int, const void *, double, void *, double *, void *, double *,   \
                                          hipStream_t);
EIK_INV_INSTANTIATE(float)
EIK_INV_INSTANTIATE(double)

} // namespace eik
