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
    template void launch_tie_isotropic<R>(int64_t, void *, hipStream_t);
EIK_INV_INSTANTIATE(float)
EIK_INV_INSTANTIATE(double)

} // namespace eik
