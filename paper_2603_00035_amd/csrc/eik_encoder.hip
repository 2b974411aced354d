// eik_encoder.hip -- the covariate encoder's own kernels (Sec. 6, encoder
// architecture): dense layers of the global pathway and the combination of
// the global baseline (G0, b0) with the spatial residuals (G_local, b_local),
// G = G0 + alpha G_local, b = b0 + alpha b_local, and their backward passes.
//
// The dense layers are tiny (a handful of rows, tens of channels): one thread
// per output, sums in a fixed order. The combination is an elementwise pass
// over five HBM-resident planes (bandwidth-bound: 20 B read + 12 or 24 B
// written per node forward); its backward reduces each plane with fixed
// blocks and a fixed-order tree, in double.
#include <math.h>

#include "eik_internal.h"

namespace eik {

constexpr int kEncThreads = 256;

__global__ __launch_bounds__(kEncThreads) void k_dense(int B, int Cin, int Cout, const float *__restrict__ x,
                                                       const float *__restrict__ W, const float *__restrict__ b,
                                                       int relu, float *__restrict__ y)
{
    const int idx = blockIdx.x * kEncThreads + threadIdx.x;
    if (idx >= B * Cout) return;
    const int r = idx / Cout, o = idx - r * Cout;
    float s = b ? b[o] : 0.0f;
    for (int i = 0; i < Cin; ++i) s = fmaf(W[o * Cin + i], x[r * Cin + i], s);
    y[idx] = (relu && !(s > 0.0f)) ? 0.0f : s;
}

__device__ __forceinline__ float dense_g(const float *y, const float *dy, int relu, int k)
{
    return (relu && !(y[k] > 0.0f)) ? 0.0f : dy[k];
}

// dx[r][i] = sum_o W[o][i] g[r][o]
__global__ __launch_bounds__(kEncThreads) void k_dense_dx(int B, int Cin, int Cout, const float *__restrict__ W,
                                                          const float *__restrict__ y, int relu,
                                                          const float *__restrict__ dy, float *__restrict__ dx)
{
    const int idx = blockIdx.x * kEncThreads + threadIdx.x;
    if (idx >= B * Cin) return;
    const int r = idx / Cin, i = idx - r * Cin;
    float s = 0.0f;
    for (int o = 0; o < Cout; ++o) s = fmaf(W[o * Cin + i], dense_g(y, dy, relu, r * Cout + o), s);
    dx[idx] = s;
}

// dW[o][i] += sum_r g[r][o] x[r][i] (i < Cin); db[o] += sum_r g[r][o] (i == Cin)
__global__ __launch_bounds__(kEncThreads) void k_dense_dw(int B, int Cin, int Cout, const float *__restrict__ x,
                                                          const float *__restrict__ y, int relu,
                                                          const float *__restrict__ dy, float *__restrict__ dW,
                                                          float *__restrict__ db)
{
    const int idx = blockIdx.x * kEncThreads + threadIdx.x;
    if (idx >= Cout * (Cin + 1)) return;
    const int o = idx / (Cin + 1), i = idx - o * (Cin + 1);
    const int ix = i < Cin ? i : Cin - 1; // the bias slot reads a valid x and ignores it
    float s = 0.0f;
    for (int r = 0; r < B; ++r) {
        const float g = dense_g(y, dy, relu, r * Cout + o);
        const float xv = x[r * Cin + ix];
        s = (i < Cin) ? fmaf(g, xv, s) : s + g;
    }
    if (i < Cin)
        dW[o * Cin + i] += s;
    else if (db)
        db[o] += s;
}

template <typename R>
__global__ __launch_bounds__(kEncThreads) void k_combine(int64_t n, double alpha, const float *__restrict__ base,
                                                         const float *__restrict__ local, R *__restrict__ M,
                                                         R *__restrict__ om)
{
    double b[kEncPlanes];
    for (int c = 0; c < kEncPlanes; ++c) b[c] = (double)base[c];
    for (int64_t k = blockIdx.x * (int64_t)kEncThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kEncThreads) {
        for (int c = 0; c < 3; ++c) M[c * n + k] = R(b[c] + alpha * (double)local[c * n + k]);
        for (int c = 0; c < 2; ++c) om[c * n + k] = R(b[3 + c] + alpha * (double)local[(3 + c) * n + k]);
    }
}

// Fixed-order tree sum of a block's values; the total in thread 0.
__device__ __forceinline__ double enc_block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kEncThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// grid (kInvBlocks, 5): plane c of (dM, dom); writes alpha d and one double
// partial per block.
template <typename R>
__global__ __launch_bounds__(kEncThreads) void k_combine_bwd(int64_t n, double alpha, const R *__restrict__ dM,
                                                             const R *__restrict__ dom, float *__restrict__ dlocal,
                                                             double *__restrict__ partial)
{
    __shared__ double sh[kEncThreads];
    const int c = blockIdx.y;
    const R *d = c < 3 ? dM + c * n : dom + (c - 3) * n;
    double acc = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)kEncThreads + threadIdx.x; k < n; k += (int64_t)kInvBlocks * kEncThreads) {
        const double v = (double)d[k];
        dlocal[c * n + k] = (float)(alpha * v);
        acc += v;
    }
    const double s = enc_block_sum(acc, sh);
    if (threadIdx.x == 0) partial[c * kInvBlocks + blockIdx.x] = s;
}

// one block per plane: dbase[c] += sum of its partials in a fixed order
__global__ __launch_bounds__(kEncThreads) void k_combine_bwd_finish(const double *__restrict__ partial,
                                                                    float *__restrict__ dbase)
{
    __shared__ double sh[kEncThreads];
    const int c = blockIdx.x;
    double x = 0.0;
    for (int b = threadIdx.x; b < kInvBlocks; b += kEncThreads) x += partial[c * kInvBlocks + b];
    const double s = enc_block_sum(x, sh);
    if (threadIdx.x == 0) dbase[c] = (float)((double)dbase[c] + s);
}

// ---------------------------------------------------------------------------
void launch_enc_dense(int B, int Cin, int Cout, const float *x, const float *W, const float *b, int relu, float *y,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_dense, dim3((B * Cout + kEncThreads - 1) / kEncThreads), dim3(kEncThreads), 0, st, B, Cin,
                       Cout, x, W, b, relu, y);
}

void launch_enc_dense_backward(int B, int Cin, int Cout, const float *x, const float *W, const float *y, int relu,
                               const float *dy, float *dx, float *dW, float *db, hipStream_t st)
{
    if (dx)
        hipLaunchKernelGGL(k_dense_dx, dim3((B * Cin + kEncThreads - 1) / kEncThreads), dim3(kEncThreads), 0, st, B,
                           Cin, Cout, W, y, relu, dy, dx);
    hipLaunchKernelGGL(k_dense_dw, dim3((Cout * (Cin + 1) + kEncThreads - 1) / kEncThreads), dim3(kEncThreads), 0,
                       st, B, Cin, Cout, x, y, relu, dy, dW, db);
}

template <typename R>
void launch_enc_combine(int64_t n, double alpha, const float *base, const float *local, void *M, void *om,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_combine<R>, dim3(blocks_for(n, kEncThreads)), dim3(kEncThreads), 0, st, n, alpha, base,
                       local, (R *)M, (R *)om);
}

template <typename R>
void launch_enc_combine_backward(int64_t n, double alpha, const void *dM, const void *dom, float *dlocal,
                                 float *dbase, double *partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_combine_bwd<R>, dim3(kInvBlocks, kEncPlanes), dim3(kEncThreads), 0, st, n, alpha,
                       (const R *)dM, (const R *)dom, dlocal, partial);
    hipLaunchKernelGGL(k_combine_bwd_finish, dim3(kEncPlanes), dim3(kEncThreads), 0, st, partial, dbase);
}

template void launch_enc_combine<float>(int64_t, double, const float *, const float *, void *, void *, hipStream_t);
template void launch_enc_combine<double>(int64_t, double, const float *, const float *, void *, void *, hipStream_t);
template void launch_enc_combine_backward<float>(int64_t, double, const void *, const void *, float *, float *,
                                                 double *, hipStream_t);
template void launch_enc_combine_backward<double>(int64_t, double, const void *, const void *, float *, float *,
                                                  double *, hipStream_t);

} // namespace eik
