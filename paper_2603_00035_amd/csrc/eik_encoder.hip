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

// B scenes: base [B][5], local [5][B][n], M [B][3][n], om [B][2][n]
template <typename R>
__global__ __launch_bounds__(kEncThreads) void k_combine(int B, int64_t n, double alpha,
                                                         const float *__restrict__ base,
                                                         const float *__restrict__ local, R *__restrict__ M,
                                                         R *__restrict__ om)
{
    const int64_t total = (int64_t)B * n;
    for (int64_t e = blockIdx.x * (int64_t)kEncThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kEncThreads) {
        const int b = (int)(e / n);
        const int64_t k = e - (int64_t)b * n;
        const float *bb = base + kEncPlanes * b;
        for (int c = 0; c < 3; ++c)
            M[(3 * (int64_t)b + c) * n + k] = R((double)bb[c] + alpha * (double)local[((int64_t)c * B + b) * n + k]);
        for (int c = 0; c < 2; ++c)
            om[(2 * (int64_t)b + c) * n + k] =
                R((double)bb[3 + c] + alpha * (double)local[((int64_t)(3 + c) * B + b) * n + k]);
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

// grid (kInvBlocks, 5 B): plane c of scene b (blockIdx.y = 5 b + c) of
// (dM, dom); writes alpha d into dlocal [5][B][n] and one double partial per
// block.
template <typename R>
__global__ __launch_bounds__(kEncThreads) void k_combine_bwd(int B, int64_t n, double alpha,
                                                             const R *__restrict__ dM, const R *__restrict__ dom,
                                                             float *__restrict__ dlocal, double *__restrict__ partial)
{
    __shared__ double sh[kEncThreads];
    const int pc = blockIdx.y, b = pc / kEncPlanes, c = pc - kEncPlanes * b;
    const R *d = c < 3 ? dM + (3 * (int64_t)b + c) * n : dom + (2 * (int64_t)b + c - 3) * n;
    float *dl = dlocal + ((int64_t)c * B + b) * n;
    double acc = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)kEncThreads + threadIdx.x; k < n; k += (int64_t)kInvBlocks * kEncThreads) {
        const double v = (double)d[k];
        dl[k] = (float)(alpha * v);
        acc += v;
    }
    const double s = enc_block_sum(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)pc * kInvBlocks + blockIdx.x] = s;
}

// one block per (scene, plane): dbase[5 b + c] += sum of its partials in a
// fixed order
__global__ __launch_bounds__(kEncThreads) void k_combine_bwd_finish(const double *__restrict__ partial,
                                                                    float *__restrict__ dbase)
{
    __shared__ double sh[kEncThreads];
    const int pc = blockIdx.x;
    double x = 0.0;
    for (int b = threadIdx.x; b < kInvBlocks; b += kEncThreads) x += partial[(int64_t)pc * kInvBlocks + b];
    const double s = enc_block_sum(x, sh);
    if (threadIdx.x == 0) dbase[pc] = (float)((double)dbase[pc] + s);
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
void launch_enc_combine(int B, int64_t n, double alpha, const float *base, const float *local, void *M, void *om,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_combine<R>, dim3(blocks_for((int64_t)B * n, kEncThreads)), dim3(kEncThreads), 0, st, B, n,
                       alpha, base, local, (R *)M, (R *)om);
}

template <typename R>
void launch_enc_combine_backward(int B, int64_t n, double alpha, const void *dM, const void *dom, float *dlocal,
                                 float *dbase, double *partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_combine_bwd<R>, dim3(kInvBlocks, kEncPlanes * B), dim3(kEncThreads), 0, st, B, n, alpha,
                       (const R *)dM, (const R *)dom, dlocal, partial);
    hipLaunchKernelGGL(k_combine_bwd_finish, dim3(kEncPlanes * B), dim3(kEncThreads), 0, st, partial, dbase);
}

template void launch_enc_combine<float>(int, int64_t, double, const float *, const float *, void *, void *,
                                        hipStream_t);
template void launch_enc_combine<double>(int, int64_t, double, const float *, const float *, void *, void *,
                                         hipStream_t);
template void launch_enc_combine_backward<float>(int, int64_t, double, const void *, const void *, float *, float *,
                                                 double *, hipStream_t);
template void launch_enc_combine_backward<double>(int, int64_t, double, const void *, const void *, float *,
                                                  float *, double *, hipStream_t);

} // namespace eik
