// eik_backward.hip -- adjoint of the converged solve on gfx950 (Sec. 3.3,
// Alg. backward; Eqs. implicit, param_grad, adjoint).
//
// With the active update of node j fixed, dT_j/dT_i is the donor weight w
// (barycentric weight of a two-point update, 1 for a one-point update), so the
// adjoint system J^T lambda = dL/dT is lower-triangular in the causal order and
// reads lambda_i = g_i + sum over the nodes j that i feeds of w_ji lambda_j.
// Instead of sorting by T, nodes are bucketed by dependency level (counting
// sort) and levels are processed from the deepest down: every node of a level
// gathers from its (at most eight) receivers, which all sit at deeper levels,
// so no atomics are needed. dL/dtheta_i = lambda_i dT_i/dtheta_i is fused in.
#include "eik_device.h"
#include "eik_internal.h"

namespace eik {

static inline int blocks_for(int64_t n, int bs) { return (int)std::min<int64_t>((n + bs - 1) / bs, 4096); }

__global__ void k_fill_u64(unsigned long long *__restrict__ p, int64_t n)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        p[c] = 0ull;
}

// Donor weights of each active two-point update, level histogram, and zeroed
// gradient planes.
template <typename R>
__global__ void k_adj_prep(GridArgs g, const R *__restrict__ M, const R *__restrict__ om, const R *__restrict__ T,
                           const uint8_t *__restrict__ parent, const int32_t *__restrict__ level,
                           R *__restrict__ w1buf, int32_t *__restrict__ counts, R *__restrict__ dM,
                           R *__restrict__ dom)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    const R h = R(g.h);
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        dM[c] = R(0);
        dM[n + c] = R(0);
        dM[2 * n + c] = R(0);
        dom[c] = R(0);
        dom[n + c] = R(0);
        const int lv = level[c];
        if (lv >= 0 && lv < n) atomicAdd(&counts[lv], 1);
        const int code = parent[c];
        R w = R(1);
        const int i = (int)(c % g.nx), j = (int)(c / g.nx);
        const int kq = (code + 1) & 7;
        const bool inside = code < 8 && i + nb_dx(code) >= 0 && i + nb_dx(code) < g.nx && j + nb_dy(code) >= 0 &&
                            j + nb_dy(code) < g.ny && i + nb_dx(kq) >= 0 && i + nb_dx(kq) < g.nx &&
                            j + nb_dy(kq) >= 0 && j + nb_dy(kq) < g.ny;
        if (inside) {
            const R Tp = T[(size_t)(j + nb_dy(code)) * g.nx + i + nb_dx(code)];
            const R Tq = T[(size_t)(j + nb_dy(kq)) * g.nx + i + nb_dx(kq)];
            NodeConst<R> k;
            node_const<R>(M[c], M[n + c], M[2 * n + c], om[c], om[n + c], h, k);
            R t, mu1, mu2;
            two_point<R>(k, code, Tp, Tq, t, mu1, mu2);
            w = mu1 / (mu1 + mu2);
        }
        w1buf[c] = w;
    }
}

// Exclusive scan of the level histogram (one workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void k_scan_levels(int32_t *__restrict__ counts, int32_t *__restrict__ offsets,
                                                      int32_t *__restrict__ cursor,
                                                      const unsigned long long *__restrict__ ctr)
{
    __shared__ int32_t part[1024];
    __shared__ int32_t carry;
    const int L = (int)ctr[kCtrMaxLevel] + 1;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < L; base += 1024) {
        const int idx = base + threadIdx.x;
        const int v = idx < L ? counts[idx] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        const int excl = carry + part[threadIdx.x] - v;
        if (idx < L) {
            offsets[idx] = excl;
            cursor[idx] = excl;
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) offsets[L] = carry;
}

__global__ void k_scatter_levels(int64_t n, const int32_t *__restrict__ level, int32_t *__restrict__ cursor,
                                 int32_t *__restrict__ list)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const int lv = level[c];
        if (lv >= 0 && lv < n) list[atomicAdd(&cursor[lv], 1)] = (int32_t)c;
    }
}

// Levels L_hi down to L_lo. In single-workgroup mode the whole loop runs in
// one launch with a barrier between levels (L_hi < 0 means: the deepest level
// recorded in ctr); otherwise the launch covers one level.
template <typename R>
__global__ __launch_bounds__(1024) void k_adj_levels(GridArgs g, int L_hi, int L_lo,
                                                     const unsigned long long *__restrict__ ctr,
                                                     const int32_t *__restrict__ offsets,
                                                     const int32_t *__restrict__ list,
                                                     const uint8_t *__restrict__ parent, const R *__restrict__ w1buf,
                                                     const R *__restrict__ dLdT, const R *__restrict__ M,
                                                     R *__restrict__ lam, R *__restrict__ dM, R *__restrict__ dom)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    const R h = R(g.h);
    if (L_hi < 0) L_hi = (int)ctr[kCtrMaxLevel];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int L = L_hi; L >= L_lo; --L) {
        const int b = offsets[L], e = offsets[L + 1];
        for (int64_t p = b + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < e; p += stride) {
            const int c = list[p];
            const int i = c % g.nx, j = c / g.nx;
            R acc = dLdT[c];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int a = i + nb_dx(k), bb = j + nb_dy(k);
                if (a < 0 || a >= g.nx || bb < 0 || bb >= g.ny) continue;
                const int jc = bb * g.nx + a;
                const int pc = parent[jc];
                const int kk = (k + 4) & 7; // i seen from jc is neighbour kk of jc
                if (pc == kk)
                    acc += w1buf[jc] * lam[jc];
                else if (pc == ((kk + 7) & 7))
                    acc += (R(1) - w1buf[jc]) * lam[jc];
                else if (pc == 8 + kk)
                    acc += lam[jc];
            }
            lam[c] = acc;
            const int code = parent[c];
            if (code < 16) {
                R d[5];
                param_derivs<R>(code, w1buf[c], M[c], M[n + c], M[2 * n + c], h, d);
                dM[c] = acc * d[0];
                dM[n + c] = acc * d[1];
                dM[2 * n + c] = acc * d[2];
                dom[c] = acc * d[3];
                dom[n + c] = acc * d[4];
            }
        }
        if (gridDim.x == 1) __syncthreads();
    }
}

template <typename R>
__global__ void k_dsrc(int n_src, int64_t n, const int32_t *__restrict__ src_idx, const R *__restrict__ lam,
                       R *__restrict__ dsrc)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_src) return;
    const int c = src_idx[s];
    dsrc[s] = (c >= 0 && c < n) ? lam[c] : R(0);
}

// ---------------------------------------------------------------------------
template <typename R>
void launch_adj_prep(const GridArgs &g, const void *M, const void *om, const void *T, const uint8_t *parent,
                     const int32_t *level, void *w1, int32_t *counts, void *dM, void *dom, hipStream_t st)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    hipLaunchKernelGGL(k_adj_prep<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, g, (const R *)M, (const R *)om,
                       (const R *)T, parent, level, (R *)w1, counts, (R *)dM, (R *)dom);
}

void launch_scan_levels(int32_t *counts, int32_t *offsets, int32_t *cursor, const unsigned long long *ctr,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_scan_levels, dim3(1), dim3(1024), 0, st, counts, offsets, cursor, ctr);
}

void launch_scatter_levels(int64_t n, const int32_t *level, int32_t *cursor, int32_t *list, hipStream_t st)
{
    hipLaunchKernelGGL(k_scatter_levels, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, level, cursor, list);
}

void launch_fill_u64(unsigned long long *p, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
}

template <typename R>
void launch_adj_levels(const GridArgs &g, int L_hi, int L_lo, bool single_wg, const unsigned long long *ctr,
                       const int32_t *offsets, const int32_t *list, const uint8_t *parent, const void *w1,
                       const void *dLdT, const void *M, void *lam, void *dM, void *dom, hipStream_t st)
{
    const int blocks = single_wg ? 1 : 64;
    const int threads = single_wg ? 1024 : 256;
    hipLaunchKernelGGL(k_adj_levels<R>, dim3(blocks), dim3(threads), 0, st, g, L_hi, L_lo, ctr, offsets, list,
                       parent, (const R *)w1, (const R *)dLdT, (const R *)M, (R *)lam, (R *)dM, (R *)dom);
}

template <typename R>
void launch_dsrc(const GridArgs &g, const int32_t *src_idx, const void *lam, void *dsrc, hipStream_t st)
{
    hipLaunchKernelGGL(k_dsrc<R>, dim3((g.n_src + 255) / 256), dim3(256), 0, st, g.n_src, (int64_t)g.nx * g.ny,
                       src_idx, (const R *)lam, (R *)dsrc);
}

#define EIK_INST(R)                                                                                              \
    template void launch_adj_prep<R>(const GridArgs &, const void *, const void *, const void *, const uint8_t *, \
                                     const int32_t *, void *, int32_t *, void *, void *, hipStream_t);           \
    template void launch_adj_levels<R>(const GridArgs &, int, int, bool, const unsigned long long *,             \
                                       const int32_t *, const int32_t *, const uint8_t *, const void *,          \
                                       const void *, const void *, void *, void *, void *, hipStream_t);         \
    template void launch_dsrc<R>(const GridArgs &, const int32_t *, const void *, void *, hipStream_t);
EIK_INST(float)
EIK_INST(double)
#undef EIK_INST

} // namespace eik
