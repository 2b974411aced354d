// eik_levels.hip -- the adjoint in the order of Alg. backward, made parallel
// by dependency levels (Sec. 3.3; App. "Jacobian Details and Backward Pass").
//
// Alg. backward visits the nodes by decreasing arrival time and
// back-substitutes lambda_i = g_i + sum over the nodes j that i feeds of
// (dT_j/dT_i) lambda_j. The dependency level of a node (0 at a source, one
// more than the largest level of its donors) orders the same triangular
// system more loosely: every node a node feeds sits on a strictly higher
// level, so the nodes of one level are independent of each other once all
// higher levels are done.
//
// Level bucketing (per grid, at the grid's node offset in the packed arrays):
// a counting sort of the reached nodes by level -- largest level, histogram,
// exclusive scan, scatter -- into `order`; afterwards bins[l] is the end of
// bin l (its start is bins[l - 1], or 0). Integer atomics only place nodes.
//
// Gather: one workgroup per grid walks the levels from the largest down. The
// nodes of a level are spread over the workgroup; each sums over its
// receivers with the receiver descriptors and donor weights of the
// relaxation adjoint (same coefficients, same neighbour order, so the same
// rounding), and a workgroup barrier separates levels. Nothing is scattered
// and the arithmetic uses no atomics. A level's node list, descriptors and
// dL/dT do not depend on lambda, so the workgroup loads the next level's
// while it solves the current one.
#include "eik_device.h"
#include "eik_internal.h"

namespace eik {

constexpr int kLvlThreads = 1024;  // gather workgroup (one per grid)
constexpr int kLvlLdsBins = 4096;  // per-tile histogram range held in LDS

struct TileGeoL {
    GridDesc gd;
    int i0, j0, w, h, g;
};

template <int TH>
__device__ __forceinline__ TileGeoL tile_geo_l(const LaunchArgs &a, int t)
{
    TileGeoL r;
    r.g = a.tile_grid[t];
    r.gd = a.grids[r.g];
    const int lt = t - r.gd.tile_base;
    const int tx = lt % r.gd.ntx, ty = lt / r.gd.ntx;
    r.i0 = tx * TW;
    r.j0 = ty * TH;
    r.w = min(TW, r.gd.nx - r.i0);
    r.h = min(TH, r.gd.ny - r.j0);
    return r;
}

__device__ __forceinline__ int block_reduce_max(int v, int *sred)
{
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off));
    const int wave = threadIdx.x / TW, nw = blockDim.x / TW;
    __syncthreads();
    if ((threadIdx.x % TW) == 0) sred[wave] = v;
    __syncthreads();
    int m = sred[0];
    for (int k = 1; k < nw; ++k) m = max(m, sred[k]);
    return m;
}

__device__ __forceinline__ int block_reduce_min(int v, int *sred)
{
    for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off));
    const int wave = threadIdx.x / TW, nw = blockDim.x / TW;
    __syncthreads();
    if ((threadIdx.x % TW) == 0) sred[wave] = v;
    __syncthreads();
    int m = sred[0];
    for (int k = 1; k < nw; ++k) m = min(m, sred[k]);
    return m;
}

// Largest level of each grid (gmax preset to -1). Levels outside
// [0, n_g - 1] (impossible for a level field of the grid) are ignored.
template <int TH>
__global__ __launch_bounds__(256) void k_lvl_max(LaunchArgs a, const int32_t *__restrict__ levall,
                                                 int32_t *__restrict__ gmax)
{
    __shared__ int sred[4];
    const TileGeoL g = tile_geo_l<TH>(a, blockIdx.x);
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const int32_t *level = levall + g.gd.off;
    int m = -1;
    for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
        const int r = idx / TW, c = idx - r * TW;
        if (r >= g.h || c >= g.w) continue;
        const int l = level[(size_t)(g.j0 + r) * g.gd.nx + g.i0 + c];
        if (l >= 0 && l < n) m = max(m, l);
    }
    m = block_reduce_max(m, sred);
    if (threadIdx.x == 0 && m >= 0) atomicMax(&gmax[g.g], m);
}

// bins[0 .. gmax] = 0 per grid (one workgroup per grid).
__global__ __launch_bounds__(256) void k_lvl_clear(LaunchArgs a, const int32_t *__restrict__ gmax,
                                                   int32_t *__restrict__ bins)
{
    const GridDesc gd = a.grids[blockIdx.x];
    const int nb = gmax[blockIdx.x] + 1;
    for (int l = threadIdx.x; l < nb; l += blockDim.x) bins[gd.off + l] = 0;
}

// Histogram (SCATTER = false) or placement (SCATTER = true) of one tile's
// reached nodes by level. A tile whose levels span at most kLvlLdsBins
// values counts them in LDS first and touches each global bin once (placement:
// one atomic reserves the tile's run inside the bin, LDS atomics hand out the
// slots); a wider tile goes to the global bins node by node.
template <int TH, bool SCATTER>
__global__ __launch_bounds__(256) void k_lvl_bucket(LaunchArgs a, const int32_t *__restrict__ levall,
                                                    int32_t *__restrict__ bins, int32_t *__restrict__ order)
{
    __shared__ int32_t hist[kLvlLdsBins];
    __shared__ int sred[4];
    const TileGeoL g = tile_geo_l<TH>(a, blockIdx.x);
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const int32_t *level = levall + g.gd.off;
    int32_t *gb = bins + g.gd.off;
    int32_t *go = order + g.gd.off;
    int lo = INT32_MAX, hi = -1;
    for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
        const int r = idx / TW, c = idx - r * TW;
        if (r >= g.h || c >= g.w) continue;
        const int l = level[(size_t)(g.j0 + r) * g.gd.nx + g.i0 + c];
        if (l >= 0 && l < n) {
            lo = min(lo, l);
            hi = max(hi, l);
        }
    }
    lo = block_reduce_min(lo, sred);
    hi = block_reduce_max(hi, sred);
    if (hi < 0) return; // nothing reached in this tile (uniform)
    const bool in_lds = hi - lo < kLvlLdsBins;
    if (in_lds) {
        for (int b = threadIdx.x; b <= hi - lo; b += blockDim.x) hist[b] = 0;
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
        const int r = idx / TW, c = idx - r * TW;
        if (r >= g.h || c >= g.w) continue;
        const int l = level[(size_t)(g.j0 + r) * g.gd.nx + g.i0 + c];
        if (l < 0 || l >= n) continue;
        if (in_lds) atomicAdd(&hist[l - lo], 1);
        else if (!SCATTER) atomicAdd(&gb[l], 1);
        else go[atomicAdd(&gb[l], 1)] = (g.j0 + r) * g.gd.nx + g.i0 + c;
    }
    if (!in_lds) return;
    __syncthreads();
    for (int b = threadIdx.x; b <= hi - lo; b += blockDim.x) {
        const int cnt = hist[b];
        if (cnt == 0) continue;
        const int base = atomicAdd(&gb[lo + b], cnt);
        if (SCATTER) hist[b] = base; // the tile's run inside bin lo + b starts here
    }
    if (!SCATTER) return;
    __syncthreads();
    for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
        const int r = idx / TW, c = idx - r * TW;
        if (r >= g.h || c >= g.w) continue;
        const int l = level[(size_t)(g.j0 + r) * g.gd.nx + g.i0 + c];
        if (l < 0 || l >= n) continue;
        go[atomicAdd(&hist[l - lo], 1)] = (g.j0 + r) * g.gd.nx + g.i0 + c;
    }
}

// Exclusive scan of bins[0 .. gmax] per grid, in place (one workgroup of 256
// per grid, chunks of 256 with a running carry).
__global__ __launch_bounds__(256) void k_lvl_scan(LaunchArgs a, const int32_t *__restrict__ gmax,
                                                  int32_t *__restrict__ bins)
{
    __shared__ int32_t s[256];
    const GridDesc gd = a.grids[blockIdx.x];
    const int nb = gmax[blockIdx.x] + 1;
    int32_t *b = bins + gd.off;
    int carry = 0;
    for (int base = 0; base < nb; base += 256) {
        const int l = base + threadIdx.x;
        const int v = l < nb ? b[l] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) { // Hillis-Steele inclusive scan
            const int x = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += x;
            __syncthreads();
        }
        if (l < nb) b[l] = carry + s[threadIdx.x] - v;
        carry += s[255];
        __syncthreads();
    }
}

// The gather by levels, from the largest down (one workgroup per grid). A
// thread holds the node list entry, descriptor and dL/dT of its first node of
// the next level while it solves the current one.
template <typename R>
__global__ __launch_bounds__(kLvlThreads) void k_lvl_gather(LaunchArgs a, const int32_t *__restrict__ gmax,
                                                            const int32_t *__restrict__ bins,
                                                            const int32_t *__restrict__ order,
                                                            const uint16_t *__restrict__ Dall,
                                                            const R *__restrict__ gall,
                                                            const R *__restrict__ w1all, R *__restrict__ lamall)
{
    const GridDesc gd = a.grids[blockIdx.x];
    const int top = gmax[blockIdx.x];
    if (top < 0) return;
    const int nx = gd.nx;
    const int32_t *b = bins + gd.off;
    const int32_t *ord = order + gd.off;
    const uint16_t *D = Dall + gd.off;
    const R *gv = gall + gd.off;
    const R *w1 = w1all + gd.off;
    R *lam = lamall + gd.off;
    const int tid = threadIdx.x;

    auto solve = [&](int c, uint32_t d, R acc) {
        const int i = c % nx, j = c / nx;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t sel = (d >> (2 * k)) & 3u;
            if (sel == 0u) continue;
            const int nb = (j + nb_dy(k)) * nx + i + nb_dx(k);
            const R lk = lam[nb], wk = w1[nb];
            R coef = sel == 3u ? R(1) : R(0);
            coef = sel == 2u ? R(1) - wk : coef;
            coef = sel == 1u ? wk : coef;
            acc += coef * lk;
        }
        lam[c] = acc;
    };

    // first node of this thread in level l (prefetched one level ahead)
    int l = top;
    int s = l > 0 ? b[l - 1] : 0, e = b[l];
    int c0 = -1;
    uint32_t d0 = 0;
    R g0 = R(0);
    if (s + tid < e) {
        c0 = ord[s + tid];
        d0 = D[c0];
        g0 = gv[c0];
    }
    for (; l >= 0; --l) {
        // next level's bounds and first nodes, independent of lambda
        int sn = 0, en = 0, c1 = -1;
        uint32_t d1 = 0;
        R g1 = R(0);
        if (l > 0) {
            sn = l > 1 ? b[l - 2] : 0;
            en = b[l - 1];
            if (sn + tid < en) {
                c1 = ord[sn + tid];
                d1 = D[c1];
                g1 = gv[c1];
            }
        }
        if (c0 >= 0) solve(c0, d0, g0);
        for (int p = s + tid + kLvlThreads; p < e; p += kLvlThreads) {
            const int c = ord[p];
            solve(c, D[c], gv[c]);
        }
        __syncthreads(); // the level's lambdas are written before the next level reads them
        s = sn;
        e = en;
        c0 = c1;
        d0 = d1;
        g0 = g1;
    }
}

#define EIK_TH_DISPATCH_L(TH_VAR, ...)                                                                           \
    do {                                                                                                         \
        if ((TH_VAR) == 64) {                                                                                    \
            constexpr int TH = 64;                                                                               \
            __VA_ARGS__;                                                                                         \
        } else {                                                                                                 \
            constexpr int TH = 32;                                                                               \
            __VA_ARGS__;                                                                                         \
        }                                                                                                        \
    } while (0)

void launch_level_buckets(const LaunchArgs &a, const int32_t *level, int32_t *gmax, int32_t *bins, int32_t *order,
                          hipStream_t st)
{
    launch_fill_i32(gmax, a.n_grids, -1, st);
    EIK_TH_DISPATCH_L(a.th, hipLaunchKernelGGL(k_lvl_max<TH>, dim3(a.n_tiles), dim3(256), 0, st, a, level, gmax));
    hipLaunchKernelGGL(k_lvl_clear, dim3(a.n_grids), dim3(256), 0, st, a, (const int32_t *)gmax, bins);
    EIK_TH_DISPATCH_L(a.th, hipLaunchKernelGGL((k_lvl_bucket<TH, false>), dim3(a.n_tiles), dim3(256), 0, st, a, level,
                                               bins, order));
    hipLaunchKernelGGL(k_lvl_scan, dim3(a.n_grids), dim3(256), 0, st, a, (const int32_t *)gmax, bins);
    EIK_TH_DISPATCH_L(a.th, hipLaunchKernelGGL((k_lvl_bucket<TH, true>), dim3(a.n_tiles), dim3(256), 0, st, a, level,
                                               bins, order));
}

template <typename R>
void launch_level_gather(const LaunchArgs &a, const int32_t *gmax, const int32_t *bins, const int32_t *order,
                         const uint16_t *D, const void *g, const void *w1, void *lam, hipStream_t st)
{
    hipLaunchKernelGGL(k_lvl_gather<R>, dim3(a.n_grids), dim3(kLvlThreads), 0, st, a, gmax, bins, order, D,
                       (const R *)g, (const R *)w1, (R *)lam);
}

template void launch_level_gather<float>(const LaunchArgs &, const int32_t *, const int32_t *, const int32_t *,
                                         const uint16_t *, const void *, const void *, void *, hipStream_t);
template void launch_level_gather<double>(const LaunchArgs &, const int32_t *, const int32_t *, const int32_t *,
                                          const uint16_t *, const void *, const void *, void *, hipStream_t);

} // namespace eik
