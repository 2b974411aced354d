// eik_backward.hip -- adjoint of the converged solve on gfx950 (Sec. 3.3,
// Alg. backward; Eqs. implicit, param_grad, adjoint).
//
// With the active update of node j fixed, dT_j/dT_i is the donor weight w
// (barycentric weight of a two-point update, 1 for a one-point update), so the
// adjoint system J^T lambda = dL/dT is triangular in the causal order and
// reads lambda_i = g_i + sum over the nodes j that i feeds of w_ji lambda_j.
// Instead of sorting by T, nodes are ordered by dependency level: a node's
// receivers all sit at deeper levels. Each tile keeps its nodes sorted by
// decreasing level (a counting sort done once) and, holding lambda, the donor
// weights and the active updates of the tile plus a one-node halo in LDS,
// processes its levels from the deepest down; all nodes of one level gather
// from their (at most eight) receivers at once, and nothing is scattered, so
// no atomics are needed. Receivers in neighbouring tiles are read from the
// halo; tiles whose halo changed run again in the next round, and the rounds
// end when no lambda on a tile border changes -- then every lambda satisfies
// its equation exactly, as a single global level-by-level pass would give.
// dL/dtheta_i = lambda_i dT_i/dtheta_i (Alg. backward, last loop) follows in
// one pass over the nodes.
#include "eik_device.h"
#include "eik_internal.h"
#include "eik_queue.h"

namespace eik {

struct TileGeoB {
    GridDesc gd;
    int tx, ty, i0, j0, w, h;
};

template <int TH>
__device__ __forceinline__ TileGeoB tile_geo_b(const LaunchArgs &a, int t)
{
    TileGeoB g;
    g.gd = a.grids[a.tile_grid[t]];
    const int lt = t - g.gd.tile_base;
    g.tx = lt % g.gd.ntx;
    g.ty = lt / g.gd.ntx;
    g.i0 = g.tx * TW;
    g.j0 = g.ty * TH;
    g.w = min(TW, g.gd.nx - g.i0);
    g.h = min(TH, g.gd.ny - g.j0);
    return g;
}

// Donor weights of each active two-point update; lambda cleared.
template <typename R, int TH>
__global__ __launch_bounds__(256) void k_adj_prep(LaunchArgs a, const R *__restrict__ M, const R *__restrict__ om,
                                                  const R *__restrict__ Tall, const uint8_t *__restrict__ parall,
                                                  R *__restrict__ w1all, R *__restrict__ lamall)
{
    const TileGeoB g = tile_geo_b<TH>(a, blockIdx.x);
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const R *T = Tall + g.gd.off;
    const R *Mg = M + 3 * g.gd.off, *og = om + 2 * g.gd.off;
    const R h = R(g.gd.h), inv_h = R(1) / R(g.gd.h);
    for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
        const int r = idx / TW, cl = idx - r * TW;
        if (r >= g.h || cl >= g.w) continue;
        const int i = g.i0 + cl, j = g.j0 + r;
        const size_t c = (size_t)j * g.gd.nx + i;
        const int code = parall[g.gd.off + c];
        R w = R(1);
        if (code < 8) {
            const int kq = (code + 1) & 7;
            const int xp = i + nb_dx(code), yp = j + nb_dy(code), xq = i + nb_dx(kq), yq = j + nb_dy(kq);
            if (xp >= 0 && xp < g.gd.nx && yp >= 0 && yp < g.gd.ny && xq >= 0 && xq < g.gd.nx && yq >= 0 &&
                yq < g.gd.ny) {
                NodeConst<R> k;
                node_const<R>(Mg[c], Mg[n + c], Mg[2 * n + c], og[c], og[n + c], h, inv_h, k);
                R t, mu1, mu2;
                two_point<R>(k, code, T[(size_t)yp * g.gd.nx + xp], T[(size_t)yq * g.gd.nx + xq], t, mu1, mu2);
                w = mu1 / (mu1 + mu2);
            }
        }
        w1all[g.gd.off + c] = w;
        lamall[g.gd.off + c] = R(0);
    }
}

// Per tile: reached nodes sorted by decreasing level into the tile's segment
// of `list` (local indices r * 64 + c), count in cnt[tile]. Counting sort in
// LDS, in chunks of kSortChunk levels.
template <int TH>
__global__ __launch_bounds__(256) void k_adj_sort(LaunchArgs a, const int32_t *__restrict__ levall,
                                                  int32_t *__restrict__ list, int32_t *__restrict__ cnt)
{
    __shared__ int32_t hist[kSortChunk];
    __shared__ int32_t part[256];
    __shared__ int32_t s_lo, s_hi, s_base;
    const int t = blockIdx.x;
    const TileGeoB g = tile_geo_b<TH>(a, t);
    const int32_t *level = levall + g.gd.off;
    int32_t *seg = list + (size_t)t * TW * TH;
    if (threadIdx.x == 0) {
        s_lo = 0x7fffffff;
        s_hi = -1;
        s_base = 0;
    }
    __syncthreads();
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    int lo = 0x7fffffff, hi = -1;
    for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
        const int r = idx / TW, c = idx - r * TW;
        if (r >= g.h || c >= g.w) continue;
        const int lv = level[(size_t)(g.j0 + r) * g.gd.nx + g.i0 + c];
        if (lv >= 0 && lv < n) {
            lo = min(lo, lv);
            hi = max(hi, lv);
        }
    }
    atomicMin(&s_lo, lo);
    atomicMax(&s_hi, hi);
    __syncthreads();
    lo = s_lo;
    hi = s_hi;
    if (hi < 0) {
        if (threadIdx.x == 0) cnt[t] = 0;
        return;
    }
    for (int k0 = 0; k0 <= hi - lo; k0 += kSortChunk) {
        for (int b = threadIdx.x; b < kSortChunk; b += blockDim.x) hist[b] = 0;
        __syncthreads();
        for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
            const int r = idx / TW, c = idx - r * TW;
            if (r >= g.h || c >= g.w) continue;
            const int lv = level[(size_t)(g.j0 + r) * g.gd.nx + g.i0 + c];
            const int key = hi - lv - k0;
            if (lv >= 0 && lv < n && key >= 0 && key < kSortChunk) atomicAdd(&hist[key], 1);
        }
        __syncthreads();
        // exclusive scan of hist: 16 entries per thread, then across threads
        constexpr int PER = kSortChunk / 256;
        int sum = 0;
        for (int q = 0; q < PER; ++q) sum += hist[threadIdx.x * PER + q];
        part[threadIdx.x] = sum;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        int run = s_base + part[threadIdx.x] - sum;
        for (int q = 0; q < PER; ++q) {
            const int v = hist[threadIdx.x * PER + q];
            hist[threadIdx.x * PER + q] = run;
            run += v;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
            const int r = idx / TW, c = idx - r * TW;
            if (r >= g.h || c >= g.w) continue;
            const int lv = level[(size_t)(g.j0 + r) * g.gd.nx + g.i0 + c];
            const int key = hi - lv - k0;
            if (lv >= 0 && lv < n && key >= 0 && key < kSortChunk) seg[atomicAdd(&hist[key], 1)] = r * TW + c;
        }
        __syncthreads();
        if (threadIdx.x == 255) s_base += part[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[t] = s_base;
}

// One visit of a tile: lambda of every reached node of the tile, levels
// deepest first, from the receivers' lambda (inside the tile, or in the halo
// as last written back by the neighbours). Returns the halo bits of the
// neighbours whose halo changed (OR over the wave).
template <typename R, int TH>
__device__ __forceinline__ int adj_visit(const LaunchArgs &a, int t, const uint8_t *__restrict__ parall,
                                         const int32_t *__restrict__ levall, const R *__restrict__ w1all,
                                         const R *__restrict__ gall, const int32_t *__restrict__ list,
                                         const int32_t *__restrict__ cnt, R *lamall, R *sLam, R *sW, uint8_t *sP)
{
    constexpr int LP = TW + 3;
    const int lane = threadIdx.x;
    const TileGeoB g = tile_geo_b<TH>(a, t);
    const int nx = g.gd.nx, ny = g.gd.ny;
    R *lam = lamall + g.gd.off;
    const int32_t *level = levall + g.gd.off;
    const R *gT = gall + g.gd.off;

    for (int idx = lane; idx < (TH + 2) * (TW + 2); idx += TW) {
        const int r = idx / (TW + 2), c = idx - r * (TW + 2);
        const int gi = g.i0 + c - 1, gj = g.j0 + r - 1;
        R lv = R(0), wv = R(1);
        uint8_t pv = kUnreached;
        if (gi >= 0 && gi < nx && gj >= 0 && gj < ny) {
            const size_t gc = (size_t)gj * nx + gi;
            lv = lam[gc];
            wv = w1all[g.gd.off + gc];
            pv = parall[g.gd.off + gc];
        }
        sLam[r * LP + c] = lv;
        sW[r * LP + c] = wv;
        sP[r * LP + c] = pv;
    }
    __syncthreads();

    const int count = cnt[t];
    const int32_t *seg = list + (size_t)t * TW * TH;
    // chunk of 64 sorted entries per pass; the next chunk's entry, level and
    // dL/dT are loaded while the current one is processed
    auto fetch = [&](int base, int &e, int &lv, R &gv) {
        const bool have = base + lane < count;
        e = have ? seg[base + lane] : -1;
        const int rr = have ? e / TW : 0, cc = have ? e - rr * TW : 0;
        const size_t gc = (size_t)(g.j0 + rr) * nx + g.i0 + cc;
        lv = have ? level[gc] : -1;
        gv = have ? gT[gc] : R(0);
    };
    int e_n, lv_n;
    R g_n;
    fetch(0, e_n, lv_n, g_n);
    for (int base = 0; base < count; base += TW) {
        const int e = e_n;
        int lv = lv_n;
        const R gi = g_n;
        if (base + TW < count) fetch(base + TW, e_n, lv_n, g_n);
        const bool have = e >= 0;
        const int r = have ? e / TW : 0, c = have ? e - r * TW : 0;
        bool done = !have;
        // levels inside the chunk are non-increasing; take them deepest first
        while (__ballot(!done)) {
            int cur = done ? -1 : lv;
            for (int off = 32; off >= 1; off >>= 1) cur = max(cur, __shfl_xor(cur, off));
            const bool mine = !done && lv == cur;
            if (mine) {
                R acc = gi;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int sl = (r + 1 + nb_dy(k)) * LP + (c + 1 + nb_dx(k));
                    const int pc = sP[sl];
                    const int kk = (k + 4) & 7; // this node seen from the neighbour
                    if (pc == kk)
                        acc += sW[sl] * sLam[sl];
                    else if (pc == ((kk + 7) & 7))
                        acc += (R(1) - sW[sl]) * sLam[sl];
                    else if (pc == 8 + kk)
                        acc += sLam[sl];
                }
                sLam[(r + 1) * LP + c + 1] = acc;
                done = true;
            }
            // one-wave workgroup: LDS requests are served in issue order, so
            // only compiler motion across the level boundary is blocked
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }

    int bits = 0;
    for (int idx = lane; idx < TH * TW; idx += TW) {
        const int r = idx / TW, c = idx - r * TW;
        if (c >= g.w || r >= g.h) continue;
        const size_t gc = (size_t)(g.j0 + r) * nx + (g.i0 + c);
        const R nv = sLam[(r + 1) * LP + c + 1];
        if (nv != lam[gc]) {
            lam[gc] = nv;
            const bool W = c == 0, E = c == g.w - 1, S = r == 0, N = r == g.h - 1;
            bits |= (W ? 1 : 0) | (E ? 2 : 0) | (S ? 4 : 0) | (N ? 8 : 0) | ((S && W) ? 16 : 0) |
                    ((S && E) ? 32 : 0) | ((N && W) ? 64 : 0) | ((N && E) ? 128 : 0);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) bits |= __shfl_xor(bits, off);
    return bits;
}

// tile index of the neighbour in halo-bit direction b, or -1 outside the grid
__device__ __forceinline__ int adj_neighbour(const TileGeoB &g, int b)
{
    const int DX[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
    const int DY[8] = {0, 0, -1, 1, -1, -1, 1, 1};
    const int ux = g.tx + DX[b], uy = g.ty + DY[b];
    if (ux < 0 || ux >= g.gd.ntx || uy < 0 || uy >= g.gd.nty) return -1;
    return g.gd.tile_base + uy * g.gd.ntx + ux;
}

// One round of the tile-local level-descending gather.
template <typename R, int TH>
__global__ __launch_bounds__(TW) void k_adj_round(LaunchArgs a, const uint8_t *__restrict__ parall,
                                                  const int32_t *__restrict__ levall, const R *__restrict__ w1all,
                                                  const R *__restrict__ gall, const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ cnt, R *__restrict__ lamall,
                                                  int32_t *__restrict__ act_in, int32_t *__restrict__ act_out,
                                                  int32_t *__restrict__ count_next)
{
    constexpr int LP = TW + 3;
    const int t = blockIdx.x;
    if (act_in[t] == 0) return;
    if (threadIdx.x == 0) act_in[t] = 0;
    __shared__ R sLam[(TH + 2) * LP];
    __shared__ R sW[(TH + 2) * LP];
    __shared__ uint8_t sP[(TH + 2) * LP];
    const int bits = adj_visit<R, TH>(a, t, parall, levall, w1all, gall, list, cnt, lamall, sLam, sW, sP);
    if (threadIdx.x == 0) {
        const TileGeoB g = tile_geo_b<TH>(a, t);
        for (int b = 0; b < 8; ++b) {
            if (!(bits & (1 << b))) continue;
            const int u = adj_neighbour(g, b);
            if (u >= 0 && atomicExch(&act_out[u], 1) == 0) atomicAdd(count_next, 1);
        }
    }
}

// Work-queue form: one launch; waves take flagged tiles from the device
// queue (same protocol as the forward's queue scheduler), visit them and flag
// the neighbours whose halo changed.
template <typename R, int TH>
__global__ __launch_bounds__(TW) void k_adj_queue(LaunchArgs a, const uint8_t *__restrict__ parall,
                                                  const int32_t *__restrict__ levall, const R *__restrict__ w1all,
                                                  const R *__restrict__ gall, const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ cnt, R *lamall, WorkQueue q)
{
    constexpr int LP = TW + 3;
    __shared__ R sLam[(TH + 2) * LP];
    __shared__ R sW[(TH + 2) * LP];
    __shared__ uint8_t sP[(TH + 2) * LP];
    for (;;) {
        int t = threadIdx.x == 0 ? q_take(q) : 0;
        t = __shfl(t, 0);
        if (t < 0) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int bits = adj_visit<R, TH>(a, t, parall, levall, w1all, gall, list, cnt, lamall, sLam, sW, sP);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0) {
            const TileGeoB g = tile_geo_b<TH>(a, t);
            for (int b = 0; b < 8; ++b) {
                if (!(bits & (1 << b))) continue;
                const int u = adj_neighbour(g, b);
                if (u >= 0) q_flag(q, u);
            }
            q_done(q, t, true);
        }
        __syncthreads(); // LDS reuse by the next visit
    }
}

// dL/dtheta_i = lambda_i dT_i/dtheta_i for reached non-source nodes, 0 elsewhere.
template <typename R, int TH>
__global__ __launch_bounds__(256) void k_adj_params(LaunchArgs a, const R *__restrict__ M,
                                                    const uint8_t *__restrict__ parall, const R *__restrict__ w1all,
                                                    const R *__restrict__ lamall, R *__restrict__ dM,
                                                    R *__restrict__ dom)
{
    const TileGeoB g = tile_geo_b<TH>(a, blockIdx.x);
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const R *Mg = M + 3 * g.gd.off;
    R *dMg = dM + 3 * g.gd.off, *dog = dom + 2 * g.gd.off;
    const R h = R(g.gd.h);
    for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
        const int r = idx / TW, cl = idx - r * TW;
        if (r >= g.h || cl >= g.w) continue;
        const size_t c = (size_t)(g.j0 + r) * g.gd.nx + g.i0 + cl;
        const int code = parall[g.gd.off + c];
        R d[5] = {R(0), R(0), R(0), R(0), R(0)};
        if (code < 16) {
            param_derivs<R>(code, w1all[g.gd.off + c], Mg[c], Mg[n + c], Mg[2 * n + c], h, d);
            const R l = lamall[g.gd.off + c];
#pragma unroll
            for (int q = 0; q < 5; ++q) d[q] *= l;
        }
        dMg[c] = d[0];
        dMg[n + c] = d[1];
        dMg[2 * n + c] = d[2];
        dog[c] = d[3];
        dog[n + c] = d[4];
    }
}

template <typename R>
__global__ void k_dsrc(LaunchArgs a, const int32_t *__restrict__ src_idx, const R *__restrict__ lam,
                       R *__restrict__ dsrc)
{
    const GridDesc gd = a.grids[blockIdx.x];
    for (int s = threadIdx.x; s < gd.n_src; s += blockDim.x) {
        const int c = src_idx[gd.src_base + s];
        dsrc[gd.src_base + s] = (c >= 0 && (int64_t)c < (int64_t)gd.nx * gd.ny) ? lam[gd.off + c] : R(0);
    }
}

// ---------------------------------------------------------------------------
#define EIK_TH_DISPATCH(TH_VAR, ...)                                                                             \
    do {                                                                                                         \
        if ((TH_VAR) == 64) {                                                                                    \
            constexpr int TH = 64;                                                                               \
            __VA_ARGS__;                                                                                         \
        } else {                                                                                                 \
            constexpr int TH = 32;                                                                               \
            __VA_ARGS__;                                                                                         \
        }                                                                                                        \
    } while (0)

template <typename R>
void launch_adj_prep(const LaunchArgs &a, const void *M, const void *om, const void *T, const uint8_t *parent,
                     void *w1, void *lam, hipStream_t st)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_adj_prep<R, TH>), dim3(a.n_tiles), dim3(256), 0, st, a,
                                             (const R *)M, (const R *)om, (const R *)T, parent, (R *)w1, (R *)lam));
}

void launch_adj_sort(const LaunchArgs &a, const int32_t *level, int32_t *list, int32_t *cnt, hipStream_t st)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL(k_adj_sort<TH>, dim3(a.n_tiles), dim3(256), 0, st, a, level, list, cnt));
}

template <typename R>
void launch_adj_round(const LaunchArgs &a, const uint8_t *parent, const int32_t *level, const void *w1,
                      const void *dLdT, const int32_t *list, const int32_t *cnt, void *lam, int32_t *act_in,
                      int32_t *act_out, int32_t *count_next, hipStream_t st)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_adj_round<R, TH>), dim3(a.n_tiles), dim3(TW), 0, st, a, parent,
                                             level, (const R *)w1, (const R *)dLdT, list, cnt, (R *)lam, act_in,
                                             act_out, count_next));
}

template <typename R>
void launch_adj_queue(const LaunchArgs &a, int n_waves, const uint8_t *parent, const int32_t *level, const void *w1,
                      const void *dLdT, const int32_t *list, const int32_t *cnt, void *lam, const WorkQueue &q,
                      hipStream_t st)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_adj_queue<R, TH>), dim3(n_waves), dim3(TW), 0, st, a, parent, level,
                                             (const R *)w1, (const R *)dLdT, list, cnt, (R *)lam, q));
}

int adj_queue_waves(int th, int dtype)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e;
    if (dtype == 1)
        e = th == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_queue<double, 64>, TW, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_queue<double, 32>, TW, 0);
    else
        e = th == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_queue<float, 64>, TW, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_queue<float, 32>, TW, 0);
    if (e != hipSuccess) return 0;
    return std::max(1, per_cu) * cus;
}

template <typename R>
void launch_adj_params(const LaunchArgs &a, const void *M, const uint8_t *parent, const void *w1, const void *lam,
                       void *dM, void *dom, hipStream_t st)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_adj_params<R, TH>), dim3(a.n_tiles), dim3(256), 0, st, a,
                                             (const R *)M, parent, (const R *)w1, (const R *)lam, (R *)dM,
                                             (R *)dom));
}

template <typename R>
void launch_dsrc(const LaunchArgs &a, const int32_t *src_idx, const void *lam, void *dsrc, hipStream_t st)
{
    hipLaunchKernelGGL(k_dsrc<R>, dim3(a.n_grids), dim3(64), 0, st, a, src_idx, (const R *)lam, (R *)dsrc);
}

#define EIK_INST(R)                                                                                              \
    template void launch_adj_prep<R>(const LaunchArgs &, const void *, const void *, const void *,              \
                                     const uint8_t *, void *, void *, hipStream_t);                             \
    template void launch_adj_round<R>(const LaunchArgs &, const uint8_t *, const int32_t *, const void *,        \
                                      const void *, const int32_t *, const int32_t *, void *, int32_t *,         \
                                      int32_t *, int32_t *, hipStream_t);                                        \
    template void launch_adj_queue<R>(const LaunchArgs &, int, const uint8_t *, const int32_t *, const void *,  \
                                      const void *, const int32_t *, const int32_t *, void *, const WorkQueue &, \
                                      hipStream_t);                                                              \
    template void launch_adj_params<R>(const LaunchArgs &, const void *, const uint8_t *, const void *,         \
                                       const void *, void *, void *, hipStream_t);                               \
    template void launch_dsrc<R>(const LaunchArgs &, const int32_t *, const void *, void *, hipStream_t);
EIK_INST(float)
EIK_INST(double)
#undef EIK_INST

} // namespace eik
