// eik_forward.hip -- forward fast-sweeping solve on gfx950 (Sec. 3.2,
// Alg. forward) and the recording of active stencils and dependency levels.
//
// Schedule. The grid is cut into tiles of 64 x TH nodes; one 64-lane wave owns
// a tile, keeps the tile plus a one-node halo of T in LDS and runs the four
// directional sweeps of Fig. sweep_directions over it: columns left-to-right,
// rows bottom-to-top in j (j increasing), columns right-to-left, rows j
// decreasing. Each step updates a whole line of the tile at once, one node per
// lane, reading the previous line (already updated) and the next line (not yet)
// from LDS, so lines are processed in parallel exactly as the column/row
// decomposition describes. A tile repeats four-sweep cycles until one full
// cycle changes nothing, then writes back and flags the neighbour tiles whose
// halo it changed; flagged tiles run in the next round. Rounds end when no
// tile is flagged. The fixed point reached is the one of the discrete local
// update, which does not depend on the order of the updates.
#include "eik_device.h"
#include "eik_internal.h"

namespace eik {

constexpr int TW = 64; // tile width = wave size

// ---------------------------------------------------------------------------
// Initialisation: T, source marks in parent, first active tiles.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_init(GridArgs g, const R *__restrict__ T_init, R *__restrict__ T, uint8_t *__restrict__ parent,
                       int32_t *__restrict__ level)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        T[c] = T_init ? T_init[c] : inf_v<R>();
        parent[c] = kUnreached;
        level[c] = -1;
    }
}

// Sources: times, marks and initial tile flags. Out-of-range indices and
// duplicates are counted in ctr[kCtrBadSource] and otherwise ignored.
template <typename R>
__global__ void k_sources(GridArgs g, const int32_t *__restrict__ src_idx, const R *__restrict__ src_t,
                          R *__restrict__ T, uint8_t *__restrict__ parent, int32_t *__restrict__ act,
                          int32_t *__restrict__ act_count, unsigned long long *__restrict__ ctr)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.n_src) return;
    const int32_t c = src_idx[s];
    if (c < 0 || (int64_t)c >= (int64_t)g.nx * g.ny) {
        atomicAdd(&ctr[kCtrBadSource], 1ull);
        return;
    }
    T[c] = src_t ? src_t[s] : R(0);
    parent[c] = kSource;
    const int i = c % g.nx, j = c / g.nx;
    const int t = (j / g.th) * g.ntx + i / TW;
    if (atomicExch(&act[t], 1) == 0) atomicAdd(&act_count[0], 1);
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        p[c] = v;
}

// Flag every tile that holds a source-free node (warm start, level rounds).
__global__ void k_all_active(int32_t *__restrict__ act, int n_tiles, int32_t *__restrict__ act_count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tiles) act[t] = 1;
    if (t == 0) act_count[0] = n_tiles;
}

// ---------------------------------------------------------------------------
// Tile loading helpers.
// ---------------------------------------------------------------------------
template <typename V, int TH, int LP>
__device__ __forceinline__ void load_tile_halo(const V *__restrict__ src, V *sT, int i0, int j0, int nx, int ny,
                                               V outside)
{
    for (int idx = threadIdx.x; idx < (TH + 2) * (TW + 2); idx += TW) {
        const int r = idx / (TW + 2), c = idx - r * (TW + 2);
        const int gi = i0 + c - 1, gj = j0 + r - 1;
        V v = outside;
        if (gi >= 0 && gi < nx && gj >= 0 && gj < ny) v = src[(size_t)gj * nx + gi];
        sT[r * LP + c] = v;
    }
}

// Bits of the neighbour tiles that see node (ci, cj) of a w x h tile in their
// halo: 0 W, 1 E, 2 S (j-1), 3 N (j+1), 4 SW, 5 SE, 6 NW, 7 NE.
__device__ __forceinline__ int halo_bits(int ci, int cj, int w, int h)
{
    const bool W = ci == 0, E = ci == w - 1, S = cj == 0, N = cj == h - 1;
    return (W ? 1 : 0) | (E ? 2 : 0) | (S ? 4 : 0) | (N ? 8 : 0) | ((S && W) ? 16 : 0) | ((S && E) ? 32 : 0) |
           ((N && W) ? 64 : 0) | ((N && E) ? 128 : 0);
}

__device__ __forceinline__ void flag_neighbours(int bits, int tx, int ty, int ntx, int nty, int32_t *act_out,
                                                int32_t *count_next)
{
    const int DX[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
    const int DY[8] = {0, 0, -1, 1, -1, -1, 1, 1};
    for (int b = 0; b < 8; ++b) {
        if (!(bits & (1 << b))) continue;
        const int ux = tx + DX[b], uy = ty + DY[b];
        if (ux < 0 || ux >= ntx || uy < 0 || uy >= nty) continue;
        const int u = uy * ntx + ux;
        if (atomicExch(&act_out[u], 1) == 0) atomicAdd(count_next, 1);
    }
}

// ---------------------------------------------------------------------------
// One round of tile sweeps.
// ---------------------------------------------------------------------------
template <typename R, int TH>
__global__ __launch_bounds__(TW) void k_sweep_round(GridArgs g, const R *__restrict__ M, const R *__restrict__ om,
                                                    R *__restrict__ T, const uint8_t *__restrict__ parent,
                                                    int32_t *__restrict__ act_in, int32_t *__restrict__ act_out,
                                                    int32_t *__restrict__ count_next,
                                                    unsigned long long *__restrict__ ctr, R tol, int max_cycles)
{
    constexpr int LP = TW + 3; // odd pitch: conflict-free column access
    const int t = blockIdx.x;
    if (act_in[t] == 0) return;
    const int lane = threadIdx.x;
    if (lane == 0) act_in[t] = 0;

    const int tx = t % g.ntx, ty = t / g.ntx;
    const int i0 = tx * TW, j0 = ty * TH;
    const int w = min(TW, g.nx - i0), hgt = min(TH, g.ny - j0);
    const int64_t n = (int64_t)g.nx * g.ny;
    const R h = R(g.h);

    __shared__ R sT[(TH + 2) * LP];
    __shared__ uint8_t sFix[TH * TW];
    load_tile_halo<R, TH, LP>(T, sT, i0, j0, g.nx, g.ny, inf_v<R>());
    for (int idx = lane; idx < TH * TW; idx += TW) {
        const int r = idx / TW, c = idx - r * TW;
        sFix[idx] = (c < w && r < hgt) ? (parent[(size_t)(j0 + r) * g.nx + i0 + c] == kSource) : 1;
    }
    __syncthreads();

    int quiet = 0, sweeps = 0;
    const int max_sweeps = 4 * max_cycles;
    while (quiet < 4 && sweeps < max_sweeps) {
        const int dir = sweeps & 3;
        const bool col = (dir & 1) == 0;
        const int len = col ? w : hgt;
        const int span = col ? hgt : w;
        bool changed = false;
        for (int s = 0; s < len; ++s) {
            const int pos = dir < 2 ? s : len - 1 - s;
            const int ci = col ? pos : lane;
            const int cj = col ? lane : pos;
            if (lane < span && !sFix[cj * TW + ci]) {
                const size_t gc = (size_t)(j0 + cj) * g.nx + (i0 + ci);
                NodeConst<R> k;
                node_const<R>(M[gc], M[n + gc], M[2 * n + gc], om[gc], om[n + gc], h, k);
                R Tn[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) Tn[q] = sT[(cj + 1 + nb_dy(q)) * LP + (ci + 1 + nb_dx(q))];
                int code;
                R w1;
                const R v = local_update<R>(k, Tn, inf_v<R>(), code, w1);
                R &slot = sT[(cj + 1) * LP + ci + 1];
                changed |= counts_as_change<R>(slot, v, tol);
                slot = v;
            }
            __syncthreads();
        }
        ++sweeps;
        quiet = __ballot(changed) ? 0 : quiet + 1;
    }

    // write back; flag neighbours whose halo moved by more than tol
    int bits = 0;
    for (int idx = lane; idx < TH * TW; idx += TW) {
        const int r = idx / TW, c = idx - r * TW;
        if (c >= w || r >= hgt) continue;
        const size_t gc = (size_t)(j0 + r) * g.nx + (i0 + c);
        const R nv = sT[(r + 1) * LP + c + 1];
        const R ov = T[gc];
        if (nv != ov) {
            T[gc] = nv;
            if (counts_as_change<R>(ov, nv, tol)) bits |= halo_bits(c, r, w, hgt);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) bits |= __shfl_xor(bits, off);
    if (lane == 0) {
        flag_neighbours(bits, tx, ty, g.ntx, g.nty, act_out, count_next);
        if (quiet < 4) { // cycle budget ran out before the tile settled
            if (atomicExch(&act_out[t], 1) == 0) atomicAdd(count_next, 1);
        }
        atomicAdd(&ctr[kCtrCellUpdates], (unsigned long long)sweeps * (unsigned long long)(w * hgt));
    }
}

// ---------------------------------------------------------------------------
// Active stencils from the final field (the stencil identification of
// Alg. backward, moved into the forward pass).
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_parents(GridArgs g, const R *__restrict__ M, const R *__restrict__ om, const R *__restrict__ T,
                          uint8_t *__restrict__ parent, int32_t *__restrict__ level)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    const R h = R(g.h);
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        if (parent[c] == kSource) {
            level[c] = 0;
            continue;
        }
        const R Tc = T[c];
        if (!(Tc < inf_v<R>())) {
            parent[c] = kUnreached;
            level[c] = -1;
            continue;
        }
        const int i = (int)(c % g.nx), j = (int)(c / g.nx);
        R Tn[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int a = i + nb_dx(q), b = j + nb_dy(q);
            Tn[q] = (a >= 0 && a < g.nx && b >= 0 && b < g.ny) ? T[(size_t)b * g.nx + a] : inf_v<R>();
        }
        NodeConst<R> k;
        node_const<R>(M[c], M[n + c], M[2 * n + c], om[c], om[n + c], h, k);
        int code;
        R w1;
        local_update<R>(k, Tn, Tc, code, w1);
        parent[c] = (uint8_t)code;
        level[c] = code == kUnreached ? -1 : 0;
    }
}

// ---------------------------------------------------------------------------
// Dependency levels: level = 1 + max level of the donors, relaxed upward with
// the same tile sweeps (the donor graph is acyclic, so this terminates).
// ---------------------------------------------------------------------------
template <int TH>
__global__ __launch_bounds__(TW) void k_level_round(GridArgs g, const uint8_t *__restrict__ parent,
                                                    int32_t *__restrict__ level, int32_t *__restrict__ act_in,
                                                    int32_t *__restrict__ act_out, int32_t *__restrict__ count_next,
                                                    int max_cycles)
{
    constexpr int LP = TW + 3;
    const int t = blockIdx.x;
    if (act_in[t] == 0) return;
    const int lane = threadIdx.x;
    if (lane == 0) act_in[t] = 0;
    const int tx = t % g.ntx, ty = t / g.ntx;
    const int i0 = tx * TW, j0 = ty * TH;
    const int w = min(TW, g.nx - i0), hgt = min(TH, g.ny - j0);

    __shared__ int32_t sL[(TH + 2) * LP];
    __shared__ uint8_t sP[TH * TW];
    load_tile_halo<int32_t, TH, LP>(level, sL, i0, j0, g.nx, g.ny, -1);
    for (int idx = lane; idx < TH * TW; idx += TW) {
        const int r = idx / TW, c = idx - r * TW;
        sP[idx] = (c < w && r < hgt) ? parent[(size_t)(j0 + r) * g.nx + i0 + c] : kUnreached;
    }
    __syncthreads();

    int quiet = 0, sweeps = 0;
    const int max_sweeps = 4 * max_cycles;
    while (quiet < 4 && sweeps < max_sweeps) {
        const int dir = sweeps & 3;
        const bool col = (dir & 1) == 0;
        const int len = col ? w : hgt;
        const int span = col ? hgt : w;
        bool changed = false;
        for (int s = 0; s < len; ++s) {
            const int pos = dir < 2 ? s : len - 1 - s;
            const int ci = col ? pos : lane;
            const int cj = col ? lane : pos;
            const int code = lane < span ? sP[cj * TW + ci] : kUnreached;
            if (code < 16) {
                const int kp = code < 8 ? code : code - 8;
                int lv = sL[(cj + 1 + nb_dy(kp)) * LP + ci + 1 + nb_dx(kp)];
                if (code < 8) {
                    const int kq = (code + 1) & 7;
                    lv = max(lv, sL[(cj + 1 + nb_dy(kq)) * LP + ci + 1 + nb_dx(kq)]);
                }
                int32_t &slot = sL[(cj + 1) * LP + ci + 1];
                const int nv = lv + 1;
                changed |= nv != slot;
                slot = nv;
            }
            __syncthreads();
        }
        ++sweeps;
        quiet = __ballot(changed) ? 0 : quiet + 1;
    }

    int bits = 0;
    for (int idx = lane; idx < TH * TW; idx += TW) {
        const int r = idx / TW, c = idx - r * TW;
        if (c >= w || r >= hgt) continue;
        const size_t gc = (size_t)(j0 + r) * g.nx + (i0 + c);
        const int32_t nv = sL[(r + 1) * LP + c + 1];
        if (nv != level[gc]) {
            level[gc] = nv;
            bits |= halo_bits(c, r, w, hgt);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) bits |= __shfl_xor(bits, off);
    if (lane == 0) {
        flag_neighbours(bits, tx, ty, g.ntx, g.nty, act_out, count_next);
        if (quiet < 4 && atomicExch(&act_out[t], 1) == 0) atomicAdd(count_next, 1);
    }
}

// Largest level (for the level count).
__global__ void k_max_level(int64_t n, const int32_t *__restrict__ level, unsigned long long *__restrict__ ctr)
{
    int m = -1;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        if (level[c] < n) m = max(m, level[c]);
    for (int off = 32; off >= 1; off >>= 1) m = max(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0 && m >= 0) atomicMax(&ctr[kCtrMaxLevel], (unsigned long long)m);
}

// Feasibility check: m11 > 0, det > 0, |omega|_{M^-1} < 1 (and finite).
template <typename R>
__global__ void k_check_feasible(int64_t n, const R *__restrict__ M, const R *__restrict__ om,
                                 unsigned long long *__restrict__ ctr)
{
    int bad = 0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const R m11 = M[c], m12 = M[n + c], m22 = M[2 * n + c], bx = om[c], by = om[n + c];
        const R det = m11 * m22 - m12 * m12;
        const R q = bx * bx * m22 - R(2) * bx * by * m12 + by * by * m11;
        bad |= !(m11 > R(0) && det > R(0) && q < det);
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicAdd(&ctr[kCtrInfeasible], 1ull);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static inline int blocks_for(int64_t n, int bs) { return (int)std::min<int64_t>((n + bs - 1) / bs, 4096); }

template <typename R>
void launch_init(const GridArgs &g, const void *T_init, void *T, uint8_t *parent, int32_t *level,
                 const int32_t *src_idx, const void *src_t, int32_t *act, int32_t *act_count,
                 unsigned long long *ctr, bool warm, hipStream_t st)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    hipLaunchKernelGGL(k_init<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, g, (const R *)T_init, (R *)T, parent,
                       level);
    if (warm)
        hipLaunchKernelGGL(k_all_active, dim3((g.n_tiles + 255) / 256), dim3(256), 0, st, act, g.n_tiles, act_count);
    hipLaunchKernelGGL(k_sources<R>, dim3((g.n_src + 255) / 256), dim3(256), 0, st, g, src_idx, (const R *)src_t,
                       (R *)T, parent, act, act_count, ctr);
}

template <typename R>
void launch_sweep_round(const GridArgs &g, const void *M, const void *om, void *T, const uint8_t *parent,
                        int32_t *act_in, int32_t *act_out, int32_t *count_next, unsigned long long *ctr, double tol,
                        int max_cycles, hipStream_t st)
{
    if (g.th == 64)
        hipLaunchKernelGGL((k_sweep_round<R, 64>), dim3(g.n_tiles), dim3(TW), 0, st, g, (const R *)M, (const R *)om,
                           (R *)T, parent, act_in, act_out, count_next, ctr, R(tol), max_cycles);
    else
        hipLaunchKernelGGL((k_sweep_round<R, 32>), dim3(g.n_tiles), dim3(TW), 0, st, g, (const R *)M, (const R *)om,
                           (R *)T, parent, act_in, act_out, count_next, ctr, R(tol), max_cycles);
}

template <typename R>
void launch_parents(const GridArgs &g, const void *M, const void *om, const void *T, uint8_t *parent,
                    int32_t *level, hipStream_t st)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    hipLaunchKernelGGL(k_parents<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, g, (const R *)M, (const R *)om,
                       (const R *)T, parent, level);
}

void launch_level_prep(const GridArgs &g, int32_t *act, int32_t *act_count, hipStream_t st)
{
    hipLaunchKernelGGL(k_all_active, dim3((g.n_tiles + 255) / 256), dim3(256), 0, st, act, g.n_tiles, act_count);
}

void launch_level_round(const GridArgs &g, const uint8_t *parent, int32_t *level, int32_t *act_in,
                        int32_t *act_out, int32_t *count_next, int max_cycles, hipStream_t st)
{
    if (g.th == 64)
        hipLaunchKernelGGL(k_level_round<64>, dim3(g.n_tiles), dim3(TW), 0, st, g, parent, level, act_in, act_out,
                           count_next, max_cycles);
    else
        hipLaunchKernelGGL(k_level_round<32>, dim3(g.n_tiles), dim3(TW), 0, st, g, parent, level, act_in, act_out,
                           count_next, max_cycles);
}

void launch_max_level(int64_t n, const int32_t *level, unsigned long long *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(k_max_level, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, level, ctr);
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
}

template <typename R>
void launch_check_feasible(int64_t n, const void *M, const void *om, unsigned long long *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_feasible<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, (const R *)M,
                       (const R *)om, ctr);
}

#define EIK_INST(R)                                                                                            \
    template void launch_init<R>(const GridArgs &, const void *, void *, uint8_t *, int32_t *, const int32_t *, \
                                 const void *, int32_t *, int32_t *, unsigned long long *, bool, hipStream_t);  \
    template void launch_sweep_round<R>(const GridArgs &, const void *, const void *, void *, const uint8_t *,  \
                                        int32_t *, int32_t *, int32_t *, unsigned long long *, double, int,     \
                                        hipStream_t);                                                           \
    template void launch_parents<R>(const GridArgs &, const void *, const void *, const void *, uint8_t *,      \
                                    int32_t *, hipStream_t);                                                    \
    template void launch_check_feasible<R>(int64_t, const void *, const void *, unsigned long long *, hipStream_t);
EIK_INST(float)
EIK_INST(double)
#undef EIK_INST

} // namespace eik
