// eik_backward.hip -- adjoint of the converged solve on gfx950 (Sec. 3.3,
// Alg. backward; Eqs. implicit, param_grad, adjoint).
//
// With the active update of node j fixed, dT_j/dT_i is the donor weight w
// (barycentric weight of a two-point update, 1 for a one-point update), so the
// adjoint system J^T lambda = dL/dT is triangular in the causal order and
// reads lambda_i = g_i + sum over the nodes j that i feeds of w_ji lambda_j.
// Instead of sorting all nodes by T, each tile (holding lambda, the donor
// weights and the active updates of the tile plus a one-node halo in LDS)
// relaxes these equations with the same four directional line sweeps as the
// forward pass, each node gathering from its (at most eight) receivers, so
// nothing is scattered and no atomics are needed. On the acyclic donor graph a
// lambda is exact as soon as its receivers are, so the sweeps end at the exact
// solution. Receivers in neighbouring tiles are read from the halo; tiles
// whose halo changed are visited again, until no lambda on a tile border
// changes. dL/dtheta_i = lambda_i dT_i/dtheta_i (Alg. backward, last loop)
// follows in one pass over the nodes.
//
// LDS holds only lambda and the donor weights of a tile with its halo; the
// 16-bit receiver descriptor and dL/dT of each node are built once per
// adjoint (k_adj_stage) and read by the sweeps from global memory, one line
// ahead, from row-major arrays in row sweeps and transposed copies in column
// sweeps, so every load is coalesced and four tiles fit in a CU's LDS.
#include "eik_device.h"
#include "eik_internal.h"
#include "eik_queue.h"
#include "eik_tile.h"

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
                                                  R *__restrict__ w1all, R *__restrict__ lamall, Prep32 p32)
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
                two_point_any<R>(k, code, T[(size_t)yp * g.gd.nx + xp], T[(size_t)yq * g.gd.nx + xq], t, mu1, mu2);
                w = mu1 / (mu1 + mu2);
            }
        }
        w1all[g.gd.off + c] = w;
        lamall[g.gd.off + c] = R(0);
        if (p32.w1) { // the FP32 relaxation's inputs, rounded as a cast would
            p32.w1[g.gd.off + c] = (float)w;
            p32.g[g.gd.off + c] = (float)((const R *)p32.g_src)[g.gd.off + c];
            p32.lam[g.gd.off + c] = 0.0f;
        }
    }
}

// The round state of a relaxation: every tile flagged for round 0, the other
// buffer and every later round's count cleared (one writer per element).
__global__ void k_round_reset(int32_t *__restrict__ act, int n_tiles, int32_t *__restrict__ act_count)
{
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < 2 * (int64_t)n_tiles; i += stride) act[i] = i < n_tiles ? 1 : 0;
    for (int64_t i = tid; i < kMaxRounds + 2; i += stride) act_count[i] = i == 0 ? n_tiles : 0;
}

void launch_round_reset(const LaunchArgs &a, int32_t *act, int32_t *act_count, hipStream_t st)
{
    const int64_t work = std::max<int64_t>(2 * (int64_t)a.n_tiles, kMaxRounds + 2);
    hipLaunchKernelGGL(k_round_reset, dim3(blocks_for(work, 256)), dim3(256), 0, st, act, a.n_tiles, act_count);
}

// One visit of a tile by directional sweeps: lambda_i = g_i + sum over the
// tile's and the halo's receivers j of i of (dT_j/dT_i) lambda_j, the sum in
// neighbour order k = 0..7, relaxed with the four directional line sweeps
// (Gauss-Seidel, a line of the tile per step) until a full four-sweep cycle
// changes nothing or the cycle budget runs out. The donor graph is acyclic,
// so every lambda reaches its exact value once its receivers have theirs, and
// a quiet cycle means every node satisfies its equation for the current halo.
// Each node's receivers and weight selectors are gathered once per visit into
// a 16-bit descriptor (two bits per neighbour: 1 first donor, weight w; 2
// second donor, weight 1 - w; 3 one-point donor, weight 1).
// One directional sweep of the adjoint relaxation over the tile in LDS (a
// line of the tile per step; DIR as in the forward sweeps).
template <typename R, int TH, int DIR>
__device__ __forceinline__ bool adj_sweep_dir(const TileGeoB &g, R *sLam, const R *sW,
                                              const uint16_t *__restrict__ Dsrc, const R *__restrict__ Gsrc)
{
    constexpr int LP = TW + 3;
    constexpr bool COL = (DIR & 1) == 0;
    const int lane = threadIdx.x % TW;
    const int len = COL ? g.w : g.h;
    const int span = COL ? g.h : g.w;
    const int lc = lane < span ? lane : span - 1; // clamped lane for loads
    // descriptor and dL/dT of the node this lane updates at step s (steps past
    // the last line are clamped to it): Dsrc / Gsrc are the transposed arrays
    // of the grid in column sweeps, the row-major ones in row sweeps
    // 32-bit node offsets (grids hold fewer than 2^32 nodes), advanced by one
    // line per step
    const uint32_t stride = COL ? (uint32_t)g.gd.ny : (uint32_t)g.gd.nx;
    const uint32_t base = COL ? (uint32_t)g.i0 * stride + (uint32_t)(g.j0 + lc) : (uint32_t)g.j0 * stride + (uint32_t)(g.i0 + lc);
    auto load = [&](int s, uint32_t &d, R &gv) {
        s = s < len ? s : len - 1;
        const int pos = DIR < 2 ? s : len - 1 - s;
        const uint32_t ad = base + (uint32_t)pos * stride;
        d = Dsrc[ad];
        gv = Gsrc[ad];
    };
    bool changed = false;
    auto step = [&](int s, uint32_t d, R acc) {
        const int pos = DIR < 2 ? s : len - 1 - s;
        const int ci = COL ? pos : lane;
        const int cj = COL ? lane : pos;
        if (lane < span) {
            // all neighbour reads are issued at once and the receivers
            // selected afterwards (no branch per neighbour); non-receivers add
            // an exact zero, so the sum is the same, in the same order
            R lam[8], wn[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int sl = (cj + 1 + nb_dy(k)) * LP + (ci + 1 + nb_dx(k));
                lam[k] = sLam[sl];
                wn[k] = sW[sl];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t sel = (d >> (2 * k)) & 3u;
                // sequential selects (no branches): 0, w, 1 - w or 1
                R coef = sel == 3u ? R(1) : R(0);
                coef = sel == 2u ? R(1) - wn[k] : coef;
                coef = sel == 1u ? wn[k] : coef;
                acc += coef * lam[k];
            }
            const int slot = (cj + 1) * LP + ci + 1;
            changed |= acc != sLam[slot];
            sLam[slot] = acc;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // double-buffered: the next line's inputs load while a line is updated
    uint32_t dX, dY;
    R gX, gY;
    load(0, dX, gX);
    for (int s = 0; s < len; s += 2) {
        load(s + 1, dY, gY);
        step(s, dX, gX);
        if (s + 1 >= len) break; // uniform over the wave
        load(s + 2, dX, gX);
        step(s + 1, dY, gY);
    }
    return changed;
}

struct AdjVisit {
    int bits;
    bool settled;
};

// CD: the workgroup holds four waves that sweep the four directions of each
// cycle at once over the same LDS tile. Every store is a full recomputation of
// a node from its receivers' current values; a store computed from values that
// another wave has since replaced counts as a change, so the cycle repeats. A
// cycle in which no wave changed anything recomputed every node from values
// that stayed fixed, so every equation of the tile holds exactly, as after a
// quiet cycle of the one-wave visit, and the fixed point is the same.
template <typename R, int TH, bool CD>
__device__ __forceinline__ AdjVisit adj_visit_sweep(const LaunchArgs &a, int t, const AdjNodes &nd,
                                                    const R *__restrict__ w1all, R *lamall, int max_cycles, R *sLam,
                                                    R *sW, int *sBits)
{
    constexpr int LP = TW + 3;
    constexpr int NW = CD ? 4 : 1;
    const int lane = threadIdx.x % TW, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / TW); // uniform per wave
    const TileGeoB g = tile_geo_b<TH>(a, t);
    const int nx = g.gd.nx, ny = g.gd.ny;
    R *lam = lamall + g.gd.off;

    load_tile_halo<R, TH, LP>(lam, sLam, nx, ny, g.i0, g.j0, R(0));
    load_tile_halo<R, TH, LP>(w1all + g.gd.off, sW, nx, ny, g.i0, g.j0, R(1));
    if (CD && threadIdx.x == 0) *sBits = 0;
    __syncthreads();
    const uint16_t *D = nd.D + g.gd.off, *DT = nd.DT + g.gd.off;
    const R *G = (const R *)nd.g + g.gd.off, *GT = (const R *)nd.gT + g.gd.off;

    int quiet = 0, sweeps = 0;
    const int max_sweeps = 4 * max_cycles;
    while (quiet < 4 && sweeps < max_sweeps) {
        bool changed;
        switch (CD ? wave : (sweeps & 3)) { // CD: one direction per wave, uniform per wave
        case 0: changed = adj_sweep_dir<R, TH, 0>(g, sLam, sW, DT, GT); break;
        case 1: changed = adj_sweep_dir<R, TH, 1>(g, sLam, sW, D, G); break;
        case 2: changed = adj_sweep_dir<R, TH, 2>(g, sLam, sW, DT, GT); break;
        default: changed = adj_sweep_dir<R, TH, 3>(g, sLam, sW, D, G); break;
        }
        if (CD) { // a cycle is the four concurrent sweeps
            sweeps += 4;
            quiet = __syncthreads_or(changed ? 1 : 0) ? 0 : 4;
        } else {
            ++sweeps;
            quiet = __ballot(changed) ? 0 : quiet + 1;
        }
    }

    // write back (old values re-read in batches), note the neighbours whose
    // halo changed
    int bits = 0;
    const int c = lane;
#pragma unroll 1
    for (int r0 = wave * kLoadBatch; r0 < TH; r0 += NW * kLoadBatch) {
        R ov[kLoadBatch];
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const int r = r0 + k;
            const int rc = r < g.h ? r : g.h - 1, cc = c < g.w ? c : g.w - 1; // in-tile, no branch
            ov[k] = lam[(size_t)(g.j0 + rc) * nx + g.i0 + cc];
        }
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const int r = r0 + k;
            if (r >= g.h || c >= g.w) continue;
            const R nv = sLam[(r + 1) * LP + c + 1];
            if (nv != ov[k]) {
                lam[(size_t)(g.j0 + r) * nx + g.i0 + c] = nv;
                const bool W = c == 0, E = c == g.w - 1, S = r == 0, N = r == g.h - 1;
                bits |= (W ? 1 : 0) | (E ? 2 : 0) | (S ? 4 : 0) | (N ? 8 : 0) | ((S && W) ? 16 : 0) |
                        ((S && E) ? 32 : 0) | ((N && W) ? 64 : 0) | ((N && E) ? 128 : 0);
            }
        }
    }
    for (int off = 32; off >= 1; off >>= 1) bits |= __shfl_xor(bits, off);
    if (CD) {
        if (lane == 0 && bits) atomicOr(sBits, bits);
        __syncthreads();
        bits = *sBits;
    }
    AdjVisit v;
    v.bits = bits;
    v.settled = quiet >= 4;
    return v;
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

// Round scheduler with sweep visits (CD: four waves per tile).
template <typename R, int TH, bool CD>
__global__ __launch_bounds__(CD ? 4 * TW : TW) void k_adj_sweep_round(LaunchArgs a, AdjNodes nd,
                                                                      const R *__restrict__ w1all,
                                                                      R *__restrict__ lamall, int max_cycles,
                                                                      int32_t *__restrict__ act_in,
                                                                      int32_t *__restrict__ act_out,
                                                                      int32_t *__restrict__ count_next)
{
    constexpr int LP = TW + 3;
    const int t = blockIdx.x;
    if (act_in[t] == 0) return; // uniform over the workgroup
    __shared__ R sLam[(TH + 2) * LP];
    __shared__ R sW[(TH + 2) * LP];
    __shared__ int sBits;
    if (CD) __syncthreads(); // every wave has read act_in[t] before it is cleared
    if (threadIdx.x == 0) act_in[t] = 0;
    const AdjVisit v = adj_visit_sweep<R, TH, CD>(a, t, nd, w1all, lamall, max_cycles, sLam, sW, &sBits);
    if (threadIdx.x == 0) {
        const TileGeoB g = tile_geo_b<TH>(a, t);
        for (int b = 0; b < 8; ++b) {
            if (!(v.bits & (1 << b))) continue;
            const int u = adj_neighbour(g, b);
            if (u >= 0 && atomicExch(&act_out[u], 1) == 0) atomicAdd(count_next, 1);
        }
        if (!v.settled && atomicExch(&act_out[t], 1) == 0) atomicAdd(count_next, 1);
    }
}

// Work-queue scheduler with sweep visits.
template <typename R, int TH>
__global__ __launch_bounds__(TW) void k_adj_sweep_queue(LaunchArgs a, AdjNodes nd, const R *__restrict__ w1all,
                                                        R *lamall, int max_cycles, WorkQueue q)
{
    constexpr int LP = TW + 3;
    __shared__ R sLam[(TH + 2) * LP];
    __shared__ R sW[(TH + 2) * LP];
    for (;;) {
        int t = threadIdx.x == 0 ? q_take(q) : 0;
        t = __shfl(t, 0);
        if (t < 0) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const AdjVisit v =
            adj_visit_sweep<R, TH, false>(a, t, nd, w1all, lamall, max_cycles, sLam, sW, nullptr);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0) {
            const TileGeoB g = tile_geo_b<TH>(a, t);
            for (int b = 0; b < 8; ++b) {
                if (!(v.bits & (1 << b))) continue;
                const int u = adj_neighbour(g, b);
                if (u >= 0) q_flag(q, u);
            }
            q_done(q, t, v.settled);
        }
        __syncthreads(); // LDS reuse by the next visit
    }
}

// Per-node inputs of the relaxation sweeps, once per adjoint: the receiver
// descriptor of each node (two bits per neighbour k: 1 if k's active update is
// the two-point stencil whose first donor is this node (weight w of k), 2 if
// it is the one whose second donor is this node (weight 1 - w), 3 if it is the
// one-point update from this node (weight 1), 0 otherwise; neighbours outside
// the grid count as unreached), row-major D and transposed DT, and the
// transposed copy GT of dL/dT.
template <typename R, int TH>
__global__ __launch_bounds__(256) void k_adj_stage(LaunchArgs a, const uint8_t *__restrict__ parall,
                                                   const R *__restrict__ gall, uint16_t *__restrict__ D,
                                                   uint16_t *__restrict__ DT, R *__restrict__ GT)
{
    __shared__ uint16_t bd[TH][TW + 2];
    __shared__ R bg[TH][TW + 1];
    const TileGeoB g = tile_geo_b<TH>(a, blockIdx.x);
    const int nx = g.gd.nx, ny = g.gd.ny;
    const uint8_t *par = parall + g.gd.off;
    for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
        const int r = idx / TW, c = idx - r * TW;
        if (r >= g.h || c >= g.w) continue;
        const int i = g.i0 + c, j = g.j0 + r;
        uint32_t d = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int x = i + nb_dx(k), y = j + nb_dy(k);
            const int pc = (x >= 0 && x < nx && y >= 0 && y < ny) ? (int)par[(size_t)y * nx + x] : (int)kUnreached;
            const int kk = (k + 4) & 7; // this node seen from the neighbour
            const uint32_t sel = pc == kk ? 1u : (pc == ((kk + 7) & 7) ? 2u : (pc == 8 + kk ? 3u : 0u));
            d |= sel << (2 * k);
        }
        const size_t c0 = (size_t)j * nx + i;
        D[g.gd.off + c0] = (uint16_t)d;
        bd[r][c] = (uint16_t)d;
        bg[r][c] = gall[g.gd.off + c0];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
        const int c = idx / TH, r = idx - c * TH;
        if (r >= g.h || c >= g.w) continue;
        const size_t t0 = (size_t)(g.i0 + c) * ny + g.j0 + r;
        DT[g.gd.off + t0] = bd[r][c];
        GT[g.gd.off + t0] = bg[r][c];
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
                     void *w1, void *lam, hipStream_t st, const Prep32 &p32)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_adj_prep<R, TH>), dim3(a.n_tiles), dim3(256), 0, st, a,
                                             (const R *)M, (const R *)om, (const R *)T, parent, (R *)w1, (R *)lam,
                                             p32));
}

template <typename R>
void launch_adj_stage(const LaunchArgs &a, const uint8_t *parent, const void *g, uint16_t *D, uint16_t *DT, void *gT,
                      hipStream_t st)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_adj_stage<R, TH>), dim3(a.n_tiles), dim3(256), 0, st, a, parent,
                                             (const R *)g, D, DT, (R *)gT));
}

template <typename R>
void launch_adj_round(const LaunchArgs &a, const AdjNodes &nd, const void *w1, void *lam, int max_cycles, int waves,
                      int32_t *act_in, int32_t *act_out, int32_t *count_next, hipStream_t st)
{
#define EIK_ADJ_ROUND(CD)                                                                                        \
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_adj_sweep_round<R, TH, CD>), dim3(a.n_tiles), dim3(CD ? 4 * TW : TW), \
                                             0, st, a, nd, (const R *)w1, (R *)lam, max_cycles, act_in, act_out,  \
                                             count_next))
    if (waves >= 4) EIK_ADJ_ROUND(true);
    else EIK_ADJ_ROUND(false);
#undef EIK_ADJ_ROUND
}

template <typename R>
void launch_adj_queue(const LaunchArgs &a, int n_waves, const AdjNodes &nd, const void *w1, void *lam,
                      int max_cycles, const WorkQueue &q, hipStream_t st)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_adj_sweep_queue<R, TH>), dim3(n_waves), dim3(TW), 0, st, a, nd,
                                             (const R *)w1, (R *)lam, max_cycles, q));
}

int adj_queue_waves(int th, int dtype)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e;
    if (dtype == 1)
        e = th == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_sweep_queue<double, 64>, TW, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_sweep_queue<double, 32>, TW, 0);
    else
        e = th == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_sweep_queue<float, 64>, TW, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_sweep_queue<float, 32>, TW, 0);
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
                                     const uint8_t *, void *, void *, hipStream_t, const Prep32 &);             \
    template void launch_adj_stage<R>(const LaunchArgs &, const uint8_t *, const void *, uint16_t *, uint16_t *, \
                                      void *, hipStream_t);                                                      \
    template void launch_adj_round<R>(const LaunchArgs &, const AdjNodes &, const void *, void *, int, int,     \
                                      int32_t *, int32_t *, int32_t *, hipStream_t);                             \
    template void launch_adj_queue<R>(const LaunchArgs &, int, const AdjNodes &, const void *, void *, int,     \
                                      const WorkQueue &, hipStream_t);                                           \
    template void launch_adj_params<R>(const LaunchArgs &, const void *, const uint8_t *, const void *,         \
                                       const void *, void *, void *, hipStream_t);                               \
    template void launch_dsrc<R>(const LaunchArgs &, const int32_t *, const void *, void *, hipStream_t);
EIK_INST(float)
EIK_INST(double)
#undef EIK_INST

} // namespace eik
