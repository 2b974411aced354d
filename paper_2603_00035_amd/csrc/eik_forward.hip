// eik_forward.hip -- forward fast-sweeping solve on gfx950 (Sec. 3.2,
// Alg. forward) and the recording of active stencils and dependency levels.
//
// Schedule. Each grid is cut into tiles of 64 x TH nodes; one 64-lane wave owns
// a tile, keeps T and the dependency levels of the tile plus a one-node halo in
// LDS, and runs the four directional sweeps of Fig. sweep_directions over it:
// columns with x increasing, rows with y increasing, columns with x
// decreasing, rows with y decreasing. Each step updates a whole line of the
// tile at once, one node per lane, reading the line updated just before and
// the line ahead from LDS; the line's parameters are loaded one step ahead
// (columns read a transposed copy, so every load is coalesced). A tile repeats
// four-sweep cycles until a full cycle changes nothing, writes back, and flags
// the neighbour tiles whose halo it changed; flagged tiles run in the next
// round, and rounds end when no tile is flagged.
//
// Two update modes. FULL: every candidate, the new value overwrites T (warm
// starts, and the rounds that certify the final field). FAST, used from the
// cold start where T only decreases: each direction evaluates the candidates
// whose donors lie on the line just updated or on the current line, and keeps
// the smaller of the old and the new value. Both converge to the fixed point of
// the full local update; the solve always ends with FULL rounds, so the field
// returned is a fixed point of the full update to the requested tolerance.
//
// The active update (code) and the dependency level of each node are carried
// along with T, so the level field is settled when T is.
#include "eik_device.h"
#include "eik_internal.h"
#include "eik_queue.h"
#include "eik_tile.h"

namespace eik {

// ---------------------------------------------------------------------------
// Descriptors and staging.
// ---------------------------------------------------------------------------
__global__ void k_write_single_desc(GridDesc d, GridDesc *__restrict__ dst, int32_t *__restrict__ tile_grid,
                                    int n_tiles)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) *dst = d;
    if (t < n_tiles) tile_grid[t] = 0;
}

struct TileGeo {
    GridDesc gd;
    int tx, ty, i0, j0, w, h;
};

template <int TH>
__device__ __forceinline__ TileGeo tile_geo(const LaunchArgs &a, int t)
{
    TileGeo g;
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

// Staged per-node inputs of the sweeps, once per solve. The staging region
// holds, for all grids, first the transposed planes Pt[cols][nx][ny] of each
// grid at cols * off: the five parameters and, in FP64, node_roots' values;
// then, in FP64, the row-major root planes Pc[kRoots][ny][nx] of each grid at
// cols * n_nodes + kRoots * off. Column sweeps read Pt, row sweeps the
// caller's M and omega (and Pc), so every load is coalesced. FP64 sweeps read
// the roots instead of computing them in every line step (the correctly
// rounded FP64 square root and reciprocal are instruction sequences); FP32
// sweeps compute them (one instruction each), which costs less than the
// six more loads per step.
template <typename R>
struct Staged {
    static constexpr bool roots = sizeof(R) == 8;
    static constexpr int cols = roots ? 5 + kRoots : 5;
};

template <typename R>
__device__ __forceinline__ const R *staged_cols(const LaunchArgs &a, const R *Ptall, const GridDesc &gd)
{
    return Ptall + Staged<R>::cols * gd.off;
}

template <typename R>
__device__ __forceinline__ const R *staged_roots_rows(const LaunchArgs &a, const R *Ptall, const GridDesc &gd)
{
    return Staged<R>::roots ? Ptall + Staged<R>::cols * a.n_nodes + kRoots * gd.off : nullptr;
}

template <typename R, int TH>
__device__ __forceinline__ void stage_tile(const LaunchArgs &a, int t, const R *__restrict__ M,
                                           const R *__restrict__ om, R *__restrict__ Pt)
{
    constexpr int kCols = Staged<R>::cols;
    __shared__ R buf[TH][TW + 1];
    const TileGeo g = tile_geo<TH>(a, t);
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const R *Mg = M + 3 * g.gd.off;
    R *Pc = Pt + kCols * a.n_nodes + kRoots * g.gd.off;
    if (Staged<R>::roots) { // row-major roots
        for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
            const int r = idx / TW, c = idx - r * TW;
            if (r >= g.h || c >= g.w) continue;
            const size_t ad = (size_t)(g.j0 + r) * g.gd.nx + g.i0 + c;
            R rt[kRoots];
            node_roots<R>(Mg[ad], Mg[n + ad], Mg[2 * n + ad], rt);
#pragma unroll
            for (int q = 0; q < kRoots; ++q) Pc[q * n + ad] = rt[q];
        }
        __syncthreads(); // this block's root planes are read back below
    }
    for (int p = 0; p < kCols; ++p) {
        const R *src = p < 3 ? Mg + p * n : (p < 5 ? om + 2 * g.gd.off + (p - 3) * n : Pc + (p - 5) * n);
        R *dst = Pt + kCols * g.gd.off + p * n;
        for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
            const int r = idx / TW, c = idx - r * TW;
            if (r < g.h && c < g.w) buf[r][c] = src[(size_t)(g.j0 + r) * g.gd.nx + g.i0 + c];
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
            const int c = idx / TH, r = idx - c * TH;
            if (r < g.h && c < g.w) dst[(size_t)(g.i0 + c) * g.gd.ny + g.j0 + r] = buf[r][c];
        }
        __syncthreads();
    }
}

// The FP32 staging straight from FP64 parameters (the mixed path's FP32
// phase): each plane of a tile is read once in FP64, rounded to FP32, written
// row-major (the FP32 copies the row sweeps read, as a cast would make them)
// and transposed (the column sweeps' copy).
template <int TH>
__global__ __launch_bounds__(256) void k_stage_from64(LaunchArgs a, const double *__restrict__ M,
                                                      const double *__restrict__ om, float *__restrict__ M32,
                                                      float *__restrict__ om32, float *__restrict__ Pt)
{
    constexpr int kCols = Staged<float>::cols;
    __shared__ float buf[TH][TW + 1];
    const TileGeo g = tile_geo<TH>(a, blockIdx.x);
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    for (int p = 0; p < kCols; ++p) {
        const double *src = p < 3 ? M + 3 * g.gd.off + p * n : om + 2 * g.gd.off + (p - 3) * n;
        float *row = p < 3 ? M32 + 3 * g.gd.off + p * n : om32 + 2 * g.gd.off + (p - 3) * n;
        float *dst = Pt + kCols * g.gd.off + p * n;
        for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
            const int r = idx / TW, c = idx - r * TW;
            if (r < g.h && c < g.w) {
                const size_t ad = (size_t)(g.j0 + r) * g.gd.nx + g.i0 + c;
                const float v = (float)src[ad];
                row[ad] = v;
                buf[r][c] = v;
            }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
            const int c = idx / TH, r = idx - c * TH;
            if (r < g.h && c < g.w) dst[(size_t)(g.i0 + c) * g.gd.ny + g.j0 + r] = buf[r][c];
        }
        __syncthreads();
    }
}

// One workgroup per tile, or (a grid of fewer workgroups) each workgroup
// taking tiles blockIdx.x, blockIdx.x + gridDim.x, ...: a narrow grid leaves
// most CUs to work running beside it on another stream.
template <typename R, int TH>
__global__ __launch_bounds__(256) void k_stage(LaunchArgs a, const R *__restrict__ M, const R *__restrict__ om,
                                               R *__restrict__ Pt)
{
    for (int t = blockIdx.x; t < a.n_tiles; t += gridDim.x) stage_tile<R, TH>(a, t, M, om, Pt);
}

// ---------------------------------------------------------------------------
// Initialisation: T, codes (source marks), levels, first active tiles.
// ---------------------------------------------------------------------------
// With act non-null it also resets the round state, one writer per element:
// the tile flags of both buffers and the per-round counts (every tile flagged
// for round 0 when warm), and the counter block.
template <typename R>
__global__ void k_init(int64_t n, const R *T_init, R *T, uint8_t *__restrict__ code, int32_t *__restrict__ level,
                       int32_t *__restrict__ act, int32_t *__restrict__ act_count, unsigned long long *__restrict__ ctr,
                       int n_tiles, int warm)
{ // T_init may be T itself (in-place warm start): each element is read before it is written
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = tid; c < n; c += stride) {
        T[c] = T_init ? T_init[c] : inf_v<R>();
        code[c] = kUnreached;
        if (level) level[c] = -1;
    }
    if (act) {
        for (int64_t i = tid; i < 2 * (int64_t)n_tiles; i += stride) act[i] = (warm && i < n_tiles) ? 1 : 0;
        for (int64_t i = tid; i < kMaxRounds + 2; i += stride) act_count[i] = (warm && i == 0) ? n_tiles : 0;
        for (int64_t i = tid; i < kCtrCount; i += stride) ctr[i] = 0;
    }
}

// One workgroup per grid. Out-of-range indices are counted in
// ctr[kCtrBadSource] and otherwise ignored.
template <typename R, int TH>
__global__ void k_sources(LaunchArgs a, const int32_t *__restrict__ src_idx, const R *__restrict__ src_t,
                          R *__restrict__ T, uint8_t *__restrict__ code, int32_t *__restrict__ level,
                          int32_t *__restrict__ act, int32_t *__restrict__ act_count,
                          unsigned long long *__restrict__ ctr)
{
    const GridDesc gd = a.grids[blockIdx.x];
    for (int s = threadIdx.x; s < gd.n_src; s += blockDim.x) {
        const int32_t c = src_idx[gd.src_base + s];
        if (c < 0 || (int64_t)c >= (int64_t)gd.nx * gd.ny) {
            atomicAdd(&ctr[kCtrBadSource], 1ull);
            continue;
        }
        T[gd.off + c] = src_t ? src_t[gd.src_base + s] : R(0);
        code[gd.off + c] = kSource;
        if (level) level[gd.off + c] = 0;
        const int i = c % gd.nx, j = c / gd.nx;
        const int t = gd.tile_base + (j / TH) * gd.ntx + i / TW;
        if (atomicExch(&act[t], 1) == 0) atomicAdd(&act_count[0], 1);
    }
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        p[c] = v;
}

__global__ void k_fill_u64(unsigned long long *__restrict__ p, int64_t n)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        p[c] = 0ull;
}

// Element-wise precision change (round to nearest; infinities kept).
template <typename S, typename D>
__global__ void k_cast(int64_t n, const S *__restrict__ src, D *__restrict__ dst)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        dst[c] = (D)src[c];
}

__global__ void k_all_active(int32_t *__restrict__ act, int n_tiles, int32_t *__restrict__ act_count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tiles) act[t] = 1;
    if (t == 0) act_count[0] = n_tiles;
}

// ---------------------------------------------------------------------------
// Tile helpers.
// ---------------------------------------------------------------------------
// Bits of the neighbour tiles that see node (ci, cj) of a w x h tile in their
// halo: 0 W, 1 E, 2 S (j-1), 3 N (j+1), 4 SW, 5 SE, 6 NW, 7 NE.
__device__ __forceinline__ int halo_bits(int ci, int cj, int w, int h)
{
    const bool W = ci == 0, E = ci == w - 1, S = cj == 0, N = cj == h - 1;
    return (W ? 1 : 0) | (E ? 2 : 0) | (S ? 4 : 0) | (N ? 8 : 0) | ((S && W) ? 16 : 0) | ((S && E) ? 32 : 0) |
           ((N && W) ? 64 : 0) | ((N && E) ? 128 : 0);
}

__device__ __forceinline__ void flag_tile(int32_t *act_out, int32_t *count_next, int u)
{
    if (atomicExch(&act_out[u], 1) == 0) atomicAdd(count_next, 1);
}

__device__ __forceinline__ void flag_neighbours(int bits, const TileGeo &g, int32_t *act_out, int32_t *count_next)
{
    const int DX[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
    const int DY[8] = {0, 0, -1, 1, -1, -1, 1, 1};
    for (int b = 0; b < 8; ++b) {
        if (!(bits & (1 << b))) continue;
        const int ux = g.tx + DX[b], uy = g.ty + DY[b];
        if (ux < 0 || ux >= g.gd.ntx || uy < 0 || uy >= g.gd.nty) continue;
        flag_tile(act_out, count_next, g.gd.tile_base + uy * g.gd.ntx + ux);
    }
}

__device__ __forceinline__ int wave_or(int v)
{
    for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off);
    return v;
}

// Step boundary inside a one-wave workgroup. The LDS serves one wave's
// requests in issue order, so a line written in one step is seen by the reads
// of the next; only compiler motion of LDS accesses across the boundary must
// be prevented. Unlike a workgroup barrier this does not wait for the
// in-flight global loads (the next line's parameters).
__device__ __forceinline__ void wave_step_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// One sweep of one direction over the tile held in LDS.
// ---------------------------------------------------------------------------
// Mb: three metric planes, Ob: two drift planes, both of n nodes each, laid out
// column-major (transposed copy) for column sweeps and row-major otherwise.
// LEV: carry the active update's code and dependency level along with T.
template <typename R, int TH, int DIR, bool FULL, bool LEV>
__device__ __forceinline__ bool sweep_dir(const TileGeo &g, const R *__restrict__ Mb, const R *__restrict__ Ob,
                                          const R *__restrict__ Cb, R *sT, int32_t *sL, uint8_t *sC, R tol, R h,
                                          R inv_h)
{
    constexpr int LP = TW + 3;
    constexpr bool COL = (DIR & 1) == 0; // a column (fixed x) per step
    const int lane = threadIdx.x % TW;
    const int len = COL ? g.w : g.h;
    const int span = COL ? g.h : g.w;
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const int lc = lane < span ? lane : span - 1; // clamped lane for loads
    // Parameters of the node this lane updates at step s (steps past the last
    // line are clamped to it). The planes' bases are uniform across the wave
    // and the node's index is a 32-bit offset (grids hold fewer than 2^32
    // nodes), so each load takes a scalar base and one vector offset.
    const R *__restrict__ P0 = Mb, *__restrict__ P1 = Mb + n, *__restrict__ P2 = Mb + 2 * n;
    const R *__restrict__ P3 = Ob, *__restrict__ P4 = Ob + n;
    const uint32_t stride = COL ? (uint32_t)g.gd.ny : (uint32_t)g.gd.nx;
    const uint32_t base = COL ? (uint32_t)g.i0 * stride + (uint32_t)(g.j0 + lc) : (uint32_t)g.j0 * stride + (uint32_t)(g.i0 + lc);
    auto load = [&](int s, R *p) {
        s = s < len ? s : len - 1;
        const int pos = DIR < 2 ? s : len - 1 - s;
        const uint32_t ad = base + (uint32_t)pos * stride;
        p[0] = P0[ad]; p[1] = P1[ad]; p[2] = P2[ad]; p[3] = P3[ad]; p[4] = P4[ad];
        if (Staged<R>::roots) {
#pragma unroll
            for (int q = 0; q < kRoots; ++q) p[5 + q] = Cb[(size_t)q * n + ad];
        }
    };
    bool changed = false;
    auto step = [&](int s, const R *q) {
        const int pos = DIR < 2 ? s : len - 1 - s;
        const int ci = COL ? pos : lane;
        const int cj = COL ? lane : pos;
        const int cc = cj * kBytePitch + ci;
        if (lane < span && sC[cc] != kSource) {
            NodeConst<R> k;
            if (Staged<R>::roots) node_const_pre<R>(q[0], q[1], q[2], q[3], q[4], q + 5, h, inv_h, k);
            else node_const<R>(q[0], q[1], q[2], q[3], q[4], h, inv_h, k);
            R Tn[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) Tn[d] = sT[(cj + 1 + nb_dy(d)) * LP + (ci + 1 + nb_dx(d))];
            int code;
            R v = local_update_dir<R, DIR, FULL>(k, Tn, code);
            const int slot = (cj + 1) * LP + ci + 1;
            const R old = sT[slot];
            int newcode = code;
            if (!FULL && !(v < old)) { // keep the old value and its code
                v = old;
                newcode = sC[cc];
            }
            if (LEV) {
                // dependency level of the current active update
                int lv = -1;
                if (newcode < 16) {
                    const int kp = newcode < 8 ? newcode : newcode - 8;
                    lv = sL[(cj + 1 + nb_dy(kp)) * LP + ci + 1 + nb_dx(kp)];
                    if (newcode < 8) {
                        const int kq = (newcode + 1) & 7;
                        lv = max(lv, sL[(cj + 1 + nb_dy(kq)) * LP + ci + 1 + nb_dx(kq)]);
                    }
                    lv = lv + 1;
                }
                sL[slot] = lv;
                sC[cc] = (uint8_t)newcode;
            }
            // only T decides convergence; levels ride along and are made
            // consistent with the final active updates afterwards
            changed |= counts_as_change<R>(old, v, tol);
            if (FULL) {
                if (v != old) sT[slot] = v; // skipping equal stores changes nothing in turn, loses less at once
            } else if (v < old) { // FAST: LDS atomic minimum (ds_min), safe under concurrent directions
                __hip_atomic_fetch_min(&sT[slot], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        wave_step_sync();
    };
    // Double-buffered parameters: the next line's five values load while a
    // line is updated. Two steps per iteration alternate the buffers, and each
    // buffer is refilled only after its last use, so no register copy (and no
    // wait for the loads in flight) sits between steps.
    R X[Staged<R>::cols], Y[Staged<R>::cols];
    load(0, X);
    for (int s = 0; s < len; s += 2) {
        load(s + 1, Y);
        step(s, X);
        if (s + 1 >= len) break; // uniform over the wave
        load(s + 2, X);
        step(s + 1, Y);
    }
    return changed;
}

// ---------------------------------------------------------------------------
// One visit of a tile: load T, levels and codes with a one-node halo, run
// four-sweep cycles until a full cycle changes nothing (or the cycle budget
// runs out), write back. Returns the halo bits of the neighbours that must see
// the new boundary values (OR over the wave) and whether the tile settled.
// ---------------------------------------------------------------------------
struct Visit {
    int bits;
    bool settled;
    int sweeps;
};

template <typename R, int TH, bool FULL, bool LEV>
__device__ __forceinline__ Visit visit_tile(const LaunchArgs &a, int t, const R *__restrict__ M,
                                            const R *__restrict__ om, const R *__restrict__ Ptall, R *Tall,
                                            uint8_t *codeall, int32_t *levall, R tol, int max_cycles, R *sT,
                                            int32_t *sL, uint8_t *sC)
{
    constexpr int LP = TW + 3; // odd pitch: conflict-free column access
    const int lane = threadIdx.x;
    const TileGeo g = tile_geo<TH>(a, t);
    R *T = Tall + g.gd.off;
    uint8_t *code = codeall + g.gd.off;
    int32_t *level = LEV ? levall + g.gd.off : nullptr;
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const R *Mg = M + 3 * g.gd.off, *Og = om + 2 * g.gd.off; // row-major planes
    const R *Pt = staged_cols(a, Ptall, g.gd), *Pto = Pt + 3 * n, *Ptr = Pt + 5 * n; // column-major copy
    const R *Pc = staged_roots_rows(a, Ptall, g.gd);
    const R h = R(g.gd.h), inv_h = R(1) / R(g.gd.h);

    load_tile_halo<R, TH, LP>(T, sT, g.gd.nx, g.gd.ny, g.i0, g.j0, inf_v<R>());
    if (LEV) load_tile_halo<int32_t, TH, LP>(level, sL, g.gd.nx, g.gd.ny, g.i0, g.j0, -1);
    load_block<uint8_t, TH, kBytePitch, 0>(code, sC, g.gd.nx, g.gd.ny, g.i0, g.j0, kSource);
    __syncthreads();

    int quiet = 0, sweeps = 0;
    const int max_sweeps = 4 * max_cycles;
    while (quiet < 4 && sweeps < max_sweeps) {
        bool ch;
        switch (sweeps & 3) {
        case 0: ch = sweep_dir<R, TH, 0, FULL, LEV>(g, Pt, Pto, Ptr, sT, sL, sC, tol, h, inv_h); break;
        case 1: ch = sweep_dir<R, TH, 1, FULL, LEV>(g, Mg, Og, Pc, sT, sL, sC, tol, h, inv_h); break;
        case 2: ch = sweep_dir<R, TH, 2, FULL, LEV>(g, Pt, Pto, Ptr, sT, sL, sC, tol, h, inv_h); break;
        default: ch = sweep_dir<R, TH, 3, FULL, LEV>(g, Mg, Og, Pc, sT, sL, sC, tol, h, inv_h); break;
        }
        ++sweeps;
        quiet = __ballot(ch) ? 0 : quiet + 1;
    }

    // write back (old values re-read in batches, see load_block), note the
    // neighbours whose halo moved
    int bits = 0;
    const int c = lane;
#pragma unroll 1
    for (int r0 = 0; r0 < TH; r0 += kLoadBatch) {
        R ov[kLoadBatch];
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const int r = r0 + k;
            const int rc = r < g.h ? r : g.h - 1, cc = c < g.w ? c : g.w - 1; // in-tile, no branch
            ov[k] = T[(size_t)(g.j0 + rc) * g.gd.nx + g.i0 + cc];
        }
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const int r = r0 + k;
            if (r >= g.h || c >= g.w) continue;
            const size_t gc = (size_t)(g.j0 + r) * g.gd.nx + (g.i0 + c);
            const int sl = (r + 1) * LP + c + 1;
            const R nv = sT[sl];
            if (nv != ov[k]) T[gc] = nv;
            if (LEV) {
                level[gc] = sL[sl];
                code[gc] = sC[r * kBytePitch + c];
            }
            if (counts_as_change<R>(ov[k], nv, tol)) bits |= halo_bits(c, r, g.w, g.h);
        }
    }
    Visit v;
    v.bits = wave_or(bits);
    v.settled = quiet >= 4;
    v.sweeps = sweeps * g.w * g.h;
    return v;
}

// ---------------------------------------------------------------------------
// Round scheduler: one launch per round over the flagged tiles.
// ---------------------------------------------------------------------------
template <typename R, int TH, bool FULL, bool LEV>
__global__ __launch_bounds__(TW) void k_sweep_round(LaunchArgs a, const R *__restrict__ M, const R *__restrict__ om,
                                                    const R *__restrict__ Ptall, R *__restrict__ Tall,
                                                    uint8_t *__restrict__ codeall, int32_t *__restrict__ levall,
                                                    int32_t *__restrict__ act_in, int32_t *__restrict__ act_out,
                                                    int32_t *__restrict__ count_next,
                                                    unsigned long long *__restrict__ ctr, R tol, int max_cycles)
{
    constexpr int LP = TW + 3;
    const int t = blockIdx.x;
    if (act_in[t] == 0) return;
    if (threadIdx.x == 0) act_in[t] = 0;
    __shared__ R sT[(TH + 2) * LP];
    __shared__ int32_t sL[LEV ? (TH + 2) * LP : 1];
    __shared__ uint8_t sC[TH * kBytePitch];
    const Visit v =
        visit_tile<R, TH, FULL, LEV>(a, t, M, om, Ptall, Tall, codeall, levall, tol, max_cycles, sT, sL, sC);
    if (threadIdx.x == 0) {
        const TileGeo g = tile_geo<TH>(a, t);
        flag_neighbours(v.bits, g, act_out, count_next);
        if (!v.settled) flag_tile(act_out, count_next, t); // cycle budget ran out before the tile settled
        atomicAdd(&ctr[kCtrCellUpdates], (unsigned long long)v.sweeps);
    }
}

// ---------------------------------------------------------------------------
// Concurrent-direction visits: four waves sweep the four directions of the
// same LDS tile at once, so the chain of dependent line steps per cycle is one
// direction's instead of four. FAST (cold start): T only decreases and the
// update is monotone in the donor values; improvements are stored with an LDS
// atomic minimum, so concurrent stores never raise a value. FULL: every store
// is a recomputation of the node from its neighbours' current values; a store
// computed from values another wave has since replaced is itself a change
// beyond tol or is corrected by the change that replaced them, so the cycle
// repeats. Either way a cycle ends quiet only when no wave changed anything
// beyond tol, which means every node of the tile holds its update (to tol)
// from the final values, as after a quiet cycle of the one-wave visit.
// ---------------------------------------------------------------------------
template <typename R, int TH, bool FULL>
__device__ __forceinline__ Visit visit_tile_cd(const LaunchArgs &a, int t, const R *__restrict__ M,
                                               const R *__restrict__ om, const R *__restrict__ Ptall, R *Tall,
                                               R tol, int max_cycles, R *sT, uint8_t *sC, int *sBits)
{
    constexpr int LP = TW + 3;
    // the wave index is uniform across each wave: taken from the first lane, the
    // direction switch below is a scalar branch and its plane pointers stay scalar
    const int lane = threadIdx.x % TW, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / TW);
    const TileGeo g = tile_geo<TH>(a, t);
    R *T = Tall + g.gd.off;
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const R *Mg = M + 3 * g.gd.off, *Og = om + 2 * g.gd.off;
    const R *Pt = staged_cols(a, Ptall, g.gd), *Pto = Pt + 3 * n, *Ptr = Pt + 5 * n;
    const R *Pc = staged_roots_rows(a, Ptall, g.gd);
    const R h = R(g.gd.h), inv_h = R(1) / R(g.gd.h);

    load_tile_halo<R, TH, LP>(T, sT, g.gd.nx, g.gd.ny, g.i0, g.j0, inf_v<R>());
    if (threadIdx.x == 0) *sBits = 0;
    __syncthreads();

    int cycles = 0;
    bool quiet = false;
    while (!quiet && cycles < max_cycles) {
        bool ch;
        switch (wave) { // uniform per wave
        case 0: ch = sweep_dir<R, TH, 0, FULL, false>(g, Pt, Pto, Ptr, sT, nullptr, sC, tol, h, inv_h); break;
        case 1: ch = sweep_dir<R, TH, 1, FULL, false>(g, Mg, Og, Pc, sT, nullptr, sC, tol, h, inv_h); break;
        case 2: ch = sweep_dir<R, TH, 2, FULL, false>(g, Pt, Pto, Ptr, sT, nullptr, sC, tol, h, inv_h); break;
        default: ch = sweep_dir<R, TH, 3, FULL, false>(g, Mg, Og, Pc, sT, nullptr, sC, tol, h, inv_h); break;
        }
        ++cycles;
        quiet = !__syncthreads_or(ch ? 1 : 0);
    }

    // write back: wave w takes row batches w, w + 4, ...
    int bits = 0;
    const int c = lane;
#pragma unroll 1
    for (int r0 = wave * kLoadBatch; r0 < TH; r0 += 4 * kLoadBatch) {
        R ov[kLoadBatch];
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const int r = r0 + k;
            const int rc = r < g.h ? r : g.h - 1, cc = c < g.w ? c : g.w - 1;
            ov[k] = T[(size_t)(g.j0 + rc) * g.gd.nx + g.i0 + cc];
        }
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const int r = r0 + k;
            if (r >= g.h || c >= g.w) continue;
            const R nv = sT[(r + 1) * LP + c + 1];
            if (nv != ov[k]) T[(size_t)(g.j0 + r) * g.gd.nx + (g.i0 + c)] = nv;
            if (counts_as_change<R>(ov[k], nv, tol)) bits |= halo_bits(c, r, g.w, g.h);
        }
    }
    bits = wave_or(bits);
    if (lane == 0 && bits) atomicOr(sBits, bits);
    __syncthreads();
    Visit v;
    v.bits = *sBits;
    v.settled = quiet;
    v.sweeps = 4 * cycles * g.w * g.h;
    return v;
}

template <typename R, int TH, bool FULL>
__global__ __launch_bounds__(4 * TW) void k_sweep_round_cd(LaunchArgs a, const R *__restrict__ M,
                                                         const R *__restrict__ om, const R *__restrict__ Ptall,
                                                         R *__restrict__ Tall, const uint8_t *__restrict__ codeall,
                                                         int32_t *__restrict__ act_in, int32_t *__restrict__ act_out,
                                                         int32_t *__restrict__ count_next,
                                                         unsigned long long *__restrict__ ctr, R tol, int max_cycles)
{
    constexpr int LP = TW + 3;
    const int t = blockIdx.x;
    if (act_in[t] == 0) return;
    __shared__ R sT[(TH + 2) * LP];
    __shared__ uint8_t sC[TH * kBytePitch];
    __shared__ int sBits;
    {
        const TileGeo g = tile_geo<TH>(a, t);
        load_block<uint8_t, TH, kBytePitch, 0>(codeall + g.gd.off, sC, g.gd.nx, g.gd.ny, g.i0, g.j0, kSource);
    }
    const Visit v = visit_tile_cd<R, TH, FULL>(a, t, M, om, Ptall, Tall, tol, max_cycles, sT, sC, &sBits);
    if (threadIdx.x == 0) {
        act_in[t] = 0;
        const TileGeo g = tile_geo<TH>(a, t);
        flag_neighbours(v.bits, g, act_out, count_next);
        if (!v.settled) flag_tile(act_out, count_next, t);
        atomicAdd(&ctr[kCtrCellUpdates], (unsigned long long)v.sweeps);
    }
}

// ---------------------------------------------------------------------------
// Work-queue scheduler: one launch; each wave takes flagged tiles from a
// device queue, visits them, and puts the neighbours whose halo changed back
// on the queue. A tile is never visited by two waves at once: its state goes
// idle -> queued -> running -> idle, and a tile flagged while running is
// marked and queued again when its visit ends. Information then crosses tile
// boundaries as soon as the neighbour is visited, with no round barrier.
//
// Termination: every wait polls a bounded number of times. A wave leaves when
// no tile is queued or running (nothing can be flagged any more), when the
// visit budget is spent, or when a wait exceeds its limit (reported as an
// error); the visits themselves are bounded by the cycle budget, so every
// wave reaches the exit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void q_flag_neighbours(const WorkQueue &q, int bits, const TileGeo &g)
{
    const int DX[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
    const int DY[8] = {0, 0, -1, 1, -1, -1, 1, 1};
    for (int b = 0; b < 8; ++b) {
        if (!(bits & (1 << b))) continue;
        const int ux = g.tx + DX[b], uy = g.ty + DY[b];
        if (ux < 0 || ux >= g.gd.ntx || uy < 0 || uy >= g.gd.nty) continue;
        q_flag(q, g.gd.tile_base + uy * g.gd.ntx + ux);
    }
}

template <typename R, int TH, bool LEV>
__global__ __launch_bounds__(TW) void k_sweep_queue(LaunchArgs a, const R *__restrict__ M, const R *__restrict__ om,
                                                    const R *__restrict__ Ptall, R *Tall, uint8_t *codeall,
                                                    int32_t *levall, WorkQueue q, unsigned long long *__restrict__ ctr,
                                                    R tol, int max_cycles)
{
    constexpr int LP = TW + 3;
    __shared__ R sT[(TH + 2) * LP];
    __shared__ int32_t sL[LEV ? (TH + 2) * LP : 1];
    __shared__ uint8_t sC[TH * kBytePitch];
    unsigned long long updates = 0;
    for (;;) {
        int t = threadIdx.x == 0 ? q_take(q) : 0;
        t = __shfl(t, 0);
        if (t < 0) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); // the neighbours' written-back values
        const Visit v =
            visit_tile<R, TH, true, LEV>(a, t, M, om, Ptall, Tall, codeall, levall, tol, max_cycles, sT, sL, sC);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); // this tile's values before its flags
        updates += (unsigned long long)v.sweeps;
        if (threadIdx.x == 0) {
            q_flag_neighbours(q, v.bits, tile_geo<TH>(a, t));
            q_done(q, t, v.settled);
        }
        __syncthreads(); // LDS reuse by the next visit
    }
    if (threadIdx.x == 0 && updates) atomicAdd(&ctr[kCtrCellUpdates], updates);
}

// Queue set-up from the flags of round 0 (sources, or every tile for a warm
// start): flagged tiles are queued and their flags cleared.
__global__ void k_queue_seed(int n_tiles, int32_t *__restrict__ act, WorkQueue q)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles || act[t] == 0) return;
    act[t] = 0;
    q.state[t] = kTileQueued;
    atomicAdd(&q.ctl[kQPending], 1u);
    const uint32_t pos = atomicAdd(&q.ctl[kQTail], 1u);
    q.ring[pos & q.mask] = (uint32_t)(t + 1);
}

// Control words: cleared, with the visit budget set.
__global__ void k_queue_reset(WorkQueue q, uint32_t budget)
{
    const int i = threadIdx.x;
    if (i < kQCtlWords) q.ctl[i] = i == kQBudget ? budget : 0u;
}

// ---------------------------------------------------------------------------
// Split update: SUB lanes per node, a workgroup of SUB waves per tile. Lane
// `sub` of a node evaluates the two-point stencils NS sub .. NS sub + NS - 1
// (NS = 8 / SUB) and the one-point candidates of their first donors, from
// per-node constants it forms itself; the group's minimum is taken with
// cross-lane moves inside the group, ordered by value and then by code, which
// is the canonical order of the one-lane update. A wave then issues a fraction
// of the instructions per line step, which shortens the chain of dependent
// steps that bounds a tile visit.
// ---------------------------------------------------------------------------
namespace split {

// neighbour offsets, two bits per k holding offset + 1
constexpr uint32_t kDx = (0u << 0) | (0u << 2) | (0u << 4) | (1u << 6) | (2u << 8) | (2u << 10) | (2u << 12) | (1u << 14);
constexpr uint32_t kDy = (2u << 0) | (1u << 2) | (0u << 4) | (0u << 6) | (0u << 8) | (1u << 10) | (2u << 12) | (2u << 14);
__device__ __forceinline__ int odx(int k) { return (int)((kDx >> (2 * k)) & 3u) - 1; }
__device__ __forceinline__ int ody(int k) { return (int)((kDy >> (2 * k)) & 3u) - 1; }

// data-parallel-primitive moves inside a group of four lanes
constexpr int kXor1 = 0xB1; // lanes (1, 0, 3, 2)
constexpr int kXor2 = 0x4E; // lanes (2, 3, 0, 1)
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_r(float v)
{
    return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_r(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)dpp_i<CTRL>((int)(unsigned)(b & 0xffffffffull));
    const unsigned hi = (unsigned)dpp_i<CTRL>((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <int CTRL, typename R>
__device__ __forceinline__ void lex_min(R &v, int &c)
{
    const R ov = dpp_r<CTRL>(v);
    const int oc = dpp_i<CTRL>(c);
    const bool take = (ov < v) | ((ov == v) & (oc < c)); // selects, no branch
    v = take ? ov : v;
    c = take ? oc : c;
}
template <int SUB, typename R>
__device__ __forceinline__ void group_min(R &v, int &c)
{
    if (SUB >= 2) lex_min<kXor1>(v, c);
    if (SUB >= 4) lex_min<kXor2>(v, c);
}

// The node's full local update from the NS + 1 donors this lane reads
// (donor k_q = (NS sub + q) mod 8 has time Tq[q]); code as in local_update.
template <typename R, int SUB>
__device__ __forceinline__ R update(int sub, R m11, R m12, R m22, R bx, R by, R h, R inv_h, const R *Tq, int &code)
{
    constexpr int NS = 8 / SUB;
    const R inf = inf_v<R>();
    R mx[NS + 1], my[NS + 1], e[NS + 1], bm[NS + 1];
#pragma unroll
    for (int q = 0; q <= NS; ++q) {
        const int k = (NS * sub + q) & 7;
        mx[q] = R(-odx(k)); // receiver minus donor
        my[q] = R(-ody(k));
        e[q] = mx[q] * (m11 * mx[q] + m12 * my[q]) + my[q] * (m12 * mx[q] + m22 * my[q]);
        bm[q] = mx[q] * bx + my[q] * by;
    }
    // one-point candidates of donors 0..NS-1, then the group's best
    R b1 = inf;
    int c1 = kUnreached;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const R t = Tq[q] + h * (bm[q] + dsqrt(e[q]));
        const bool take = t < b1;
        b1 = take ? t : b1;
        c1 = take ? 8 + ((NS * sub + q) & 7) : c1;
    }
    group_min<SUB>(b1, c1);
    // two-point stencils whose donors are both below the best one-point value
    const R det = m11 * m22 - m12 * m12;
    R b2 = inf;
    int c2 = kUnreached;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const R Tp = Tq[q], Tr = Tq[q + 1];
        if (Tp < b1 && Tr < b1) {
            const R Ep = e[q], Er = e[q + 1];
            const R Epr = mx[q] * (m11 * mx[q + 1] + m12 * my[q + 1]) + my[q] * (m12 * mx[q + 1] + m22 * my[q + 1]);
            const R dx = mx[q + 1] - mx[q], dy = my[q + 1] - my[q];
            const R a = dx * dx * m11 + R(2) * dx * dy * m12 + dy * dy * m22; // m11 or m22 exactly
            const R delta = (Tr - Tp) * inv_h + (bm[q + 1] - bm[q]);
            const bool base_r = delta < R(0);
            const R s1 = base_r ? -delta : R(0);
            const R s2 = base_r ? R(0) : delta;
            const R S0 = base_r ? Tr + h * bm[q + 1] : Tp + h * bm[q];
            const R beta = s1 * (Er - Epr) + s2 * (Ep - Epr);
            const R c = Er * s1 * s1 + Ep * s2 * s2 - det;
            const R D = beta * beta - a * c;
            if (D >= R(0)) {
                const R tau = (beta + dsqrt(D)) * drcp(a);
                const R mu1 = Er * (tau - s1) - Epr * (tau - s2);
                const R mu2 = Ep * (tau - s2) - Epr * (tau - s1);
                const R t = S0 + h * tau;
                if (mu1 >= R(0) && mu2 >= R(0) && t > Tp && t > Tr && t < b2) {
                    b2 = t;
                    c2 = (NS * sub + q) & 7;
                }
            }
        }
    }
    group_min<SUB>(b2, c2);
    if (b2 <= b1) {
        code = c2;
        return b2;
    }
    code = c1;
    return b1;
}

} // namespace split

template <typename R, int TH, int DIR, int SUB>
__device__ __forceinline__ bool sweep_dir_split(const TileGeo &g, const R *__restrict__ Mb, const R *__restrict__ Ob,
                                                R *sT, const uint8_t *sC, R tol, R h, R inv_h)
{
    constexpr int LP = TW + 3;
    constexpr int NS = 8 / SUB;
    constexpr bool COL = (DIR & 1) == 0;
    const int node = threadIdx.x / SUB, sub = threadIdx.x % SUB;
    const int len = COL ? g.w : g.h;
    const int span = COL ? g.h : g.w;
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const int lc = node < span ? node : span - 1;
    auto addr = [&](int s) -> size_t {
        const int pos = DIR < 2 ? s : len - 1 - s;
        return COL ? (size_t)(g.i0 + pos) * g.gd.ny + (g.j0 + lc) : (size_t)(g.j0 + pos) * g.gd.nx + (g.i0 + lc);
    };
    // the parameters of the next PD lines are in flight while a line is
    // updated (register ring, static indices through the unrolled inner loop;
    // addresses past the last line are clamped to it)
    constexpr int PD = 1;
    R P[PD][5];
#pragma unroll
    for (int d = 0; d < PD; ++d) {
        const size_t a0 = addr(d < len ? d : len - 1);
        P[d][0] = Mb[a0]; P[d][1] = Mb[n + a0]; P[d][2] = Mb[2 * n + a0]; P[d][3] = Ob[a0]; P[d][4] = Ob[n + a0];
    }
    bool changed = false;
    for (int s0 = 0; s0 < len; s0 += PD) {
#pragma unroll
        for (int d = 0; d < PD; ++d) {
            const int s = s0 + d;
            if (s >= len) break; // uniform over the workgroup
            const R q0 = P[d][0], q1 = P[d][1], q2 = P[d][2], q3 = P[d][3], q4 = P[d][4];
            {
                const size_t an = addr(s + PD < len ? s + PD : len - 1);
                P[d][0] = Mb[an]; P[d][1] = Mb[n + an]; P[d][2] = Mb[2 * n + an]; P[d][3] = Ob[an];
                P[d][4] = Ob[n + an];
            }
            const int pos = DIR < 2 ? s : len - 1 - s;
            const int ci = COL ? pos : node;
            const int cj = COL ? node : pos;
            // the SUB lanes of a node share this test, so groups stay whole
            if (node < span && sC[cj * kBytePitch + ci] != kSource) {
                R Tq[NS + 1];
#pragma unroll
                for (int q = 0; q <= NS; ++q) {
                    const int k = (NS * sub + q) & 7;
                    Tq[q] = sT[(cj + 1 + split::ody(k)) * LP + (ci + 1 + split::odx(k))];
                }
                int code;
                const R v = split::update<R, SUB>(sub, q0, q1, q2, q3, q4, h, inv_h, Tq, code);
                if (sub == 0) {
                    const int slot = (cj + 1) * LP + ci + 1;
                    changed |= counts_as_change<R>(sT[slot], v, tol);
                    sT[slot] = v;
                }
            }
            __syncthreads();
        }
    }
    return changed;
}

// One visit of a tile by SUB waves (full update, no levels carried).
template <typename R, int TH, int SUB>
__device__ __forceinline__ Visit visit_tile_split(const LaunchArgs &a, int t, const R *__restrict__ M,
                                                  const R *__restrict__ om, const R *__restrict__ Ptall, R *Tall,
                                                  const uint8_t *codeall, R tol, int max_cycles, R *sT, uint8_t *sC,
                                                  int *sbits)
{
    constexpr int LP = TW + 3;
    const TileGeo g = tile_geo<TH>(a, t);
    R *T = Tall + g.gd.off;
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const R *Mg = M + 3 * g.gd.off, *Og = om + 2 * g.gd.off;
    const R *Pt = staged_cols(a, Ptall, g.gd), *Pto = Pt + 3 * n;
    const R h = R(g.gd.h), inv_h = R(1) / R(g.gd.h);

    if (threadIdx.x == 0) *sbits = 0;
    load_tile_halo<R, TH, LP>(T, sT, g.gd.nx, g.gd.ny, g.i0, g.j0, inf_v<R>());
    load_block<uint8_t, TH, kBytePitch, 0>(codeall + g.gd.off, sC, g.gd.nx, g.gd.ny, g.i0, g.j0, kSource);
    __syncthreads();

    int quiet = 0, sweeps = 0;
    const int max_sweeps = 4 * max_cycles;
    while (quiet < 4 && sweeps < max_sweeps) {
        bool ch;
        switch (sweeps & 3) {
        case 0: ch = sweep_dir_split<R, TH, 0, SUB>(g, Pt, Pto, sT, sC, tol, h, inv_h); break;
        case 1: ch = sweep_dir_split<R, TH, 1, SUB>(g, Mg, Og, sT, sC, tol, h, inv_h); break;
        case 2: ch = sweep_dir_split<R, TH, 2, SUB>(g, Pt, Pto, sT, sC, tol, h, inv_h); break;
        default: ch = sweep_dir_split<R, TH, 3, SUB>(g, Mg, Og, sT, sC, tol, h, inv_h); break;
        }
        ++sweeps;
        quiet = __syncthreads_or(ch) ? 0 : quiet + 1;
    }

    // write back: each wave takes rows in turn (old values re-read in batches)
    int bits = 0;
    const int c = threadIdx.x % TW;
    const int wave = threadIdx.x / TW;
#pragma unroll 1
    for (int r0 = wave * kLoadBatch; r0 < TH; r0 += SUB * kLoadBatch) {
        R ov[kLoadBatch];
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const int r = r0 + k;
            const int rc = r < g.h ? r : g.h - 1, cc = c < g.w ? c : g.w - 1;
            ov[k] = T[(size_t)(g.j0 + rc) * g.gd.nx + g.i0 + cc];
        }
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const int r = r0 + k;
            if (r >= g.h || c >= g.w) continue;
            const R nv = sT[(r + 1) * LP + c + 1];
            if (nv != ov[k]) T[(size_t)(g.j0 + r) * g.gd.nx + g.i0 + c] = nv;
            if (counts_as_change<R>(ov[k], nv, tol)) bits |= halo_bits(c, r, g.w, g.h);
        }
    }
    bits = wave_or(bits);
    if (threadIdx.x % TW == 0 && bits) atomicOr(sbits, bits);
    __syncthreads();
    Visit v;
    v.bits = *sbits;
    v.settled = quiet >= 4;
    v.sweeps = sweeps * g.w * g.h;
    return v;
}

template <typename R, int TH, int SUB>
__global__ __launch_bounds__(TW * SUB) void k_sweep_round_split(LaunchArgs a, const R *__restrict__ M,
                                                                const R *__restrict__ om,
                                                                const R *__restrict__ Ptall, R *__restrict__ Tall,
                                                                const uint8_t *__restrict__ codeall,
                                                                int32_t *__restrict__ act_in,
                                                                int32_t *__restrict__ act_out,
                                                                int32_t *__restrict__ count_next,
                                                                unsigned long long *__restrict__ ctr, R tol,
                                                                int max_cycles)
{
    constexpr int LP = TW + 3;
    const int t = blockIdx.x;
    if (act_in[t] == 0) return; // uniform over the workgroup
    __shared__ R sT[(TH + 2) * LP];
    __shared__ uint8_t sC[TH * kBytePitch];
    __shared__ int sbits;
    __syncthreads(); // every wave has read act_in[t] before it is cleared
    if (threadIdx.x == 0) act_in[t] = 0;
    const Visit v =
        visit_tile_split<R, TH, SUB>(a, t, M, om, Ptall, Tall, codeall, tol, max_cycles, sT, sC, &sbits);
    if (threadIdx.x == 0) {
        const TileGeo g = tile_geo<TH>(a, t);
        flag_neighbours(v.bits, g, act_out, count_next);
        if (!v.settled) flag_tile(act_out, count_next, t);
        atomicAdd(&ctr[kCtrCellUpdates], (unsigned long long)v.sweeps);
    }
}

// ---------------------------------------------------------------------------
// Active stencils from the final field (the stencil identification of
// Alg. backward, moved into the forward pass). Donors must lie strictly below
// the node's own time, which keeps the donor graph acyclic.
// ---------------------------------------------------------------------------
template <typename R, int TH>
__global__ __launch_bounds__(256) void k_parents(LaunchArgs a, const R *__restrict__ M, const R *__restrict__ om,
                                                 const R *__restrict__ Tall, uint8_t *__restrict__ parall)
{
    const TileGeo g = tile_geo<TH>(a, blockIdx.x);
    const int64_t n = (int64_t)g.gd.nx * g.gd.ny;
    const R *T = Tall + g.gd.off;
    uint8_t *parent = parall + g.gd.off;
    const R *Mg = M + 3 * g.gd.off;
    const R *og = om + 2 * g.gd.off;
    const R h = R(g.gd.h), inv_h = R(1) / R(g.gd.h);
    for (int idx = threadIdx.x; idx < TH * TW; idx += blockDim.x) {
        const int r = idx / TW, cl = idx - r * TW;
        if (r >= g.h || cl >= g.w) continue;
        const int i = g.i0 + cl, j = g.j0 + r;
        const size_t c = (size_t)j * g.gd.nx + i;
        if (parent[c] == kSource) continue;
        const R Tc = T[c];
        if (!(Tc < inf_v<R>())) {
            parent[c] = kUnreached;
            continue;
        }
        R Tn[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int x = i + nb_dx(q), y = j + nb_dy(q);
            Tn[q] = (x >= 0 && x < g.gd.nx && y >= 0 && y < g.gd.ny) ? T[(size_t)y * g.gd.nx + x] : inf_v<R>();
        }
        NodeConst<R> k;
        node_const<R>(Mg[c], Mg[n + c], Mg[2 * n + c], og[c], og[n + c], h, inv_h, k);
        int code;
        R w1;
        local_update<R>(k, Tn, Tc, code, w1);
        parent[c] = (uint8_t)code;
    }
}

// ---------------------------------------------------------------------------
// Dependency levels: level = 1 + max level of the donors, overwritten until
// stable (the donor graph is acyclic, so this converges from any start; after
// the sweep, which already carried the levels, one quiet round is typical).
// ---------------------------------------------------------------------------
template <int TH>
__global__ __launch_bounds__(TW) void k_level_round(LaunchArgs a, const uint8_t *__restrict__ parall,
                                                    int32_t *__restrict__ levall, int32_t *__restrict__ act_in,
                                                    int32_t *__restrict__ act_out, int32_t *__restrict__ count_next,
                                                    int max_cycles)
{
    constexpr int LP = TW + 3;
    const int t = blockIdx.x;
    if (act_in[t] == 0) return;
    const int lane = threadIdx.x;
    if (lane == 0) act_in[t] = 0;
    const TileGeo g = tile_geo<TH>(a, t);
    const uint8_t *parent = parall + g.gd.off;
    int32_t *level = levall + g.gd.off;

    __shared__ int32_t sL[(TH + 2) * LP];
    __shared__ uint8_t sP[TH * kBytePitch];
    load_tile_halo<int32_t, TH, LP>(level, sL, g.gd.nx, g.gd.ny, g.i0, g.j0, -1);
    load_block<uint8_t, TH, kBytePitch, 0>(parent, sP, g.gd.nx, g.gd.ny, g.i0, g.j0, kUnreached);
    __syncthreads();

    int quiet = 0, sweeps = 0;
    const int max_sweeps = 4 * max_cycles;
    while (quiet < 4 && sweeps < max_sweeps) {
        const int dir = sweeps & 3;
        const bool col = (dir & 1) == 0;
        const int len = col ? g.w : g.h;
        const int span = col ? g.h : g.w;
        bool changed = false;
        for (int s = 0; s < len; ++s) {
            const int pos = dir < 2 ? s : len - 1 - s;
            const int ci = col ? pos : lane;
            const int cj = col ? lane : pos;
            const int code = lane < span ? sP[cj * kBytePitch + ci] : kUnreached;
            int32_t *slot = &sL[(cj + 1) * LP + ci + 1];
            int nv = code == kSource ? 0 : -1;
            if (code < 16) {
                const int kp = code < 8 ? code : code - 8;
                int lv = sL[(cj + 1 + nb_dy(kp)) * LP + ci + 1 + nb_dx(kp)];
                if (code < 8) {
                    const int kq = (code + 1) & 7;
                    lv = max(lv, sL[(cj + 1 + nb_dy(kq)) * LP + ci + 1 + nb_dx(kq)]);
                }
                nv = lv + 1;
            }
            if (lane < span) {
                changed |= nv != *slot;
                *slot = nv;
            }
            wave_step_sync();
        }
        ++sweeps;
        quiet = __ballot(changed) ? 0 : quiet + 1;
    }

    int bits = 0;
    for (int idx = lane; idx < TH * TW; idx += TW) {
        const int r = idx / TW, c = idx - r * TW;
        if (c >= g.w || r >= g.h) continue;
        const size_t gc = (size_t)(g.j0 + r) * g.gd.nx + (g.i0 + c);
        const int32_t nv = sL[(r + 1) * LP + c + 1];
        if (nv != level[gc]) {
            level[gc] = nv;
            bits |= halo_bits(c, r, g.w, g.h);
        }
    }
    bits = wave_or(bits);
    if (lane == 0) {
        flag_neighbours(bits, g, act_out, count_next);
        if (quiet < 4) flag_tile(act_out, count_next, t);
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

void launch_write_single_desc(const GridDesc &d, GridDesc *dst, int32_t *tile_grid, int n_tiles, hipStream_t st)
{
    hipLaunchKernelGGL(k_write_single_desc, dim3((n_tiles + 255) / 256), dim3(256), 0, st, d, dst, tile_grid,
                       n_tiles);
}

template <typename R>
void launch_stage(const LaunchArgs &a, const void *M, const void *om, void *Pt, hipStream_t st, int max_blocks)
{
    const int blocks = max_blocks > 0 ? std::min(max_blocks, a.n_tiles) : a.n_tiles;
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_stage<R, TH>), dim3(blocks), dim3(256), 0, st, a, (const R *)M,
                                             (const R *)om, (R *)Pt));
}

void launch_stage_from64(const LaunchArgs &a, const double *M, const double *om, float *M32, float *om32, void *Pt,
                         hipStream_t st)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_stage_from64<TH>), dim3(a.n_tiles), dim3(256), 0, st, a, M, om, M32,
                                             om32, (float *)Pt));
}

template <typename R>
void launch_init(const LaunchArgs &a, const void *T_init, void *T, uint8_t *code, int32_t *level,
                 const int32_t *src_idx, const void *src_t, int32_t *act, int32_t *act_count,
                 unsigned long long *ctr, bool warm, hipStream_t st, bool reset)
{
    const int64_t work = std::max<int64_t>(a.n_nodes, reset ? kMaxRounds + 2 : 0);
    hipLaunchKernelGGL(k_init<R>, dim3(blocks_for(work, 256)), dim3(256), 0, st, a.n_nodes, (const R *)T_init,
                       (R *)T, code, level, reset ? act : nullptr, act_count, ctr, a.n_tiles, warm ? 1 : 0);
    if (warm && !reset) launch_all_active(a, act, act_count, st);
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_sources<R, TH>), dim3(a.n_grids), dim3(64), 0, st, a, src_idx,
                                             (const R *)src_t, (R *)T, code, level, act, act_count, ctr));
}

void launch_all_active(const LaunchArgs &a, int32_t *act, int32_t *act_count, hipStream_t st)
{
    hipLaunchKernelGGL(k_all_active, dim3((a.n_tiles + 255) / 256), dim3(256), 0, st, act, a.n_tiles, act_count);
}

template <typename R>
void launch_sweep_round(const LaunchArgs &a, int mode, const void *M, const void *om, const void *Pt, void *T,
                        uint8_t *code, int32_t *level, int32_t *act_in, int32_t *act_out, int32_t *count_next,
                        unsigned long long *ctr, double tol, int max_cycles, int node_lanes, hipStream_t st)
{
    if (mode == kModeFull && level == nullptr && node_lanes == kFullWavesCD) {
        EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_sweep_round_cd<R, TH, true>), dim3(a.n_tiles), dim3(4 * TW), 0, st,
                                                 a, (const R *)M, (const R *)om, (const R *)Pt, (R *)T, code, act_in,
                                                 act_out, count_next, ctr, R(tol), max_cycles));
        return;
    }
    if (mode == kModeFull && level == nullptr && node_lanes > 1) {
#define EIK_SWEEP_SPLIT(SUB)                                                                                     \
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_sweep_round_split<R, TH, SUB>), dim3(a.n_tiles), dim3(TW * SUB), 0,  \
                                             st, a, (const R *)M, (const R *)om, (const R *)Pt, (R *)T, code,     \
                                             act_in, act_out, count_next, ctr, R(tol), max_cycles))
        if (node_lanes >= 4) EIK_SWEEP_SPLIT(4);
        else EIK_SWEEP_SPLIT(2);
#undef EIK_SWEEP_SPLIT
        return;
    }
#define EIK_SWEEP_ROUND(FULL, LEV)                                                                               \
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_sweep_round<R, TH, FULL, LEV>), dim3(a.n_tiles), dim3(TW), 0, st, a, \
                                             (const R *)M, (const R *)om, (const R *)Pt, (R *)T, code, level,     \
                                             act_in, act_out, count_next, ctr, R(tol), max_cycles))
    const bool lev = level != nullptr;
    if (mode == kModeFastCD && !lev) {
        EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_sweep_round_cd<R, TH, false>), dim3(a.n_tiles), dim3(4 * TW), 0, st, a,
                                                 (const R *)M, (const R *)om, (const R *)Pt, (R *)T, code, act_in,
                                                 act_out, count_next, ctr, R(tol), max_cycles));
        return;
    }
    if (mode == kModeFull) {
        if (lev) EIK_SWEEP_ROUND(true, true);
        else EIK_SWEEP_ROUND(true, false);
    } else {
        if (lev) EIK_SWEEP_ROUND(false, true);
        else EIK_SWEEP_ROUND(false, false);
    }
#undef EIK_SWEEP_ROUND
}

void launch_queue_setup(const LaunchArgs &a, int32_t *act, const WorkQueue &q, uint32_t budget, hipStream_t st)
{
    launch_fill_i32((int32_t *)q.ring, (int64_t)q.mask + 1, 0, st);
    launch_fill_i32((int32_t *)q.state, a.n_tiles, kTileIdle, st);
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, q, budget);
    hipLaunchKernelGGL(k_queue_seed, dim3((a.n_tiles + 255) / 256), dim3(256), 0, st, a.n_tiles, act, q);
}

template <typename R>
void launch_sweep_queue(const LaunchArgs &a, int n_waves, const void *M, const void *om, const void *Pt, void *T,
                        uint8_t *code, int32_t *level, const WorkQueue &q, unsigned long long *ctr, double tol,
                        int max_cycles, hipStream_t st)
{
    if (level)
        EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_sweep_queue<R, TH, true>), dim3(n_waves), dim3(TW), 0, st, a,
                                                 (const R *)M, (const R *)om, (const R *)Pt, (R *)T, code, level, q,
                                                 ctr, R(tol), max_cycles));
    else
        EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_sweep_queue<R, TH, false>), dim3(n_waves), dim3(TW), 0, st, a,
                                                 (const R *)M, (const R *)om, (const R *)Pt, (R *)T, code, level, q,
                                                 ctr, R(tol), max_cycles));
}

int sweep_queue_waves(int th, int dtype, bool lev)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e;
#define EIK_OCC(R, TH, LEV) hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_queue<R, TH, LEV>, TW, 0)
    if (dtype == 1)
        e = th == 64 ? (lev ? EIK_OCC(double, 64, true) : EIK_OCC(double, 64, false))
                     : (lev ? EIK_OCC(double, 32, true) : EIK_OCC(double, 32, false));
    else
        e = th == 64 ? (lev ? EIK_OCC(float, 64, true) : EIK_OCC(float, 64, false))
                     : (lev ? EIK_OCC(float, 32, true) : EIK_OCC(float, 32, false));
#undef EIK_OCC
    if (e != hipSuccess) return 0;
    return std::max(1, per_cu) * cus;
}

template <typename R>
void launch_parents(const LaunchArgs &a, const void *M, const void *om, const void *T, uint8_t *parent,
                    hipStream_t st)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL((k_parents<R, TH>), dim3(a.n_tiles), dim3(256), 0, st, a,
                                             (const R *)M, (const R *)om, (const R *)T, parent));
}

void launch_level_round(const LaunchArgs &a, const uint8_t *parent, int32_t *level, int32_t *act_in,
                        int32_t *act_out, int32_t *count_next, int max_cycles, hipStream_t st)
{
    EIK_TH_DISPATCH(a.th, hipLaunchKernelGGL(k_level_round<TH>, dim3(a.n_tiles), dim3(TW), 0, st, a, parent, level,
                                             act_in, act_out, count_next, max_cycles));
}

void launch_max_level(int64_t n, const int32_t *level, unsigned long long *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(k_max_level, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, level, ctr);
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
}

void launch_fill_u64(unsigned long long *p, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
}

void launch_cast_f64_f32(int64_t n, const double *src, float *dst, hipStream_t st)
{
    hipLaunchKernelGGL((k_cast<double, float>), dim3(blocks_for(n, 256)), dim3(256), 0, st, n, src, dst);
}

void launch_cast_f32_f64(int64_t n, const float *src, double *dst, hipStream_t st)
{
    hipLaunchKernelGGL((k_cast<float, double>), dim3(blocks_for(n, 256)), dim3(256), 0, st, n, src, dst);
}

template <typename R>
void launch_check_feasible(int64_t n, const void *M, const void *om, unsigned long long *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_feasible<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, (const R *)M,
                       (const R *)om, ctr);
}

#define EIK_INST(R)                                                                                             \
    template void launch_stage<R>(const LaunchArgs &, const void *, const void *, void *, hipStream_t, int);    \
    template void launch_init<R>(const LaunchArgs &, const void *, void *, uint8_t *, int32_t *,                 \
                                 const int32_t *, const void *, int32_t *, int32_t *, unsigned long long *,      \
                                 bool, hipStream_t, bool);                                                       \
    template void launch_sweep_round<R>(const LaunchArgs &, int, const void *, const void *, const void *,       \
                                        void *, uint8_t *, int32_t *, int32_t *, int32_t *, int32_t *,           \
                                        unsigned long long *, double, int, int, hipStream_t);                    \
    template void launch_sweep_queue<R>(const LaunchArgs &, int, const void *, const void *, const void *,       \
                                        void *, uint8_t *, int32_t *, const WorkQueue &, unsigned long long *,   \
                                        double, int, hipStream_t);                                               \
    template void launch_parents<R>(const LaunchArgs &, const void *, const void *, const void *, uint8_t *,     \
                                    hipStream_t);                                                                \
    template void launch_check_feasible<R>(int64_t, const void *, const void *, unsigned long long *, hipStream_t);
EIK_INST(float)
EIK_INST(double)
#undef EIK_INST

} // namespace eik

namespace eik {

__global__ void k_note_pending(const int32_t *__restrict__ count, unsigned long long *__restrict__ slot)
{
    if (threadIdx.x == 0) *slot = (unsigned long long)(count[0] > 0 ? count[0] : 0);
}

__global__ void k_copy_u64(const unsigned long long *__restrict__ src, unsigned long long *__restrict__ dst)
{
    if (threadIdx.x == 0) *dst = *src;
}

void launch_copy_u64(const unsigned long long *src, unsigned long long *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(64), 0, st, src, dst);
}

void launch_note_pending(const int32_t *count, unsigned long long *slot, hipStream_t st)
{
    hipLaunchKernelGGL(k_note_pending, dim3(1), dim3(64), 0, st, count, slot);
}

// tiles still queued or running after the queue kernel (plus 2^32 on a failed wait)
__global__ void k_note_queue(WorkQueue q, unsigned long long *__restrict__ slot)
{
    if (threadIdx.x == 0)
        *slot = (unsigned long long)q.ctl[kQPending] + (q.ctl[kQFail] ? (1ull << 32) : 0ull) +
                (q.ctl[kQStop] && !q.ctl[kQPending] ? 1ull : 0ull);
}

void launch_note_queue(const WorkQueue &q, unsigned long long *slot, hipStream_t st)
{
    hipLaunchKernelGGL(k_note_queue, dim3(1), dim3(64), 0, st, q, slot);
}

} // namespace eik
