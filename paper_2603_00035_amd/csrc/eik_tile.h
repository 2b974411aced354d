// eik_tile.h -- loads of a tile (plus a one-node halo) into LDS by one wave.
//
// Lane c of a wave owns column i0 + c. The loads of a batch of 16 rows are
// all issued before any of them is stored to LDS, so each lane keeps 16
// global loads in flight instead of waiting for one load per row.
#pragma once

#include "eik_internal.h"

namespace eik {

constexpr int kLoadBatch = 16;

// Row pitches of the per-node LDS arrays (no halo), padded so that the 64
// lanes of a column sweep, which step through one row each, fall in distinct
// banks: 68 bytes (17 dwords) for byte arrays, 66 halves (33 dwords) for
// 16-bit arrays, 65 elements for 32-bit ones (an odd dword stride each).
constexpr int kBytePitch = TW + 4;
constexpr int kHalfPitch = TW + 2;
constexpr int kWordPitch = TW + 1;

// dst[row * PITCH + OFF + lane] = src[(jstart + row) * nx + i0 + lane] for
// row in [0, ROWS); `outside` where that node is not in the nx x ny grid.
// The block may hold several waves (blockDim.x a multiple of 64); they take
// the batches of rows in turn.
template <typename V, int ROWS, int PITCH, int OFF>
__device__ __forceinline__ void load_block(const V *__restrict__ src, V *dst, int nx, int ny, int i0, int jstart,
                                           V outside)
{
    const int lane = threadIdx.x % TW;
    const int wave = threadIdx.x / TW, n_waves = blockDim.x / TW;
    const int gi = i0 + lane;
    const bool col_in = gi >= 0 && gi < nx;
    const int gic = gi < 0 ? 0 : (gi < nx ? gi : nx - 1);
#pragma unroll 1
    for (int r0 = wave * kLoadBatch; r0 < ROWS; r0 += n_waves * kLoadBatch) {
        V v[kLoadBatch];
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            // every load reads a node inside the grid (clamped index), so the
            // batch needs no branches; nodes outside take `outside`
            const int gj = jstart + r0 + k;
            const int gjc = gj < 0 ? 0 : (gj < ny ? gj : ny - 1);
            const V x = src[(size_t)gjc * nx + gic];
            v[k] = (r0 + k < ROWS && col_in && gj >= 0 && gj < ny) ? x : outside;
        }
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k)
            if (r0 + k < ROWS) dst[(r0 + k) * PITCH + OFF + lane] = v[k];
    }
}

// A tile of TH rows x TW columns at (i0, j0) with its one-node halo into an
// LDS array of (TH + 2) rows of pitch LP: dst[(r + 1) * LP + c + 1] holds node
// (i0 + c, j0 + r); halo nodes outside the grid read `outside`.
template <typename V, int TH, int LP>
__device__ __forceinline__ void load_tile_halo(const V *__restrict__ src, V *dst, int nx, int ny, int i0, int j0,
                                               V outside)
{
    load_block<V, TH + 2, LP, 1>(src, dst, nx, ny, i0, j0 - 1, outside);
    for (int r = threadIdx.x; r < TH + 2; r += blockDim.x) { // the two side columns
        const int gj = j0 - 1 + r;
        const bool row_in = gj >= 0 && gj < ny;
        V left = outside, right = outside;
        if (row_in && i0 - 1 >= 0) left = src[(size_t)gj * nx + i0 - 1];
        if (row_in && i0 + TW < nx) right = src[(size_t)gj * nx + i0 + TW];
        dst[r * LP] = left;
        dst[r * LP + TW + 1] = right;
    }
}

} // namespace eik
