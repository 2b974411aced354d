// eik_internal.h -- host/device interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace eik {

struct GridArgs {
    int32_t nx, ny;
    double h;
    int32_t n_src;
    int32_t th;  // tile height (tile width is the wave size, 64)
    int32_t ntx, nty, n_tiles;
};

// slots of the 64-bit counter block in the workspace
enum {
    kCtrCellUpdates = 0,
    kCtrBadSource = 1,
    kCtrMaxLevel = 2,
    kCtrInfeasible = 3,
    kCtrCount = 16
};

constexpr int kMaxRounds = 1 << 16;

template <typename R>
void launch_init(const GridArgs &g, const void *T_init, void *T, uint8_t *parent, int32_t *level,
                 const int32_t *src_idx, const void *src_t, int32_t *act, int32_t *act_count,
                 unsigned long long *ctr, bool warm, hipStream_t st);
template <typename R>
void launch_sweep_round(const GridArgs &g, const void *M, const void *om, void *T, const uint8_t *parent,
                        int32_t *act_in, int32_t *act_out, int32_t *count_next, unsigned long long *ctr, double tol,
                        int max_cycles, hipStream_t st);
template <typename R>
void launch_parents(const GridArgs &g, const void *M, const void *om, const void *T, uint8_t *parent,
                    int32_t *level, hipStream_t st);
template <typename R>
void launch_check_feasible(int64_t n, const void *M, const void *om, unsigned long long *ctr, hipStream_t st);
void launch_level_prep(const GridArgs &g, int32_t *act, int32_t *act_count, hipStream_t st);
void launch_level_round(const GridArgs &g, const uint8_t *parent, int32_t *level, int32_t *act_in,
                        int32_t *act_out, int32_t *count_next, int max_cycles, hipStream_t st);
void launch_max_level(int64_t n, const int32_t *level, unsigned long long *ctr, hipStream_t st);
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
void launch_fill_u64(unsigned long long *p, int64_t n, hipStream_t st);

template <typename R>
void launch_adj_prep(const GridArgs &g, const void *M, const void *om, const void *T, const uint8_t *parent,
                     const int32_t *level, void *w1, int32_t *counts, void *dM, void *dom, hipStream_t st);
void launch_scan_levels(int32_t *counts, int32_t *offsets, int32_t *cursor, const unsigned long long *ctr,
                        hipStream_t st);
void launch_scatter_levels(int64_t n, const int32_t *level, int32_t *cursor, int32_t *list, hipStream_t st);
template <typename R>
void launch_adj_levels(const GridArgs &g, int L_hi, int L_lo, bool single_wg, const unsigned long long *ctr,
                       const int32_t *offsets, const int32_t *list, const uint8_t *parent, const void *w1,
                       const void *dLdT, const void *M, void *lam, void *dM, void *dom, hipStream_t st);
template <typename R>
void launch_dsrc(const GridArgs &g, const int32_t *src_idx, const void *lam, void *dsrc, hipStream_t st);

template <typename R>
void launch_project(int64_t n, const void *M, const void *om, void *Mo, void *oo, double eig_min, double eig_max,
                    double eucl_clip, double rho_max, hipStream_t st);
template <typename R>
void launch_project_backward(int64_t n, const void *M, const void *om, const void *gMo, const void *goo, void *gM,
                             void *go, double eig_min, double eig_max, double eucl_clip, double rho_max,
                             hipStream_t st);

} // namespace eik
