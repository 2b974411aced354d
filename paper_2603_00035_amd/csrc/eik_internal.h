// eik_internal.h -- host/device interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace eik {

constexpr int TW = 64; // tile width = wave size

// One grid of a launch. Arrays of a launch are packed grid after grid: the
// node arrays of grid g start at node offset `off`, its metric planes at
// 3*off, its drift planes at 2*off, its transposed parameters at 5*off.
struct GridDesc {
    int64_t off;      // first node of this grid in the packed node arrays
    double h;
    int32_t nx, ny;
    int32_t ntx, nty; // tiles along x and y
    int32_t tile_base;// first tile of this grid in the launch's tile list
    int32_t n_src, src_base;
    int32_t pad;
};

struct LaunchArgs {
    const GridDesc *grids;
    const int32_t *tile_grid; // tile -> grid
    int32_t n_grids, n_tiles, th;
    int64_t n_nodes;          // all grids
};

// slots of the 64-bit counter block in the workspace
enum {
    kCtrCellUpdates = 0,
    kCtrBadSource = 1,
    kCtrMaxLevel = 2,
    kCtrInfeasible = 3,
    kCtrSweepPending = 4, // tiles still flagged after the last sweep round
    kCtrLevelPending = 5, // ... after the last level round
    kCtrAdjPending = 6,   // ... after the last adjoint round
    kCtrFastUpdates = 7,  // kCtrCellUpdates when the restricted-candidate cold start ended
    kCtrCount = 16
};

// Device work queue of the queue scheduler (workspace memory, reset by
// kernels before each use).
enum { kTileIdle = 0, kTileQueued = 1, kTileRunning = 2, kTileAgain = 3 };
enum { kQHead = 0, kQTail = 1, kQPending = 2, kQStop = 3, kQFail = 4, kQBudget = 5, kQVisits = 6, kQCtlWords = 8 };
struct WorkQueue {
    uint32_t *ring;      // mask + 1 slots: tile + 1, or 0 when empty
    uint32_t *state;     // per tile: kTile*
    uint32_t *ctl;       // kQCtlWords control words
    uint32_t mask;       // slots - 1 (a power of two minus one)
    uint32_t spin_limit; // polls before a wait is declared stuck
};

constexpr int kMaxRounds = 1 << 16;

enum SweepMode { kModeFast = 0, kModeFull = 1, kModeFastCD = 2 };
// node_lanes argument of launch_sweep_round that selects the concurrent-direction FULL visits
constexpr int kFullWavesCD = -4;

// copies the flagged-tile count of the last round into a counter slot
void launch_note_pending(const int32_t *count, unsigned long long *slot, hipStream_t st);
void launch_note_queue(const WorkQueue &q, unsigned long long *slot, hipStream_t st);

// forward
template <typename R>
void launch_stage(const LaunchArgs &a, const void *M, const void *om, void *Pt, hipStream_t st, int max_blocks = 0);
// FP32 staging from FP64 parameters, writing the FP32 copies M32, om32 as well
void launch_stage_from64(const LaunchArgs &a, const double *M, const double *om, float *M32, float *om32, void *Pt,
                         hipStream_t st);
// reset: the initialisation also clears the round state (act, act_count,
// the counter block) and, when warm, flags every tile for round 0
template <typename R>
void launch_init(const LaunchArgs &a, const void *T_init, void *T, uint8_t *code, int32_t *level,
                 const int32_t *src_idx, const void *src_t, int32_t *act, int32_t *act_count,
                 unsigned long long *ctr, bool warm, hipStream_t st, bool reset = false);
template <typename R>
void launch_sweep_round(const LaunchArgs &a, int mode, const void *M, const void *om, const void *Pt, void *T,
                        uint8_t *code, int32_t *level, int32_t *act_in, int32_t *act_out, int32_t *count_next,
                        unsigned long long *ctr, double tol, int max_cycles, int node_lanes, hipStream_t st);
template <typename R>
void launch_parents(const LaunchArgs &a, const void *M, const void *om, const void *T, uint8_t *parent,
                    hipStream_t st);
template <typename R>
void launch_check_feasible(int64_t n, const void *M, const void *om, unsigned long long *ctr, hipStream_t st);
void launch_all_active(const LaunchArgs &a, int32_t *act, int32_t *act_count, hipStream_t st);
// queue scheduler: reset + seed from the round-0 flags, then one persistent launch
void launch_queue_setup(const LaunchArgs &a, int32_t *act, const WorkQueue &q, uint32_t budget, hipStream_t st);
template <typename R>
void launch_sweep_queue(const LaunchArgs &a, int n_waves, const void *M, const void *om, const void *Pt, void *T,
                        uint8_t *code, int32_t *level, const WorkQueue &q, unsigned long long *ctr, double tol,
                        int max_cycles, hipStream_t st);
// waves of the queue kernel that fit on the device at once
int sweep_queue_waves(int th, int dtype, bool lev);
void launch_level_round(const LaunchArgs &a, const uint8_t *parent, int32_t *level, int32_t *act_in,
                        int32_t *act_out, int32_t *count_next, int max_cycles, hipStream_t st);
void launch_max_level(int64_t n, const int32_t *level, unsigned long long *ctr, hipStream_t st);
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
void launch_fill_u64(unsigned long long *p, int64_t n, hipStream_t st);
void launch_copy_u64(const unsigned long long *src, unsigned long long *dst, hipStream_t st);

// Inverse-problem passes (eik_inverse.hip); reductions use kInvBlocks
// double partials in the caller's scratch.
constexpr int kInvBlocks = 1024;
template <typename R>
void launch_tv(int nx, int ny, int C, const void *F, const double *weights, double scale, void *grad,
               double *value, double *partial, hipStream_t st);
template <typename R>
void launch_obs_loss(int64_t n, const void *T, const void *To, const uint8_t *mask, void *g, double *value,
                     double *partial, hipStream_t st);
template <typename R>
void launch_sum_sq(int64_t n, const void *x, double *acc, double *partial, hipStream_t st);
template <typename R>
void launch_tie_isotropic(int64_t n, void *M, hipStream_t st);
// Log-Euclidean TV of the metric: work holds log G and its gradient (6 n reals)
template <typename R>
void launch_tv_log_euclid(int nx, int ny, const void *M, double scale, void *grad, double *value, void *work,
                          double *partial, hipStream_t st);
template <typename R>
void launch_param_step(int64_t n, int method, void *p, const void *g, void *m, void *v, double lr, double b1,
                       double b2, double eps, int t, double max_norm, const double *grad_sq, hipStream_t st);
// Covariate encoder passes (eik_encoder.hip); the combination's backward over B
// scenes uses B * kEncPlanes * kInvBlocks double partials in the caller's
// scratch.
constexpr int kEncPlanes = 5;
void launch_enc_dense(int B, int Cin, int Cout, const float *x, const float *W, const float *b, int relu, float *y,
                      hipStream_t st);
void launch_enc_dense_backward(int B, int Cin, int Cout, const float *x, const float *W, const float *y, int relu,
                               const float *dy, float *dx, float *dW, float *db, hipStream_t st);
template <typename R>
void launch_enc_combine(int B, int64_t n, double alpha, const float *base, const float *local, void *M, void *om,
                        hipStream_t st);
template <typename R>
void launch_enc_combine_backward(int B, int64_t n, double alpha, const void *dM, const void *dom, float *dlocal,
                                 float *dbase, double *partial, hipStream_t st);
constexpr int kEncMaxScenes = 4096;
void launch_cast_f64_f32(int64_t n, const double *src, float *dst, hipStream_t st);
void launch_cast_f32_f64(int64_t n, const float *src, double *dst, hipStream_t st);
void launch_write_single_desc(const GridDesc &d, GridDesc *dst, int32_t *tile_grid, int n_tiles, hipStream_t st);

// backward
// FP32 inputs of a mixed-precision relaxation, written by the adjoint
// preparation when w1 is non-null: the donor weights and dL/dT (from g_src, in
// the state's type) rounded to FP32, and lambda cleared
struct Prep32 {
    float *w1 = nullptr;
    const void *g_src = nullptr;
    float *g = nullptr, *lam = nullptr;
};
template <typename R>
void launch_adj_prep(const LaunchArgs &a, const void *M, const void *om, const void *T, const uint8_t *parent,
                     void *w1, void *lam, hipStream_t st, const Prep32 &p32 = Prep32());
// every tile flagged for round 0, the other round state cleared, one launch
void launch_round_reset(const LaunchArgs &a, int32_t *act, int32_t *act_count, hipStream_t st);
// Per-node inputs of the adjoint relaxation sweeps, per grid at its node
// offset: receiver descriptors and dL/dT, row-major (D, g) and transposed
// (DT, gT, [nx][ny] per grid) for the column sweeps.
struct AdjNodes {
    const uint16_t *D, *DT;
    const void *g, *gT;
};
template <typename R>
void launch_adj_stage(const LaunchArgs &a, const uint8_t *parent, const void *g, uint16_t *D, uint16_t *DT, void *gT,
                      hipStream_t st);
template <typename R>
void launch_adj_round(const LaunchArgs &a, const AdjNodes &nd, const void *w1, void *lam, int max_cycles, int waves,
                      int32_t *act_in, int32_t *act_out, int32_t *count_next, hipStream_t st);
template <typename R>
void launch_adj_queue(const LaunchArgs &a, int n_waves, const AdjNodes &nd, const void *w1, void *lam,
                      int max_cycles, const WorkQueue &q, hipStream_t st);
int adj_queue_waves(int th, int dtype);
template <typename R>
void launch_adj_params(const LaunchArgs &a, const void *M, const uint8_t *parent, const void *w1, const void *lam,
                       void *dM, void *dom, hipStream_t st);
template <typename R>
void launch_dsrc(const LaunchArgs &a, const int32_t *src_idx, const void *lam, void *dsrc, hipStream_t st);
// level-scheduled adjoint (eik_levels.hip): counting sort of each grid's
// reached nodes by level into order (bins[off + l] ends as the end of bin l,
// gmax[g] is the largest level of grid g), then the gather by decreasing level
void launch_level_buckets(const LaunchArgs &a, const int32_t *level, int32_t *gmax, int32_t *bins, int32_t *order,
                          hipStream_t st);
template <typename R>
void launch_level_gather(const LaunchArgs &a, const int32_t *gmax, const int32_t *bins, const int32_t *order,
                         const uint16_t *D, const void *g, const void *w1, void *lam, hipStream_t st);

// projection
template <typename R>
void launch_project(int64_t n, const void *M, const void *om, void *Mo, void *oo, double eig_min, double eig_max,
                    double eucl_clip, double rho_max, hipStream_t st);
template <typename R>
void launch_project_backward(int64_t n, const void *M, const void *om, const void *gMo, const void *goo, void *gM,
                             void *go, double eig_min, double eig_max, double eucl_clip, double rho_max,
                             hipStream_t st);

// soft-min mode (eik_soft.hip): one workgroup per grid of a batch; lines
// (rows and columns) of at most kSoftMaxLine nodes. SoftBatch points into the
// caller's workspace: descs (kSoftDescBytes per grid, written with
// write_soft_desc), per-grid iteration state (scale: one real, done and cycle
// count), source marks, the bad-source count, the transposed parameters
// (Pt, 5 reals per node), and for the adjoint the incoming weights in both
// layouts (win, wint: 8 reals per node each), the parameter partials (dth, 5),
// the transposed dL/dT (gt) and lambda. Grids whose values fit kSoftLdsBudget
// bytes of LDS are swept there.
constexpr int kSoftMaxLine = 4096;
constexpr size_t kSoftDescBytes = 32;
constexpr size_t kSoftLdsBudget = 56 * 1024; // with the static arrays, within 64 KB per workgroup
struct SoftBatch {
    int32_t n_grids;
    int32_t max_line;           // longest row or column of the batch
    int32_t max_rows, max_cols; // largest ny and nx of the batch
    int64_t n_nodes, max_nodes;
    void *descs;
    void *scale;
    int32_t *done, *cycles, *bad;
    uint8_t *mark;
    void *Pt, *win, *wint, *dth, *gt, *lam;
};
void write_soft_desc(int64_t off, double h, int32_t nx, int32_t ny, int32_t n_src, int32_t src_base, void *dst);
// sources and marks (T may be NULL: marks only); with M non-NULL also the transposed parameters
template <typename R>
void launch_soft_init(const SoftBatch &b, const int32_t *src, const void *src_t, void *T, const void *M,
                      const void *om, hipStream_t st);
// one launch of up to ncyc cycles per grid
template <typename R>
void launch_soft_cycles(const SoftBatch &b, const void *M, const void *om, void *T, double tau, double tol, int ncyc,
                        hipStream_t st);
template <typename R>
void launch_soft_coef(const SoftBatch &b, const void *M, const void *om, const void *T, const void *gT, double tau,
                      hipStream_t st);
template <typename R>
void launch_soft_adj_cycles(const SoftBatch &b, const void *gT, const void *T, double tol, int ncyc, hipStream_t st);
template <typename R>
void launch_soft_params(const SoftBatch &b, const int32_t *src, void *dM, void *dom, void *dsrc, hipStream_t st);

static inline int blocks_for(int64_t n, int bs) { return (int)std::min<int64_t>((n + bs - 1) / bs, 8192); }

} // namespace eik
