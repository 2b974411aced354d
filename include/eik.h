/*
 * eik.h -- C ABI of the MI355X (gfx950) Randers-Finsler eikonal library.
 *
 * Method: "Differentiable Randers-Finsler Eikonal Solvers" (arXiv 2603.00035).
 *   forward   Sec. 3.2 and Alg. forward: fast-sweeping solve of
 *             (grad T - b)^T G^-1 (grad T - b) = 1 (Eq. randers_eikonal) with the
 *             two-point (Eq. two_point) and one-point (Eq. one_point) local
 *             updates on the eight triangular stencils;
 *   backward  Sec. 3.3 and Alg. backward: implicit differentiation of the
 *             converged fixed point (Eqs. implicit, param_grad, adjoint) by one
 *             reverse pass over the causal order of the nodes;
 *   project   App. learning details, "Feasibility Projections";
 *   batched   the same for many independent grids of different sizes in one
 *             launch sequence (the paper batches problem instances, Sec. 4.3).
 *
 * Layout (all arrays device memory, caller-allocated, row-major, x fastest):
 *   node (i, j), 0 <= i < nx, 0 <= j < ny, flat index j*nx + i, position (i h, j h);
 *   M      [3][ny][nx]  metric planes m11, m12, m22 (G = [[m11, m12], [m12, m22]]);
 *   omega  [2][ny][nx]  drift planes bx, by;
 *   T      [ny][nx]     arrival times; +inf where no source is reachable;
 *   parent [ny][nx]     uint8 active update of each node:
 *                       0..7   two-point stencil k (neighbours k and (k+1) mod 8),
 *                       8..15  one-point from neighbour k-8,
 *                       0xFE   source, 0xFF unreached;
 *                       neighbour k of (i,j) is (i + dx_k, j + dy_k) with
 *                       (dx,dy)_k = (-1,1) (-1,0) (-1,-1) (0,-1) (1,-1) (1,0) (1,1) (0,1)
 *                       (counter-clockwise from the upper-left neighbour);
 *   level  [ny][nx]     int32 dependency level: 0 at sources, 1 + the largest
 *                       level of the donors elsewhere, -1 where unreached
 *                       (optional output of the forward; the adjoint does not
 *                       need it).
 * Real arrays are float (EIK_F32) or double (EIK_F64) as the dtype argument says.
 * Batched calls pack the grids one after the other: the node arrays of grid g
 * start at node offset off_g = sum over earlier grids of nx*ny, its M planes at
 * 3 off_g, its omega planes at 2 off_g; src_idx / src_t / dL/dt_src hold the
 * sources of grid 0, then grid 1, ..., with indices local to their grid.
 *
 * Ownership: the caller owns every buffer, including the workspace (size from
 * eik_workspace_bytes / eik_batch_workspace_bytes). The library never
 * allocates device memory and keeps no state between calls except one
 * non-blocking stream of default priority per device, created on first use
 * by eik_forward_mixed and kept until the process ends. Work is enqueued on
 * the given HIP stream (eik_forward_mixed forks part of it onto that stream
 * and joins it back with events before it returns).
 *
 * Errors: every call returns an int status and never throws. Negative values
 * are errors (nothing useful was written); EIK_NOT_CONVERGED is a warning
 * (outputs are valid, the tolerance was not reached within the budget).
 * eik_last_error() returns a thread-local message for the last non-OK status.
 */
#ifndef EIK_H
#define EIK_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { EIK_F32 = 0, EIK_F64 = 1, EIK_MIXED = 2 /* batched mixed-precision workspace only */ } eik_dtype;

enum {
    EIK_OK = 0,
    EIK_NOT_CONVERGED = 1,
    EIK_EINVAL = -1,      /* bad argument (size, pointer, dtype, source index) */
    EIK_EINFEASIBLE = -2, /* metric not SPD or |omega|_{M^-1} >= 1 (when checked) */
    EIK_EDEVICE = -3,     /* a HIP runtime call failed, or an internal schedule did not settle */
    EIK_EWORKSPACE = -4   /* workspace missing or smaller than needed */
};

/* Flags for the forward calls. */
enum {
    EIK_CHECK_FEASIBLE = 1, /* verify m11 > 0, det M > 0, |omega|_{M^-1} < 1 first */
    EIK_TIME_KERNELS = 2,   /* time each sweep-kernel launch with HIP events (stats) */
    EIK_WARM_FALLBACK = 4   /* warm starts only, in calls that synchronise (single grid, or batched with
                               stats): after two full-update rounds from T_init, if more than a quarter of
                               the tiles are still changing by more than tol, T_init is dropped and the
                               solve restarts from the cold start (stats->fell_back = 1); the two rounds
                               are counted in the stats */
};

/* One grid. src_idx: device array of n_src distinct flat node indices.
 * src_t: device array of n_src source times in the run's dtype, or NULL for 0.
 * (Batched calls take the source arrays separately and ignore these two.) */
typedef struct eik_grid {
    int32_t nx, ny;
    double h;
    int32_t n_src;
    const int32_t *src_idx;
    const void *src_t;
} eik_grid;

/* Host-side report of a call (filled only when a non-NULL pointer is given;
 * asking for it synchronises the stream). */
typedef struct eik_stats {
    int32_t rounds;         /* tile-sweep rounds (forward) or adjoint rounds (backward) */
    int32_t converged;      /* 1 when no node changed by more than tol */
    int64_t cell_updates;   /* local-update evaluations (one per node per sweep) */
    int32_t n_levels;       /* largest level + 1 (0 when levels were not asked for) */
    int32_t status;         /* same as the return value */
    int32_t sweep_launches; /* launches of the tile-sweep kernel */
    int32_t aux_rounds;     /* level rounds (forward) / adjoint rounds (backward) */
    double sweep_ms;        /* duration of the sweep launches (EIK_TIME_KERNELS; each batch of rounds between
                               host checks is timed as a whole), else 0 */
    double fast_ms;         /* the part of sweep_ms spent in the cold start's restricted-candidate rounds */
    int64_t fast_cell_updates; /* the part of cell_updates made in those rounds */
    int32_t fast_launches;  /* the part of sweep_launches made in those rounds */
    int32_t fell_back;      /* 1 when EIK_WARM_FALLBACK dropped the warm start, else 0 */
} eik_stats;

/* Scheduling knobs; NULL or a field <= 0 keeps the library default. */
typedef struct eik_tuning {
    int32_t tile_height;      /* 32 or 64 (tiles are 64 nodes wide); default 64 */
    int32_t max_local_cycles; /* four-sweep cycles a tile may run per visit; default 1 */
    int32_t rounds_per_check; /* rounds enqueued between host convergence checks; default 8 */
    int32_t fast_cold_start;  /* cold start only: 1: restricted-candidate min sweeps before the full ones;
                                 2: the same with the four directions of each cycle swept at once by four
                                 waves (one workgroup of 256 lanes per tile); 0: full sweeps only;
                                 default 2 (with levels asked for, 2 runs as 1) */
    int32_t adjoint_rounds;   /* fixed adjoint round budget of unsynchronised batched calls; default 64 */
    int32_t level_rounds;     /* fixed level round budget of unsynchronised batched calls; default 8 */
    int32_t scheduler;        /* EIK_SCHED_ROUNDS: one launch per round of flagged tiles, host checks between
                                 batches of rounds; EIK_SCHED_QUEUE: one persistent launch whose waves take
                                 flagged tiles from a device work queue (max_rounds then bounds the tile visits
                                 to max_rounds x tiles); default EIK_SCHED_ROUNDS */
    int32_t node_lanes;       /* lanes that share one node's update in the round scheduler's sweeps when no
                                 levels are asked for: 1, 2 or 4 (a tile then runs on that many waves);
                                 default 4 */
    int32_t adjoint_cycles;   /* four-sweep cycles a tile may run per adjoint visit; default 1 */
    int32_t adjoint_waves;    /* waves per tile in the round scheduler's adjoint visits: 1 (the four
                                 directional sweeps of a cycle in turn) or 4 (one direction per wave, all at
                                 once); default 4 */
    int32_t full_waves;       /* waves per tile in the round scheduler's full-update visits when no levels are
                                 asked for: 1 (the four directions in turn, node_lanes lanes per node) or 4
                                 (one direction per wave, one lane per node, all at once); default 4 */
    int32_t adjoint_mode;     /* EIK_ADJ_RELAX: tiles relax the adjoint equations by directional sweeps
                                 (default); EIK_ADJ_LEVELS: the nodes are counting-sorted by dependency level
                                 and solved level by level from the largest (needs the forward's levels) */
    int32_t level_mode;       /* with levels asked for: EIK_LEVELS_CARRIED: the sweeps carry them (one wave per
                                 tile; default); EIK_LEVELS_AFTER: the sweeps run as without levels and level
                                 rounds compute them afterwards from the active stencils */
} eik_tuning;

enum { EIK_ADJ_RELAX = 1, EIK_ADJ_LEVELS = 2 };
enum { EIK_LEVELS_CARRIED = 1, EIK_LEVELS_AFTER = 2 };

enum { EIK_SCHED_ROUNDS = 1, EIK_SCHED_QUEUE = 2 };

/* Bytes of workspace eik_forward / eik_backward need for this grid and dtype
 * (0 for an invalid grid). */
size_t eik_workspace_bytes(const eik_grid *grid, int32_t dtype);

/* Forward solve (Sec. 3.2, Alg. forward).
 *   M, omega  inputs as laid out above;
 *   T_init    optional [ny][nx] initial field (warm start; may be T itself)
 *             or NULL for the cold start (+inf away from the sources); the
 *             update overwrites T rather than taking a minimum with the
 *             previous value;
 *   tol       a node counts as changed when |dT| > tol |T| (or it changes
 *             between finite and infinite); the solve ends when a full
 *             four-direction cycle leaves no node changed. tol = 0 asks for
 *             exact stationarity;
 *   max_rounds bound on tile-sweep rounds per phase (EIK_NOT_CONVERGED past it);
 *   T, parent outputs; level optional output (NULL: not computed, which
 *             saves the level rounds); ws/ws_bytes workspace; tuning and
 *             stats optional.
 * The call synchronises the stream between batches of rounds to test for
 * convergence. Out-of-range source indices are ignored on the device and
 * reported as EIK_EINVAL.
 * Errors: EIK_EINVAL, EIK_EWORKSPACE, EIK_EINFEASIBLE (with
 * EIK_CHECK_FEASIBLE), EIK_EDEVICE. */
int eik_forward(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, const void *T_init,
                double tol, int32_t max_rounds, int32_t flags, void *T, uint8_t *parent, int32_t *level,
                void *ws, size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats, hipStream_t stream);

/* eik_forward without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid it): the same solve, arguments and results as eik_forward, with the
 * workspace taken from a fixed array the library holds on each GPU for the
 * life of the process (eik_noalloc_max_workspace_bytes(), 64 MiB: grids whose
 * eik_workspace_bytes fit, about 1 850 000 nodes (1360 x 1360) in FP32 and
 * 407 000 (638 x 638) in FP64, 512 x 512 in either). Larger grids are rejected with EIK_EWORKSPACE before anything runs;
 * EIK_TIME_KERNELS is rejected with EIK_EINVAL. The call allocates nothing.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams or host threads) race, and must be serialised by the
 * caller. The first call on each GPU looks up the array's device address. */
size_t eik_noalloc_max_workspace_bytes(void);
int eik_forward_noalloc(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, const void *T_init,
                        double tol, int32_t max_rounds, int32_t flags, void *T, uint8_t *parent, int32_t *level,
                        const eik_tuning *tuning, eik_stats *stats, hipStream_t stream);

/* Mixed-precision forward: the solve of eik_forward on FP64 parameters in two
 * phases. FP32 sweeps from the cold start, on FP32-rounded copies of M, omega
 * and the source times: with the restricted-candidate cold start on
 * (tuning32->fast_cold_start, default) they run that update until no tile
 * changes a value by more than tol32 and stop there, the full update being
 * left to the FP64 phase; with it off they run the full update to tol32
 * (EIK_NOT_CONVERGED there is not an error). FP64 full-update sweeps then continue from that field, in
 * place in T, to tol, visiting every tile first.
 * The FP32 phase carries the front across the grid at FP32 cost; the FP64
 * phase removes the FP32 rounding that the arrival times accumulate along
 * their characteristics, to which the adjoint's local derivatives are
 * sensitive. M, omega, grid->src_t (or NULL), T are double; parent and level
 * as in eik_forward, both written by the FP64 phase. max_rounds bounds each
 * phase. EIK_CHECK_FEASIBLE tests the FP32 copies. tuning32 and tuning
 * (each optional) drive the two phases; stats is NULL or an array of two
 * (FP32 phase, FP64 phase). The workspace comes from
 * eik_mixed_workspace_bytes: the FP32 copies, the FP64 phase's workspace and
 * one of its own for the FP32 phase, so that the FP64 phase's inputs are
 * staged on the side stream while the FP32 sweeps run. The FP64 state it returns feeds eik_backward
 * with EIK_F64. Errors as eik_forward; the status is that of the FP64 phase
 * unless the FP32 phase failed. */
size_t eik_mixed_workspace_bytes(const eik_grid *grid);
int eik_forward_mixed(const eik_grid *grid, const double *M, const double *omega, double tol32, double tol,
                      int32_t max_rounds, int32_t flags, double *T, uint8_t *parent, int32_t *level, void *ws,
                      size_t ws_bytes, const eik_tuning *tuning32, const eik_tuning *tuning, eik_stats *stats,
                      hipStream_t stream);

/* Adjoint (Sec. 3.3, Alg. backward): given dL/dT and the saved state
 * (M, omega, T, parent) of eik_forward, writes dL/dM [3][ny][nx]
 * (derivatives with respect to the stored m11, m12, m22), dL/domega
 * [2][ny][nx] and dL/dt_src [n_src]. The adjoint equations
 * lambda_i = dL/dT_i + sum over the nodes j that i feeds of (dT_j/dT_i) lambda_j
 * are triangular in the causal order; each node gathers from the nodes it
 * feeds (no atomics in the arithmetic). Two schedules (tuning->adjoint_mode):
 *   EIK_ADJ_RELAX (default): each tile relaxes its equations with directional
 *     line sweeps until they hold exactly, and tiles exchange their border
 *     adjoints between rounds (the call synchronises the stream to test that
 *     no border changed; stats, when given, receives the round count);
 *     `level` is not read and may be NULL;
 *   EIK_ADJ_LEVELS: Alg. backward's back-substitution in level order: the
 *     reached nodes of each grid are counting-sorted by `level` (the
 *     forward's dependency levels, required: EIK_EINVAL when NULL) and solved
 *     level by level from the largest, one workgroup per grid; no host
 *     synchronisation.
 * Both give the same lambda (the same sums in the same order). Unreached
 * nodes and the parameters of source nodes get zero gradient. */
int eik_backward(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, const void *T,
                 const uint8_t *parent, const int32_t *level, const void *dLdT, void *dLdM, void *dLdomega,
                 void *dLdsrc, void *ws, size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats,
                 hipStream_t stream);

/* Adjoint of the mixed-precision forward's FP64 state: the eik_backward
 * computation with the donor weights and the parameter derivatives in FP64
 * from (M, omega, T), and the adjoint relaxation itself in FP32 (lambda is a
 * sum of weight-times-lambda terms, which FP32 carries to about 1e-6
 * relative; the sensitivity of the gradient to T sits in the weights, which
 * stay FP64-derived). All real arrays double, laid out as in eik_backward;
 * `level` as in eik_backward (read only by EIK_ADJ_LEVELS); the workspace
 * comes from eik_mixed_workspace_bytes. Errors as eik_backward. */
int eik_backward_mixed(const eik_grid *grid, const double *M, const double *omega, const double *T,
                       const uint8_t *parent, const int32_t *level, const double *dLdT, double *dLdM,
                       double *dLdomega, double *dLdsrc, void *ws, size_t ws_bytes, const eik_tuning *tuning,
                       eik_stats *stats, hipStream_t stream);

/* Batched solving (n_grids independent grids, packed as described above).
 * eik_batch_workspace_bytes sizes the workspace; eik_batch_plan writes the
 * grid descriptors into it (host -> device copy, synchronous) and must be
 * called again when the grids or tuning.tile_height change. The forward and
 * backward batched calls then only enqueue kernels: with stats == NULL they
 * run a fixed schedule (max_rounds sweep rounds per phase, adjoint_rounds
 * adjoint rounds; rounds after convergence exit at once) and never
 * synchronise, so they can be captured in a HIP graph and replayed. */
size_t eik_batch_workspace_bytes(int32_t n_grids, const eik_grid *grids, int32_t dtype);
int eik_batch_plan(int32_t n_grids, const eik_grid *grids, int32_t dtype, const eik_tuning *tuning, void *ws,
                   size_t ws_bytes, hipStream_t stream);
int eik_forward_batched(int32_t n_grids, const eik_grid *grids, int32_t dtype, const int32_t *src_idx,
                        const void *src_t, const void *M, const void *omega, const void *T_init, double tol,
                        int32_t max_rounds, int32_t flags, void *T, uint8_t *parent, int32_t *level, void *ws,
                        size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats, hipStream_t stream);
int eik_backward_batched(int32_t n_grids, const eik_grid *grids, int32_t dtype, const int32_t *src_idx,
                         const void *M, const void *omega, const void *T, const uint8_t *parent,
                         const int32_t *level, const void *dLdT, void *dLdM, void *dLdomega, void *dLdsrc, void *ws,
                         size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats, hipStream_t stream);

/* Batched mixed precision: eik_forward_mixed / eik_backward_mixed over a
 * batch (FP64 parameters, FP32 sweeps to tol32 from the cold start, FP64
 * sweeps from that field to tol, FP64 donor weights and parameter
 * derivatives around an FP32 adjoint relaxation). The workspace, the plan and
 * eik_batch_pending take dtype EIK_MIXED (FP32 copies of the parameters and of
 * T in front of the FP64 batched workspace, which holds the plan of both
 * phases). tuning32 and tuning must share the plan's tile height. Without
 * stats both run their fixed schedules (max_rounds rounds per sweep phase,
 * adjoint_rounds adjoint rounds) and never synchronise (graph-capturable);
 * stats is NULL or an array of two (FP32 phase, FP64 phase) for the forward,
 * one for the backward. Real arrays double; errors as the batched calls. */
int eik_forward_batched_mixed(int32_t n_grids, const eik_grid *grids, const int32_t *src_idx, const double *src_t,
                              const double *M, const double *omega, double tol32, double tol, int32_t max_rounds,
                              int32_t flags, double *T, uint8_t *parent, int32_t *level, void *ws, size_t ws_bytes,
                              const eik_tuning *tuning32, const eik_tuning *tuning, eik_stats *stats,
                              hipStream_t stream);
int eik_backward_batched_mixed(int32_t n_grids, const eik_grid *grids, const int32_t *src_idx, const double *M,
                               const double *omega, const double *T, const uint8_t *parent, const int32_t *level,
                               const double *dLdT, double *dLdM, double *dLdomega, double *dLdsrc, void *ws,
                               size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats, hipStream_t stream);

/* After an unsynchronised batched forward and/or backward (e.g. a graph
 * replay), reads how many tiles were still flagged when the fixed budgets ran
 * out: pending[0] sweep rounds, pending[1] level rounds, pending[2] adjoint
 * rounds. All zero means every phase settled within its budget; otherwise the
 * budgets (max_rounds, tuning) must be raised. Synchronises the stream. */
int eik_batch_pending(int32_t n_grids, const eik_grid *grids, int32_t dtype, const void *ws, size_t ws_bytes,
                      int64_t pending[3], hipStream_t stream);

/* Feasibility projection parameters (App. learning details); the paper leaves
 * the constants open. Defaults: 1e-3, 1e3, 1e3, 0.95. */
typedef struct eik_project_params {
    double eig_min, eig_max, eucl_clip, rho_max;
} eik_project_params;

/* Per node of n: eigenvalues of M by the trace-discriminant formula, clamped to
 * [eig_min, eig_max]; when a clamp is active M is rebuilt from the clamped
 * eigenvalues and the principal angle atan2(2 m12, m11 - m22)/2, otherwise it
 * passes unchanged. omega is clipped to Euclidean norm eucl_clip, then rescaled
 * so that |omega|_{M^-1} <= rho_max. Planes as above with n = nx*ny. */
int eik_project(int64_t n, int32_t dtype, const void *M_in, const void *omega_in, void *M_out, void *omega_out,
                const eik_project_params *params, hipStream_t stream);

/* Vector-Jacobian product of eik_project: given gradients with respect to its
 * outputs, writes gradients with respect to its inputs. */
int eik_project_backward(int64_t n, int32_t dtype, const void *M_in, const void *omega_in, const void *gM_out,
                         const void *gomega_out, void *gM_in, void *gomega_in, const eik_project_params *params,
                         hipStream_t stream);

/* Soft-min mode (Sec. 3.3, the smooth alternative to selecting one stencil
 * named where the paper discusses stencil switches). Each of the eight
 * stencils contributes the minimum of the Hopf-Lax objective over its segment:
 * the two-point value of Eq. two_point when both barycentric weights are >= 0
 * (no causality test), else the smaller one-point value (Eq. one_point) of its
 * finite endpoints; the node takes T = -tau log sum_k exp(-H_k / tau) over the
 * stencils with a finite donor, sources stay at their times. The result is a
 * continuously differentiable function of the parameters; tau -> 0 recovers
 * the minimum over all candidates (within tau ln 8 per update), and the
 * derivative no longer jumps where the active stencil changes.
 *
 * tau must be small against the cost of one step: the soft minimum lies up to
 * tau ln 8 below the smallest H_k, and where that bonus outweighs the step the
 * values fall without limit (no fixed point; EIK_NOT_CONVERGED). A fixed point
 * exists when tau ln 8 < h (1 - |omega|_{M^-1}) sqrt(lambda_min(M)) at every
 * node (each H_k exceeds its smaller donor time by at least that much); it can
 * exist beyond.
 *
 * Workspace: eik_soft_workspace_bytes(grid, dtype) bytes (about 28 reals and
 * one byte per node), caller-owned; 0 for an invalid grid or dtype. Grid sides
 * up to 4096 nodes (EIK_EINVAL beyond). The arrays, dtype and source
 * conventions are those of eik_forward / eik_backward. The batched calls take
 * n_grids grids packed as in eik_forward_batched (src_idx / src_t / dL/dt_src
 * per grid in order), one workgroup per grid, and
 * eik_soft_batch_workspace_bytes; each grid stops at its own first quiet
 * cycle, so its result equals that of a call on it alone. cycle_ms (host, may
 * be NULL) receives the GPU time of the cycle launches, timed with events
 * around each batch of launches between host checks.
 *
 * eik_soft_forward: from +inf (sources at src_t, or 0), repeated cycles of
 * four sweeps of the soft update (rows up, rows down, columns up, columns
 * down; the nodes of one line at once from the current values) until a cycle
 * changes no value by more than tol max(|T|, largest |T| of the previous
 * cycle), or max_cycles cycles (EIK_NOT_CONVERGED, T valid). cycles (NULL or
 * one int32 per grid, host memory) receives the cycles each grid ran.
 * Synchronises the stream once per 4 cycles.
 *
 * eik_soft_backward: vector-Jacobian product of the converged field T of
 * eik_soft_forward (same tau, grid and parameters): solves (I - J^T) lambda =
 * dL/dT over the reached nodes, J the partial derivatives of each node's soft
 * update with respect to its neighbours' times, by cycles of the same four
 * sweeps (stopping as above, on lambda); then dL/dM, dL/domega (planes as M,
 * omega; zero at sources and unreached nodes) = lambda times the update's
 * partial derivatives with respect to the node's stored parameters, and
 * dL/dt_src[s] = lambda at source s. The system is not triangular (every node
 * depends on all its neighbours), hence the iteration. Errors as
 * eik_soft_forward. */
size_t eik_soft_workspace_bytes(const eik_grid *grid, int32_t dtype);
int eik_soft_forward(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, double tau, double tol,
                     int32_t max_cycles, void *T, void *ws, size_t ws_bytes, int32_t *cycles, hipStream_t stream);
int eik_soft_backward(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, const void *T,
                      double tau, const void *dLdT, double tol, int32_t max_cycles, void *dLdM, void *dLdomega,
                      void *dLdsrc, void *ws, size_t ws_bytes, int32_t *cycles, hipStream_t stream);
size_t eik_soft_batch_workspace_bytes(int32_t n_grids, const eik_grid *grids, int32_t dtype);
int eik_soft_forward_batched(int32_t n_grids, const eik_grid *grids, int32_t dtype, const int32_t *src_idx,
                             const void *src_t, const void *M, const void *omega, double tau, double tol,
                             int32_t max_cycles, void *T, void *ws, size_t ws_bytes, int32_t *cycles,
                             double *cycle_ms, hipStream_t stream);
int eik_soft_backward_batched(int32_t n_grids, const eik_grid *grids, int32_t dtype, const int32_t *src_idx,
                              const void *M, const void *omega, const void *T, double tau, const void *dLdT,
                              double tol, int32_t max_cycles, void *dLdM, void *dLdomega, void *dLdsrc, void *ws,
                              size_t ws_bytes, int32_t *cycles, double *cycle_ms, hipStream_t stream);

/* Thread-local description of the last non-OK status. */
const char *eik_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EIK_H */
