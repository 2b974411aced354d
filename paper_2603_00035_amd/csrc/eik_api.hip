// eik_api.hip -- the C ABI declared in include/eik.h: argument checks,
// workspace layout, and the order of kernel launches on the caller's stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/eik.h"
#include "../../include/eik_encoder.h"
#include "../../include/eik_inverse.h"
#include "eik_internal.h"

using namespace eik;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_OK(expr)                                                                                       \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess) return fail(EIK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kDefaultTH = 64;

// Sizes of a launch over a set of grids.
struct Extent {
    int64_t nodes = 0;
    int64_t tiles32 = 0, tiles64 = 0;
    int32_t n_grids = 0, n_src = 0;
};

int64_t tiles_of(int nx, int ny, int th) { return (int64_t)((nx + TW - 1) / TW) * ((ny + th - 1) / th); }

struct Layout {
    size_t descs, tile_grid, act, act_count, ctr, Pt, lam, w1, adjD, adjDT, adjGT, qring, qstate, qctl, total;
    uint32_t qslots;
};

constexpr int kMaxQueueWaves = 4096;

// Ring slots of the work queue: a power of two above twice (tiles + waves).
uint32_t queue_slots(size_t n_tiles)
{
    uint32_t c = 1024;
    while (c < 2 * (n_tiles + kMaxQueueWaves)) c <<= 1;
    return c;
}

Layout layout(const Extent &e, int dtype)
{
    const size_t rs = dtype == EIK_F64 ? 8 : 4;
    const size_t NT = (size_t)std::max(e.tiles32, e.tiles64);
    Layout L;
    size_t o = 0;
    L.descs = o;     o += align256((size_t)e.n_grids * sizeof(GridDesc));
    L.tile_grid = o; o += align256(NT * 4);
    L.act = o;       o += align256(2 * NT * 4);
    L.act_count = o; o += align256((size_t)(kMaxRounds + 2) * 4);
    L.ctr = o;       o += align256(kCtrCount * 8);
    // staged sweep inputs: parameters (and, in FP64, the metric roots in both orientations)
    L.Pt = o;        o += align256((dtype == EIK_F64 ? 5 + 2 * 6 : 5) * (size_t)e.nodes * rs);
    L.lam = o;       o += align256((size_t)e.nodes * rs);
    L.w1 = o;        o += align256((size_t)e.nodes * rs);
    L.adjD = o;      o += align256((size_t)e.nodes * 2);
    L.adjDT = o;     o += align256((size_t)e.nodes * 2);
    L.adjGT = o;     o += align256((size_t)e.nodes * rs);

    L.qslots = queue_slots(NT);
    L.qring = o;     o += align256((size_t)L.qslots * 4);
    L.qstate = o;    o += align256(NT * 4);
    L.qctl = o;      o += align256(kQCtlWords * 4);
    L.total = o;
    return L;
}

int check_one(const eik_grid *g, int idx)
{
    if (g->nx < 1 || g->ny < 1) return fail(EIK_EINVAL, "grid %d: size %d x %d", idx, g->nx, g->ny);
    if ((int64_t)g->nx * g->ny >= ((int64_t)1 << 31)) return fail(EIK_EINVAL, "grid %d: 2^31 nodes or more", idx);
    if (!(g->h > 0.0)) return fail(EIK_EINVAL, "grid %d: spacing h must be positive", idx);
    if (g->n_src < 1) return fail(EIK_EINVAL, "grid %d: at least one source is required", idx);
    return EIK_OK;
}

int extent_of(int n_grids, const eik_grid *grids, int dtype, Extent &e)
{
    if (!grids || n_grids < 1) return fail(EIK_EINVAL, "no grids");
    if (dtype != EIK_F32 && dtype != EIK_F64) return fail(EIK_EINVAL, "dtype %d", dtype);
    e = Extent();
    e.n_grids = n_grids;
    for (int g = 0; g < n_grids; ++g) {
        int rc = check_one(&grids[g], g);
        if (rc) return rc;
        e.nodes += (int64_t)grids[g].nx * grids[g].ny;
        e.tiles32 += tiles_of(grids[g].nx, grids[g].ny, 32);
        e.tiles64 += tiles_of(grids[g].nx, grids[g].ny, 64);
        e.n_src += grids[g].n_src;
    }
    if (std::max(e.tiles32, e.tiles64) >= ((int64_t)1 << 30)) return fail(EIK_EINVAL, "too many tiles");
    return EIK_OK;
}

// Host-side descriptors of a launch.
void host_descs(int n_grids, const eik_grid *grids, int th, std::vector<GridDesc> &d, std::vector<int32_t> &tg)
{
    d.resize(n_grids);
    tg.clear();
    int64_t off = 0;
    int32_t tb = 0, sb = 0;
    for (int g = 0; g < n_grids; ++g) {
        GridDesc x;
        memset(&x, 0, sizeof x);
        x.off = off;
        x.h = grids[g].h;
        x.nx = grids[g].nx;
        x.ny = grids[g].ny;
        x.ntx = (x.nx + TW - 1) / TW;
        x.nty = (x.ny + th - 1) / th;
        x.tile_base = tb;
        x.n_src = grids[g].n_src;
        x.src_base = sb;
        d[g] = x;
        for (int t = 0; t < x.ntx * x.nty; ++t) tg.push_back(g);
        off += (int64_t)x.nx * x.ny;
        tb += x.ntx * x.nty;
        sb += x.n_src;
    }
}

struct Ws {
    GridDesc *descs;
    int32_t *tile_grid, *act, *act_count;
    unsigned long long *ctr;
    void *Pt, *lam, *w1;
    uint16_t *adjD, *adjDT;
    void *adjGT;
    WorkQueue q;
};

int carve(const Extent &e, int dtype, void *ws, size_t ws_bytes, Ws &w)
{
    const Layout L = layout(e, dtype);
    if (!ws || ws_bytes < L.total)
        return fail(EIK_EWORKSPACE, "workspace %zu bytes, %zu needed", ws_bytes, L.total);
    char *b = (char *)ws;
    w.descs = (GridDesc *)(b + L.descs);
    w.tile_grid = (int32_t *)(b + L.tile_grid);
    w.act = (int32_t *)(b + L.act);
    w.act_count = (int32_t *)(b + L.act_count);
    w.ctr = (unsigned long long *)(b + L.ctr);
    w.Pt = b + L.Pt;
    w.lam = b + L.lam;
    w.w1 = b + L.w1;
    w.adjD = (uint16_t *)(b + L.adjD);
    w.adjDT = (uint16_t *)(b + L.adjDT);
    w.adjGT = b + L.adjGT;

    w.q.ring = (uint32_t *)(b + L.qring);
    w.q.state = (uint32_t *)(b + L.qstate);
    w.q.ctl = (uint32_t *)(b + L.qctl);
    w.q.mask = L.qslots - 1;
    w.q.spin_limit = 1u << 21;
    return EIK_OK;
}

eik_tuning tuning_or_default(const eik_tuning *t)
{
    eik_tuning d;
    d.tile_height = kDefaultTH;
    d.max_local_cycles = 1;
    d.rounds_per_check = 8;
    d.fast_cold_start = 2;
    d.adjoint_rounds = 64;
    d.level_rounds = 8;
    d.scheduler = EIK_SCHED_ROUNDS;
    d.node_lanes = 4;
    d.adjoint_cycles = 1;
    d.adjoint_waves = 4;
    d.full_waves = 4;
    d.adjoint_mode = EIK_ADJ_RELAX;
    d.level_mode = EIK_LEVELS_CARRIED;
    if (t) {
        if (t->tile_height == 32 || t->tile_height == 64) d.tile_height = t->tile_height;
        if (t->max_local_cycles >= 1) d.max_local_cycles = t->max_local_cycles;
        if (t->rounds_per_check >= 1) d.rounds_per_check = t->rounds_per_check;
        if (t->fast_cold_start >= 0) d.fast_cold_start = std::min(t->fast_cold_start, 2);
        if (t->adjoint_rounds >= 1) d.adjoint_rounds = t->adjoint_rounds;
        if (t->level_rounds >= 1) d.level_rounds = t->level_rounds;
        if (t->scheduler == EIK_SCHED_ROUNDS || t->scheduler == EIK_SCHED_QUEUE) d.scheduler = t->scheduler;
        if (t->node_lanes == 1 || t->node_lanes == 2 || t->node_lanes == 4) d.node_lanes = t->node_lanes;
        if (t->adjoint_cycles >= 1) d.adjoint_cycles = t->adjoint_cycles;
        if (t->adjoint_waves == 1 || t->adjoint_waves == 4) d.adjoint_waves = t->adjoint_waves;
        if (t->full_waves == 1 || t->full_waves == 4) d.full_waves = t->full_waves;
        if (t->adjoint_mode == EIK_ADJ_RELAX || t->adjoint_mode == EIK_ADJ_LEVELS) d.adjoint_mode = t->adjoint_mode;
        if (t->level_mode == EIK_LEVELS_CARRIED || t->level_mode == EIK_LEVELS_AFTER) d.level_mode = t->level_mode;
    }
    return d;
}

// Optional timing with HIP events recorded on the launch stream: one pair
// around each batch of rounds enqueued between host checks, so the timing adds
// nothing between the launches of a batch.
struct LaunchTimer {
    std::vector<hipEvent_t> ev;
    int used = 0;
    double ms = 0.0;
    bool on = false;
    ~LaunchTimer()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    int init(bool enable)
    {
        on = enable;
        if (!on) return EIK_OK;
        ev.resize(2);
        for (auto &e : ev) HIP_OK(hipEventCreate(&e));
        return EIK_OK;
    }
    void before(hipStream_t st)
    {
        if (on) (void)hipEventRecord(ev[2 * used], st);
    }
    void after(hipStream_t st)
    {
        if (on) (void)hipEventRecord(ev[2 * used + 1], st), ++used;
    }
    void collect() // after the stream has been synchronised
    {
        for (int b = 0; b < used; ++b) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[2 * b], ev[2 * b + 1]) == hipSuccess) ms += t;
        }
        used = 0;
    }
};

// Slot of the counter block, beyond those the kernels use, that carries the
// flagged-tile count of a host check.
constexpr int kCtrCheck = kCtrCount - 1;
static_assert(kCtrCheck > kCtrFastUpdates, "the check slot must be free");

// Rounds until a round flags nothing (converged) or the budget runs out.
// Without a host check (sync = false) exactly `budget` rounds are enqueued;
// rounds after convergence find no flagged tile and exit at once. With host
// checks, the first check comes after `first_batch` rounds (a phase that
// starts near its fixed point settles in one or two), else after `per_check`
// rounds (the tuned estimate of a whole phase); later checks come every
// min(per_check, 8) rounds, so a phase that needs a few rounds more than the
// estimate enqueues a few more launches, not another full batch (a host
// check costs about as much as ten launches that find no flagged tile).
// round_fn(act_in, act_out, count_next) enqueues one round. With ctr_host,
// every check also copies the counter block there (the count read through
// slot kCtrCheck, so that one copy serves both).
template <typename F>
int run_rounds(int32_t *act, int32_t *act_count, int n_tiles, int first, int budget, int per_check, bool sync,
               hipStream_t st, F round_fn, int *rounds_done, bool *converged, LaunchTimer *timer = nullptr,
               int first_batch = 0, int32_t *last_count = nullptr, unsigned long long *ctr_dev = nullptr,
               unsigned long long *ctr_host = nullptr)
{
    int r = first;
    const int end = std::min(first + budget, kMaxRounds);
    const int later = std::min(per_check, 8);
    *converged = false;
    while (r < end) {
        const int want = r == first ? (first_batch > 0 ? std::min(first_batch, per_check) : per_check) : later;
        const int batch = sync ? std::min(want, end - r) : end - r;
        if (timer && timer->on) timer->before(st);
        for (int b = 0; b < batch; ++b, ++r)
            round_fn(act + (r & 1) * n_tiles, act + ((r + 1) & 1) * n_tiles, act_count + r + 1);
        if (timer && timer->on) timer->after(st);
        if (!sync) break;
        int32_t cnt = 0;
        if (ctr_host) {
            // one copy back for both: the flagged-tile count goes into a free
            // slot of the counter block first
            launch_note_pending(act_count + r, ctr_dev + kCtrCheck, st);
            HIP_OK(hipMemcpyAsync(ctr_host, ctr_dev, kCtrCount * sizeof *ctr_host, hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
            cnt = (int32_t)ctr_host[kCtrCheck];
        } else {
            HIP_OK(hipMemcpyAsync(&cnt, act_count + r, sizeof cnt, hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
        }
        if (timer && timer->on) timer->collect();
        if (last_count) *last_count = cnt;
        if (cnt == 0) {
            *converged = true;
            break;
        }
    }
    *rounds_done = r - first;
    return EIK_OK;
}

int prepare(int n_grids, const eik_grid *grids, int dtype, void *ws, size_t ws_bytes, const eik_tuning &tn,
            bool write_desc, hipStream_t st, Extent &e, Ws &w, LaunchArgs &a)
{
    int rc = extent_of(n_grids, grids, dtype, e);
    if (rc) return rc;
    rc = carve(e, dtype, ws, ws_bytes, w);
    if (rc) return rc;
    a.grids = w.descs;
    a.tile_grid = w.tile_grid;
    a.n_grids = n_grids;
    a.th = tn.tile_height;
    a.n_tiles = (int32_t)(a.th == 64 ? e.tiles64 : e.tiles32);
    a.n_nodes = e.nodes;
    if (write_desc) { // single grid: descriptor written by a kernel, no host copy
        GridDesc d;
        memset(&d, 0, sizeof d);
        d.h = grids[0].h;
        d.nx = grids[0].nx;
        d.ny = grids[0].ny;
        d.ntx = (d.nx + TW - 1) / TW;
        d.nty = (d.ny + a.th - 1) / a.th;
        d.n_src = grids[0].n_src;
        launch_write_single_desc(d, w.descs, w.tile_grid, a.n_tiles, st);
    }
    return EIK_OK;
}

template <typename R>
int forward_impl(int n_grids, const eik_grid *grids, const int32_t *src_idx, const void *src_t, const void *M,
                 const void *om, const void *T_init, double tol, int max_rounds, int flags, void *T,
                 uint8_t *parent, int32_t *level, void *ws, size_t ws_bytes, const eik_tuning *tun,
                 eik_stats *stats, bool single, hipStream_t st, bool certify = true, bool pre_staged = false,
                 const std::function<int()> &after_init = nullptr, int full_first_batch = -1,
                 const double *M64 = nullptr, const double *om64 = nullptr)
{ // M64, om64 (FP32 solves only): M and omega are FP32 copies to be made from them by the staging
    const int dtype = sizeof(R) == 8 ? EIK_F64 : EIK_F32;
    // the sweeps keep the source marks in the parent array
    if (!T || !parent) return fail(EIK_EINVAL, "T and parent arrays are required");
    const eik_tuning tn = tuning_or_default(tun);
    Extent e;
    Ws w;
    LaunchArgs a;
    int rc = prepare(n_grids, grids, dtype, ws, ws_bytes, tn, single, st, e, w, a);
    if (rc) return rc;
    // Without a stats request a batched forward runs a fixed schedule with no
    // host synchronisation (capturable in a graph).
    const bool sync = single || stats != nullptr;
    max_rounds = std::max(1, std::min(max_rounds, kMaxRounds / 4));

    HIP_OK(hipGetLastError());
    if (flags & EIK_CHECK_FEASIBLE) {
        launch_fill_u64(w.ctr, kCtrCount, st);
        launch_check_feasible<R>(e.nodes, M, om, w.ctr, st);
        unsigned long long bad = 0;
        HIP_OK(hipMemcpyAsync(&bad, w.ctr + kCtrInfeasible, 8, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (bad) return fail(EIK_EINFEASIBLE, "metric not SPD or |omega|_{M^-1} >= 1 somewhere");
    }
    if constexpr (sizeof(R) == 4) {
        if (M64) launch_stage_from64(a, M64, om64, (float *)M, (float *)om, w.Pt, st); // casts and staging at once
        else if (!pre_staged) launch_stage<R>(a, M, om, w.Pt, st);
    } else if (!pre_staged) {
        launch_stage<R>(a, M, om, w.Pt, st); // else staged in this workspace already
    }
    // initial field, and the round state cleared in the same launch
    launch_init<R>(a, T_init, T, parent, level, src_idx, src_t, w.act, w.act_count, w.ctr, T_init != nullptr,
                   st, /*reset=*/true);
    HIP_OK(hipGetLastError());
    if (after_init) { // the caller's work to enqueue once the sweeps are next (the mixed path's side stream)
        rc = after_init();
        if (rc) return rc;
    }

    LaunchTimer timer;
    rc = timer.init((flags & EIK_TIME_KERNELS) != 0 && sync);
    if (rc) return rc;
    int r0 = 0, rounds = 0;
    bool conv = false;
    // counters as of the last host check; when the last sweep phase ends
    // converged at such a check and nothing after it counts (no level rounds),
    // they are the final ones and the call returns without another
    // synchronisation (the stencil pass that follows runs behind it)
    unsigned long long hctr[kCtrCount];
    bool hctr_final = false;
    // Warm start with a fallback: two full-update rounds from T_init probe it;
    // a field that leaves more than a quarter of the tiles changing is dropped
    // and the solve restarts from the cold start.
    bool fell_back = false, probe_done = false;
    int probe_rounds = 0;
    if (T_init && (flags & EIK_WARM_FALLBACK) && sync && tn.scheduler == EIK_SCHED_ROUNDS) {
        int32_t left = 0;
        rc = run_rounds(
            w.act, w.act_count, a.n_tiles, 0, 2, 2, sync, st,
            [&](int32_t *ain, int32_t *aout, int32_t *cnt) {
                launch_sweep_round<R>(a, kModeFull, M, om, w.Pt, T, parent, level, ain, aout, cnt, w.ctr, tol,
                                      tn.max_local_cycles, tn.full_waves == 4 ? kFullWavesCD : tn.node_lanes, st);
            },
            &probe_rounds, &conv, &timer, 0, &left, w.ctr, hctr);
        if (rc) return rc;
        probe_done = true;
        if (!conv && 4 * (int64_t)left > a.n_tiles) {
            fell_back = true;
            launch_fill_i32(w.act, 2 * (int64_t)a.n_tiles, 0, st);
            launch_fill_i32(w.act_count, kMaxRounds + 2, 0, st);
            launch_init<R>(a, nullptr, T, parent, level, src_idx, src_t, w.act, w.act_count, w.ctr, false, st);
            HIP_OK(hipGetLastError());
        } else {
            r0 = probe_rounds;
        }
    }
    const bool fast = (T_init == nullptr || fell_back) && tn.fast_cold_start;
    // levels carried by the sweeps (one-wave visits), or computed afterwards
    // by the level rounds alone while the sweeps run as without levels
    int32_t *sweep_level = tn.level_mode == EIK_LEVELS_AFTER ? nullptr : level;
    // exact stationarity before certification here; without it (the mixed
    // path's FP32 phase) the caller's tolerance, its FP64 phase converging
    // from any start
    const double fast_tol = certify ? 0.0 : tol;
    if (fast) {
        // cold start: restricted candidates, T only decreases. Run to exact
        // stationarity of this min-update (finite: every store lowers a
        // value), so the full rounds that follow start from the fixed point
        // rather than from a field left within tol of it.
        rc = run_rounds(
            w.act, w.act_count, a.n_tiles, r0, max_rounds, tn.rounds_per_check, sync, st,
            [&](int32_t *ain, int32_t *aout, int32_t *cnt) {
                launch_sweep_round<R>(a, tn.fast_cold_start == 2 ? kModeFastCD : kModeFast, M, om, w.Pt, T,
                                      parent, sweep_level, ain, aout, cnt, w.ctr, fast_tol, tn.max_local_cycles, 1,
                                      st);
            },
            &rounds, &conv, &timer, 0, nullptr, w.ctr, hctr);
        if (rc) return rc;
        r0 += rounds;
        hctr_final = !certify && sync && conv;
        // the cold start's update count, for the stats (read on the device
        // only when the counters are read again at the end)
        if (!hctr_final) launch_copy_u64(w.ctr + kCtrCellUpdates, w.ctr + kCtrFastUpdates, st);
        hctr[kCtrFastUpdates] = hctr[kCtrCellUpdates];
        // certify with the full update: every tile runs once more
        if (certify) launch_all_active(a, w.act + (r0 & 1) * a.n_tiles, w.act_count + r0, st);
    }
    int launches = r0;
    const int fast_launches = r0;
    const double fast_ms = timer.ms;
    if (fast && !certify) {
        // no full rounds: the caller continues from this field with full
        // updates of its own (the mixed path's FP64 phase), which converge to
        // the full update's fixed point from any start
    } else if (probe_done && !fell_back && conv) {
        launches = r0; // the warm start's two probe rounds reached the fixed point
        hctr_final = true;
    } else if (tn.scheduler == EIK_SCHED_QUEUE) {
        // one persistent launch over a device queue of flagged tiles
        const int waves =
            std::min({sweep_queue_waves(a.th, dtype, sweep_level != nullptr), kMaxQueueWaves, a.n_tiles});
        if (waves < 1) return fail(EIK_EDEVICE, "no occupancy for the work-queue sweep kernel");
        const uint32_t budget = (uint32_t)std::min<int64_t>((int64_t)max_rounds * a.n_tiles, INT32_MAX);
        launch_queue_setup(a, w.act + (r0 & 1) * a.n_tiles, w.q, budget, st);
        if (timer.on) timer.before(st);
        launch_sweep_queue<R>(a, waves, M, om, w.Pt, T, parent, sweep_level, w.q, w.ctr, tol, tn.max_local_cycles,
                              st);
        if (timer.on) timer.after(st);
        launch_note_queue(w.q, w.ctr + kCtrSweepPending, st);
        HIP_OK(hipGetLastError());
        launches += 1;
        if (sync) {
            uint32_t ctl[kQCtlWords];
            HIP_OK(hipMemcpyAsync(ctl, w.q.ctl, sizeof ctl, hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
            if (timer.on) timer.collect();
            if (ctl[kQFail]) return fail(EIK_EDEVICE, "work queue: a wait exceeded its poll limit");
            conv = ctl[kQPending] == 0 && !ctl[kQStop];
            r0 += (int)(((int64_t)ctl[kQVisits] + a.n_tiles - 1) / a.n_tiles);
        }
    } else {
        rc = run_rounds(
            w.act, w.act_count, a.n_tiles, r0, max_rounds, tn.rounds_per_check, sync, st,
            [&](int32_t *ain, int32_t *aout, int32_t *cnt) {
                launch_sweep_round<R>(a, kModeFull, M, om, w.Pt, T, parent, sweep_level, ain, aout, cnt, w.ctr,
                                      tol, tn.max_local_cycles, tn.full_waves == 4 ? kFullWavesCD : tn.node_lanes,
                                      st);
            },
            &rounds, &conv, &timer, full_first_batch >= 0 ? full_first_batch : ((fast || T_init) ? 2 : 0), nullptr,
            w.ctr, hctr);
        if (rc) return rc;
        r0 += rounds;
        launches = r0;
        hctr_final = sync && conv;
        launch_note_pending(w.act_count + r0, w.ctr + kCtrSweepPending, st);
        HIP_OK(hipGetLastError());
    }

    // active stencils from the final field (skipped without certification:
    // the mixed path's FP32 phase, whose stencils the FP64 phase recomputes),
    // then (when asked for) levels made consistent with them
    if (certify) launch_parents<R>(a, M, om, T, parent, st);
    int lrounds = 0;
    if (level) {
        launch_fill_i32(w.act, 2 * (int64_t)a.n_tiles, 0, st);
        launch_fill_i32(w.act_count, kMaxRounds + 2, 0, st);
        launch_all_active(a, w.act, w.act_count, st);
        bool lconv = false;
        const int level_budget = sync ? kMaxRounds / 2 : tn.level_rounds;
        rc = run_rounds(
            w.act, w.act_count, a.n_tiles, 0, level_budget, tn.rounds_per_check, sync, st,
            [&](int32_t *ain, int32_t *aout, int32_t *cnt) {
                launch_level_round(a, parent, level, ain, aout, cnt, tn.max_local_cycles, st);
            },
            &lrounds, &lconv);
        if (rc) return rc;
        if (sync && !lconv) return fail(EIK_EDEVICE, "dependency levels did not settle");
        launch_note_pending(w.act_count + lrounds, w.ctr + kCtrLevelPending, st);
        launch_max_level(e.nodes, level, w.ctr, st);
    }
    HIP_OK(hipGetLastError());
    if (!sync) return EIK_OK;

    unsigned long long ctr[kCtrCount];
    if (hctr_final && !level) {
        memcpy(ctr, hctr, sizeof ctr);
    } else {
        HIP_OK(hipMemcpyAsync(ctr, w.ctr, sizeof ctr, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
    }
    int status = conv ? EIK_OK : EIK_NOT_CONVERGED;
    if (ctr[kCtrBadSource]) status = fail(EIK_EINVAL, "%llu source indices out of range", ctr[kCtrBadSource]);
    else if (!conv) fail(EIK_NOT_CONVERGED, "tolerance not reached in %d rounds", r0);
    if (stats) {
        stats->rounds = r0 + (fell_back ? probe_rounds : 0);
        stats->converged = conv ? 1 : 0;
        stats->cell_updates = (int64_t)ctr[kCtrCellUpdates];
        stats->n_levels = level ? (int32_t)ctr[kCtrMaxLevel] + 1 : 0;
        stats->status = status;
        stats->sweep_launches = launches + (fell_back ? probe_rounds : 0);
        stats->fell_back = fell_back ? 1 : 0;
        stats->sweep_ms = timer.ms;
        stats->aux_rounds = lrounds;
        stats->fast_ms = fast_ms;
        stats->fast_cell_updates = fast ? (int64_t)ctr[kCtrFastUpdates] : 0;
        stats->fast_launches = fast_launches;
    }
    return status;
}

// Workspace of the mixed-precision calls: FP32 copies of the parameters, the
// FP32 field and source times, then the workspace of the FP64 solve, which the
// FP32 solve uses before it. The mixed adjoint keeps its FP32 weights, dL/dT
// and lambda in the first three regions.
// With split (the single-grid mixed forward), the FP32 phase gets a workspace
// of its own after the FP64 one, so that the FP64 staging can run beside the
// FP32 sweeps; the batched calls share one (their plan serves both phases).
struct MixedLayout {
    size_t M32, om32, T32, src32, base, ws32, total;
};

MixedLayout mixed_layout(const Extent &e, bool split = false)
{
    const size_t n = (size_t)e.nodes;
    MixedLayout L;
    size_t o = 0;
    L.M32 = o;   o += align256(3 * n * 4);
    L.om32 = o;  o += align256(2 * n * 4);
    L.T32 = o;   o += align256(n * 4);
    L.src32 = o; o += align256((size_t)e.n_src * 4);
    L.base = o;  o += align256(layout(e, EIK_F64).total);
    L.ws32 = split ? o : L.base;
    if (split) o += layout(e, EIK_F32).total;
    L.total = o;
    return L;
}

// Workgroups of the FP64 staging beside the FP32 sweeps, one per CU: on the
// 2048^2 stress field one per tile (1024) holds the CUs until it ends and
// delays the first rounds, 64 stretch it over the whole FP32 phase and slow
// every round; 256 gave the shortest step (4.95 ms median against 5.07 and
// 5.12; 5.26 without the overlap).
constexpr int kSideStageBlocks = 256;

// A non-blocking stream of default priority per device, created on first use
// and kept for the life of the process: the mixed forward stages its FP64
// inputs there while the FP32 sweeps run on the caller's stream.
int side_stream(hipStream_t caller, hipStream_t &out)
{
    static std::mutex mu;
    static std::vector<hipStream_t> streams;
    int dev = 0, cur = 0;
    HIP_OK(hipStreamGetDevice(caller, &dev));
    HIP_OK(hipGetDevice(&cur));
    if (dev != cur) return fail(EIK_EINVAL, "the stream belongs to device %d while device %d is current", dev, cur);
    std::lock_guard<std::mutex> lock(mu);
    if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
    if (!streams[dev]) HIP_OK(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
    out = streams[dev];
    return EIK_OK;
}

// Events of one fork/join between the caller's stream and the side stream,
// released when the call returns (a recorded event may be destroyed before it
// completes).
struct ForkEvents {
    hipEvent_t fork = nullptr, join = nullptr;
    ~ForkEvents()
    {
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
    }
};

// The adjoint relaxation (round or queue scheduler) on lambda of type RL.
template <typename RL>
int relax(const LaunchArgs &a, Ws &w, const eik_tuning &tn, bool sync, const AdjNodes &nd, const void *w1, void *lam,
          hipStream_t st, int &rounds, bool &conv)
{
    const int dtype = sizeof(RL) == 8 ? EIK_F64 : EIK_F32;
    launch_round_reset(a, w.act, w.act_count, st);
    HIP_OK(hipGetLastError());
    rounds = 0;
    conv = false;
    if (tn.scheduler == EIK_SCHED_QUEUE) {
        const int waves = std::min({adj_queue_waves(a.th, dtype), kMaxQueueWaves, a.n_tiles});
        if (waves < 1) return fail(EIK_EDEVICE, "no occupancy for the work-queue adjoint kernel");
        const int budget_rounds = sync ? kMaxRounds / 2 : tn.adjoint_rounds;
        const uint32_t budget = (uint32_t)std::min<int64_t>((int64_t)budget_rounds * a.n_tiles, INT32_MAX);
        launch_queue_setup(a, w.act, w.q, budget, st);
        launch_adj_queue<RL>(a, waves, nd, w1, lam, tn.adjoint_cycles, w.q, st);
        launch_note_queue(w.q, w.ctr + kCtrAdjPending, st);
        HIP_OK(hipGetLastError());
        if (sync) {
            uint32_t ctl[kQCtlWords];
            HIP_OK(hipMemcpyAsync(ctl, w.q.ctl, sizeof ctl, hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
            if (ctl[kQFail]) return fail(EIK_EDEVICE, "work queue: a wait exceeded its poll limit");
            conv = ctl[kQPending] == 0 && !ctl[kQStop];
            rounds = (int)(((int64_t)ctl[kQVisits] + a.n_tiles - 1) / a.n_tiles);
            if (!conv) return fail(EIK_EDEVICE, "adjoint visits did not settle");
        }
    } else {
        int rc = run_rounds(
            w.act, w.act_count, a.n_tiles, 0, sync ? kMaxRounds / 2 : tn.adjoint_rounds, tn.rounds_per_check, sync,
            st,
            [&](int32_t *ain, int32_t *aout, int32_t *cnt) {
                launch_adj_round<RL>(a, nd, w1, lam, tn.adjoint_cycles, tn.adjoint_waves, ain, aout, cnt, st);
            },
            &rounds, &conv);
        if (rc) return rc;
        if (sync && !conv) return fail(EIK_EDEVICE, "adjoint rounds did not settle");
        launch_note_pending(w.act_count + rounds, w.ctr + kCtrAdjPending, st);
    }
    return EIK_OK;
}

// FP32 buffers of the mixed-precision adjoint (donor weights, dL/dT, lambda).
struct Relax32 {
    float *w1, *g, *lam;
};

template <typename R>
int backward_impl(int n_grids, const eik_grid *grids, const int32_t *src_idx, const void *M, const void *om,
                  const void *T, const uint8_t *parent, const int32_t *level, const void *dLdT, void *dLdM,
                  void *dLdom, void *dLdsrc, void *ws, size_t ws_bytes, const eik_tuning *tun, bool single,
                  eik_stats *stats, hipStream_t st, const Relax32 *r32 = nullptr)
{
    const int dtype = sizeof(R) == 8 ? EIK_F64 : EIK_F32;
    // the sweeps keep the source marks in the parent array
    if (!T || !parent) return fail(EIK_EINVAL, "T and parent arrays are required");
    const eik_tuning tn = tuning_or_default(tun);
    Extent e;
    Ws w;
    LaunchArgs a;
    int rc = prepare(n_grids, grids, dtype, ws, ws_bytes, tn, single, st, e, w, a);
    if (rc) return rc;
    const bool sync = single || stats != nullptr;

    // The relaxation needs no levels (each tile sweeps until its equations
    // hold exactly); the level-scheduled gather sorts the nodes by the
    // forward's levels. Its node list, bins and per-grid largest level take
    // the place of the staged parameters, which only the forward sweeps use
    // (5 reals per node >= 2 ints per node + one int per grid).
    const bool by_levels = tn.adjoint_mode == EIK_ADJ_LEVELS;
    if (by_levels && !level) return fail(EIK_EINVAL, "the level-scheduled adjoint needs the forward's levels");
    int32_t *lv_order = (int32_t *)w.Pt, *lv_bins = lv_order + e.nodes, *lv_gmax = lv_bins + e.nodes;
    launch_fill_u64(w.ctr + kCtrAdjPending, 1, st);
    Prep32 p32; // the FP32 relaxation's inputs written by the preparation itself
    if (r32) {
        p32.w1 = r32->w1;
        p32.g_src = dLdT;
        p32.g = r32->g;
        p32.lam = r32->lam;
    }
    launch_adj_prep<R>(a, M, om, T, parent, w.w1, w.lam, st, p32);
    int rounds = 0;
    bool conv = false;
    if (by_levels) launch_level_buckets(a, level, lv_gmax, lv_bins, lv_order, st);
    if (r32) { // weights from the state in R, lambda relaxed in FP32, then widened
        launch_adj_stage<float>(a, parent, r32->g, w.adjD, w.adjDT, w.adjGT, st);
        if (by_levels) {
            launch_level_gather<float>(a, lv_gmax, lv_bins, lv_order, w.adjD, r32->g, r32->w1, r32->lam, st);
            conv = true;
        } else {
            const AdjNodes nd = {w.adjD, w.adjDT, r32->g, w.adjGT};
            rc = relax<float>(a, w, tn, sync, nd, r32->w1, r32->lam, st, rounds, conv);
            if (rc) return rc;
        }
        launch_cast_f32_f64(e.nodes, r32->lam, (double *)w.lam, st);
    } else {
        launch_adj_stage<R>(a, parent, dLdT, w.adjD, w.adjDT, w.adjGT, st);
        if (by_levels) {
            launch_level_gather<R>(a, lv_gmax, lv_bins, lv_order, w.adjD, dLdT, w.w1, w.lam, st);
            conv = true;
        } else {
            const AdjNodes nd = {w.adjD, w.adjDT, dLdT, w.adjGT};
            rc = relax<R>(a, w, tn, sync, nd, w.w1, w.lam, st, rounds, conv);
            if (rc) return rc;
        }
    }
    launch_adj_params<R>(a, M, parent, w.w1, w.lam, dLdM, dLdom, st);
    launch_dsrc<R>(a, src_idx, w.lam, dLdsrc, st);
    HIP_OK(hipGetLastError());
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->rounds = rounds;
        stats->converged = conv ? 1 : 0;
        stats->aux_rounds = rounds;
    }
    return EIK_OK;
}

int check_ptrs(const void *M, const void *om, const void *T, const void *parent)
{
    if (!M || !om || !T || !parent) return fail(EIK_EINVAL, "NULL field or output pointer");
    return EIK_OK;
}

// ---------------------------------------------------------------------------
// Workspace of eik_forward_noalloc: a fixed device array of this file instead
// of the caller's buffer. Each GPU holds its own copy for the life of the
// process; its device address is looked up once per device, on the first call
// made with that device current, and kept. Every call on a device uses the
// same array: the solve clears what must start at zero (counters, tile flags)
// with fill kernels and writes every other region before reading it, so the
// previous call's contents do not matter, but calls that overlap on one GPU
// (other streams or host threads) race.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void **out)
{
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(EIK_EDEVICE, "device %d is beyond the %d devices the static workspace tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(EIK_EDEVICE, "no device address for the static workspace on device %d", dev);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return EIK_OK;
}

// Workspace of the soft-min mode: grid descriptors, per-grid iteration state
// (scale, done flag, cycle count), the bad-source count, source marks, the
// transposed parameters, and for the adjoint the incoming weights in both
// layouts, the parameter partials, the transposed dL/dT and lambda.
constexpr int kSoftCheck = 4; // cycles between host checks, one launch
struct SoftLayout {
    size_t descs, scale, done, cycles, bad, mark, Pt, win, wint, dth, gt, lam, total;
};

SoftLayout soft_layout(int n_grids, int64_t n, int dtype)
{
    const size_t rs = dtype == EIK_F64 ? 8 : 4;
    SoftLayout L;
    size_t o = 0;
    L.descs = o;  o += align256((size_t)n_grids * kSoftDescBytes);
    L.scale = o;  o += align256((size_t)n_grids * rs);
    L.done = o;   o += align256((size_t)n_grids * 4);
    L.cycles = o; o += align256((size_t)n_grids * 4);
    L.bad = o;    o += align256(4);
    L.mark = o;   o += align256((size_t)n);
    L.Pt = o;     o += align256(5 * (size_t)n * rs);
    L.win = o;    o += align256(8 * (size_t)n * rs);
    L.wint = o;   o += align256(8 * (size_t)n * rs);
    L.dth = o;    o += align256(5 * (size_t)n * rs);
    L.gt = o;     o += align256((size_t)n * rs);
    L.lam = o;    o += align256((size_t)n * rs);
    L.total = o;
    return L;
}

int soft_extent(int n_grids, const eik_grid *grids, int dtype, int64_t &n, int64_t &max_n, int64_t &n_src)
{
    if (!grids || n_grids < 1) return fail(EIK_EINVAL, "no grids");
    if (dtype != EIK_F32 && dtype != EIK_F64) return fail(EIK_EINVAL, "dtype %d", dtype);
    n = max_n = n_src = 0;
    for (int g = 0; g < n_grids; ++g) {
        int rc = check_one(&grids[g], g);
        if (rc) return rc;
        if (grids[g].nx > kSoftMaxLine || grids[g].ny > kSoftMaxLine)
            return fail(EIK_EINVAL, "grid %d: soft-min mode takes sides up to %d nodes, got %d x %d", g, kSoftMaxLine,
                        grids[g].nx, grids[g].ny);
        const int64_t m = (int64_t)grids[g].nx * grids[g].ny;
        n += m;
        max_n = std::max(max_n, m);
        n_src += grids[g].n_src;
    }
    if (n_src >= ((int64_t)1 << 31)) return fail(EIK_EINVAL, "too many sources");
    return EIK_OK;
}

int soft_check(int n_grids, const eik_grid *grids, int dtype, const int32_t *src, double tau, double tol,
               int max_cycles, const void *ws, size_t ws_bytes, int64_t &n, int64_t &max_n)
{
    int64_t n_src;
    int rc = soft_extent(n_grids, grids, dtype, n, max_n, n_src);
    if (rc) return rc;
    if (!src) return fail(EIK_EINVAL, "src_idx is NULL");
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(EIK_EINVAL, "tau must be positive and finite");
    if (!(tol >= 0.0)) return fail(EIK_EINVAL, "tol must be >= 0");
    if (max_cycles < 1) return fail(EIK_EINVAL, "max_cycles must be >= 1");
    const size_t need = soft_layout(n_grids, n, dtype).total;
    if (!ws || ws_bytes < need) return fail(EIK_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    return EIK_OK;
}

// Carves the workspace and uploads the grid descriptors.
int soft_batch(int n_grids, const eik_grid *grids, int dtype, int64_t n, int64_t max_n, void *ws, SoftBatch &b,
               hipStream_t st)
{
    const SoftLayout L = soft_layout(n_grids, n, dtype);
    char *w = (char *)ws;
    b.n_grids = n_grids;
    b.n_nodes = n;
    b.max_nodes = max_n;
    b.descs = w + L.descs;
    b.scale = w + L.scale;
    b.done = (int32_t *)(w + L.done);
    b.cycles = (int32_t *)(w + L.cycles);
    b.bad = (int32_t *)(w + L.bad);
    b.mark = (uint8_t *)(w + L.mark);
    b.Pt = w + L.Pt;
    b.win = w + L.win;
    b.wint = w + L.wint;
    b.dth = w + L.dth;
    b.gt = w + L.gt;
    b.lam = w + L.lam;
    std::vector<unsigned char> d((size_t)n_grids * kSoftDescBytes);
    int64_t off = 0;
    int32_t sb = 0;
    b.max_line = b.max_rows = b.max_cols = 1;
    for (int g = 0; g < n_grids; ++g) {
        b.max_line = std::max({b.max_line, grids[g].nx, grids[g].ny});
        b.max_rows = std::max(b.max_rows, grids[g].ny);
        b.max_cols = std::max(b.max_cols, grids[g].nx);
        write_soft_desc(off, grids[g].h, grids[g].nx, grids[g].ny, grids[g].n_src, sb, d.data() + g * kSoftDescBytes);
        off += (int64_t)grids[g].nx * grids[g].ny;
        sb += grids[g].n_src;
    }
    HIP_OK(hipMemcpyAsync(b.descs, d.data(), d.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
    return EIK_OK;
}

// Runs cycles in launches of up to kSoftCheck (cycle(k) enqueues one) until
// every grid is done or max_cycles have run; the bad-source count is read with
// the first launch.
// cycles_out (n_grids, may be NULL) receives each grid's cycles.
template <typename F>
int soft_cycles(const SoftBatch &b, int max_cycles, hipStream_t st, F &&cycle, int32_t *cycles_out,
                double *cycle_ms, bool &conv, bool &bad_src)
{
    conv = false;
    bad_src = false;
    std::vector<int32_t> done(b.n_grids);
    LaunchTimer timer;
    int rc = timer.init(cycle_ms != nullptr);
    if (rc) return rc;
    int run = 0;
    while (run < max_cycles && !conv) {
        const int k = std::min(kSoftCheck, max_cycles - run);
        timer.before(st);
        cycle(k);
        timer.after(st);
        HIP_OK(hipGetLastError());
        run += k;
        int32_t bad = 0;
        HIP_OK(hipMemcpyAsync(done.data(), b.done, done.size() * 4, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(&bad, b.bad, 4, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        timer.collect();
        if (bad) {
            bad_src = true;
            break;
        }
        conv = std::all_of(done.begin(), done.end(), [](int32_t x) { return x != 0; });
    }
    if (cycles_out) {
        HIP_OK(hipMemcpyAsync(cycles_out, b.cycles, (size_t)b.n_grids * 4, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
    }
    if (cycle_ms) *cycle_ms = timer.ms;
    return EIK_OK;
}

template <typename R>
int soft_forward_impl(int n_grids, const eik_grid *grids, const int32_t *src, const void *src_t, const void *M,
                      const void *om, double tau, double tol, int max_cycles, void *T, void *ws, int64_t n,
                      int64_t max_n, int32_t *cycles_out, double *cycle_ms, hipStream_t st)
{
    SoftBatch b;
    int rc = soft_batch(n_grids, grids, sizeof(R) == 8 ? EIK_F64 : EIK_F32, n, max_n, ws, b, st);
    if (rc) return rc;
    launch_soft_init<R>(b, src, src_t, T, M, om, st);
    bool conv, bad;
    rc = soft_cycles(
        b, max_cycles, st, [&](int k) { launch_soft_cycles<R>(b, M, om, T, tau, tol, k, st); }, cycles_out, cycle_ms,
        conv, bad);
    if (rc) return rc;
    if (bad) return fail(EIK_EINVAL, "a source index is outside its grid");
    return conv ? EIK_OK : fail(EIK_NOT_CONVERGED, "a grid had no quiet cycle within %d cycles", max_cycles);
}

template <typename R>
int soft_backward_impl(int n_grids, const eik_grid *grids, const int32_t *src, const void *M, const void *om,
                       const void *T, double tau, const void *gT, double tol, int max_cycles, void *dM, void *dom,
                       void *dsrc, void *ws, int64_t n, int64_t max_n, int32_t *cycles_out, double *cycle_ms,
                       hipStream_t st)
{
    SoftBatch b;
    int rc = soft_batch(n_grids, grids, sizeof(R) == 8 ? EIK_F64 : EIK_F32, n, max_n, ws, b, st);
    if (rc) return rc;
    launch_soft_init<R>(b, src, nullptr, nullptr, nullptr, nullptr, st);
    launch_soft_coef<R>(b, M, om, T, gT, tau, st);
    bool conv, bad;
    rc = soft_cycles(
        b, max_cycles, st, [&](int k) { launch_soft_adj_cycles<R>(b, gT, T, tol, k, st); }, cycles_out, cycle_ms,
        conv, bad);
    if (rc) return rc;
    if (bad) return fail(EIK_EINVAL, "a source index is outside its grid");
    launch_soft_params<R>(b, src, dM, dom, dsrc, st);
    HIP_OK(hipGetLastError());
    return conv ? EIK_OK : fail(EIK_NOT_CONVERGED, "a grid had no quiet adjoint cycle within %d cycles", max_cycles);
}

} // namespace

extern "C" {

size_t eik_workspace_bytes(const eik_grid *grid, int32_t dtype)
{
    if (!grid || !grid->src_idx) return 0;
    Extent e;
    if (extent_of(1, grid, dtype, e)) return 0;
    return layout(e, dtype).total;
}

size_t eik_batch_workspace_bytes(int32_t n_grids, const eik_grid *grids, int32_t dtype)
{
    Extent e;
    if (dtype == EIK_MIXED) {
        if (extent_of(n_grids, grids, EIK_F64, e)) return 0;
        return mixed_layout(e).total;
    }
    if (extent_of(n_grids, grids, dtype, e)) return 0;
    return layout(e, dtype).total;
}

int eik_batch_plan(int32_t n_grids, const eik_grid *grids, int32_t dtype, const eik_tuning *tuning, void *ws,
                   size_t ws_bytes, hipStream_t stream)
{
    if (dtype == EIK_MIXED) { // the FP64 workspace behind the FP32 copies holds the plan of both phases
        Extent e;
        int rc = extent_of(n_grids, grids, EIK_F64, e);
        if (rc) return rc;
        const MixedLayout L = mixed_layout(e);
        if (!ws || ws_bytes < L.total) return fail(EIK_EWORKSPACE, "workspace %zu bytes, %zu needed", ws_bytes, L.total);
        return eik_batch_plan(n_grids, grids, EIK_F64, tuning, (char *)ws + L.base, ws_bytes - L.base, stream);
    }
    const eik_tuning tn = tuning_or_default(tuning);
    Extent e;
    int rc = extent_of(n_grids, grids, dtype, e);
    if (rc) return rc;
    Ws w;
    rc = carve(e, dtype, ws, ws_bytes, w);
    if (rc) return rc;
    std::vector<GridDesc> d;
    std::vector<int32_t> tg;
    host_descs(n_grids, grids, tn.tile_height, d, tg);
    HIP_OK(hipMemcpyAsync(w.descs, d.data(), d.size() * sizeof(GridDesc), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(w.tile_grid, tg.data(), tg.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIP_OK(hipStreamSynchronize(stream));
    return EIK_OK;
}

int eik_forward(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, const void *T_init,
                double tol, int32_t max_rounds, int32_t flags, void *T, uint8_t *parent, int32_t *level, void *ws,
                size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats, hipStream_t stream)
{
    if (!grid) return fail(EIK_EINVAL, "grid is NULL");
    if (dtype != EIK_F32 && dtype != EIK_F64) return fail(EIK_EINVAL, "dtype %d", dtype);
    int rc = check_one(grid, 0);
    if (rc) return rc;
    if (!grid->src_idx) return fail(EIK_EINVAL, "src_idx is NULL");
    rc = check_ptrs(M, omega, T, parent);
    if (rc) return rc;
    if (!(tol >= 0.0)) return fail(EIK_EINVAL, "tol must be >= 0");
    if (max_rounds < 1) return fail(EIK_EINVAL, "max_rounds must be >= 1");
    if (dtype == EIK_F64)
        return forward_impl<double>(1, grid, grid->src_idx, grid->src_t, M, omega, T_init, tol, max_rounds, flags, T,
                                    parent, level, ws, ws_bytes, tuning, stats, true, stream);
    return forward_impl<float>(1, grid, grid->src_idx, grid->src_t, M, omega, T_init, tol, max_rounds, flags, T,
                               parent, level, ws, ws_bytes, tuning, stats, true, stream);
}

size_t eik_noalloc_max_workspace_bytes(void) { return kStaticScratchBytes; }

int eik_forward_noalloc(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, const void *T_init,
                        double tol, int32_t max_rounds, int32_t flags, void *T, uint8_t *parent, int32_t *level,
                        const eik_tuning *tuning, eik_stats *stats, hipStream_t stream)
{
    if (!grid) return fail(EIK_EINVAL, "grid is NULL");
    if (dtype != EIK_F32 && dtype != EIK_F64) return fail(EIK_EINVAL, "dtype %d", dtype);
    int rc = check_one(grid, 0);
    if (rc) return rc;
    if (!grid->src_idx) return fail(EIK_EINVAL, "src_idx is NULL");
    rc = check_ptrs(M, omega, T, parent);
    if (rc) return rc;
    if (!(tol >= 0.0)) return fail(EIK_EINVAL, "tol must be >= 0");
    if (max_rounds < 1) return fail(EIK_EINVAL, "max_rounds must be >= 1");
    if (flags & EIK_TIME_KERNELS) return fail(EIK_EINVAL, "EIK_TIME_KERNELS creates events; not available here");
    Extent e;
    rc = extent_of(1, grid, dtype, e);
    if (rc) return rc;
    const size_t need = layout(e, dtype).total;
    if (need > kStaticScratchBytes)
        return fail(EIK_EWORKSPACE, "a %d x %d grid needs %zu bytes of workspace; the static workspace holds %zu",
                    grid->nx, grid->ny, need, kStaticScratchBytes);
    void *ws = nullptr;
    rc = static_scratch(&ws);
    if (rc) return rc;
    if (dtype == EIK_F64)
        return forward_impl<double>(1, grid, grid->src_idx, grid->src_t, M, omega, T_init, tol, max_rounds, flags, T,
                                    parent, level, ws, kStaticScratchBytes, tuning, stats, true, stream);
    return forward_impl<float>(1, grid, grid->src_idx, grid->src_t, M, omega, T_init, tol, max_rounds, flags, T,
                               parent, level, ws, kStaticScratchBytes, tuning, stats, true, stream);
}

size_t eik_mixed_workspace_bytes(const eik_grid *grid)
{
    if (!grid || !grid->src_idx) return 0;
    Extent e;
    if (extent_of(1, grid, EIK_F64, e)) return 0;
    return mixed_layout(e, true).total;
}

int eik_forward_mixed(const eik_grid *grid, const double *M, const double *omega, double tol32, double tol,
                      int32_t max_rounds, int32_t flags, double *T, uint8_t *parent, int32_t *level, void *ws,
                      size_t ws_bytes, const eik_tuning *tuning32, const eik_tuning *tuning, eik_stats *stats,
                      hipStream_t stream)
{
    if (!grid) return fail(EIK_EINVAL, "grid is NULL");
    int rc = check_one(grid, 0);
    if (rc) return rc;
    if (!grid->src_idx) return fail(EIK_EINVAL, "src_idx is NULL");
    rc = check_ptrs(M, omega, T, parent);
    if (rc) return rc;
    if (!(tol >= 0.0) || !(tol32 >= 0.0)) return fail(EIK_EINVAL, "tolerances must be >= 0");
    if (max_rounds < 1) return fail(EIK_EINVAL, "max_rounds must be >= 1");
    Extent e;
    rc = extent_of(1, grid, EIK_F64, e);
    if (rc) return rc;
    const MixedLayout L = mixed_layout(e, true);
    if (!ws || ws_bytes < L.total)
        return fail(EIK_EWORKSPACE, "workspace %zu bytes, %zu needed", ws_bytes, L.total);
    char *b = (char *)ws;
    float *M32 = (float *)(b + L.M32), *om32 = (float *)(b + L.om32), *T32 = (float *)(b + L.T32);
    // The FP64 phase's staged inputs (parameters and metric roots) depend on
    // M and omega only: they are staged on the side stream while the FP32
    // sweeps run (forked once the FP32 phase's own passes over the grid are
    // enqueued, which it would otherwise slow down), in the FP64 workspace,
    // which the FP32 phase does not touch.
    const eik_tuning tn64 = tuning_or_default(tuning);
    hipStream_t side = nullptr;
    rc = side_stream(stream, side);
    if (rc) return rc;
    ForkEvents ev;
    HIP_OK(hipEventCreateWithFlags(&ev.fork, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&ev.join, hipEventDisableTiming));
    bool forked = false;
    auto fork_staging = [&]() -> int {
        HIP_OK(hipEventRecord(ev.fork, stream));
        HIP_OK(hipStreamWaitEvent(side, ev.fork, 0));
        Extent e64;
        Ws w64;
        LaunchArgs a64;
        int r = prepare(1, grid, EIK_F64, b + L.base, L.ws32 - L.base, tn64, true, side, e64, w64, a64);
        if (r) return r;
        launch_stage<double>(a64, M, omega, w64.Pt, side, kSideStageBlocks);
        HIP_OK(hipGetLastError());
        HIP_OK(hipEventRecord(ev.join, side));
        forked = true;
        return EIK_OK;
    };
    // the FP32 copies of M and omega: made by the FP32 staging itself, unless
    // the feasibility check must read them before it
    const bool fused = !(flags & EIK_CHECK_FEASIBLE);
    if (!fused) {
        launch_cast_f64_f32(3 * e.nodes, M, M32, stream);
        launch_cast_f64_f32(2 * e.nodes, omega, om32, stream);
    }
    eik_grid g32 = *grid;
    if (grid->src_t) {
        g32.src_t = b + L.src32;
        launch_cast_f64_f32(grid->n_src, (const double *)grid->src_t, (float *)(b + L.src32), stream);
    }
    HIP_OK(hipGetLastError());
    // FP32 sweeps from the cold start; not reaching tol32 is no error here
    rc = forward_impl<float>(1, &g32, g32.src_idx, g32.src_t, M32, om32, nullptr, tol32, max_rounds, flags, T32,
                             parent, nullptr, b + L.ws32, ws_bytes - L.ws32, tuning32, stats, true, stream,
                             /*certify=*/false, /*pre_staged=*/false, fork_staging, -1, fused ? M : nullptr,
                             fused ? omega : nullptr);
    if (forked) HIP_OK(hipStreamWaitEvent(stream, ev.join, 0)); // joined before any return: the side work ends in order
    if (rc < 0) return rc;
    if (!forked) return fail(EIK_EDEVICE, "the FP64 staging was not enqueued");
    // FP64 sweeps from that field, in place in T
    launch_cast_f32_f64(e.nodes, T32, T, stream);
    HIP_OK(hipGetLastError());
    return forward_impl<double>(1, grid, grid->src_idx, grid->src_t, M, omega, T, tol, max_rounds,
                                flags & ~(EIK_CHECK_FEASIBLE | EIK_WARM_FALLBACK), T, parent, level, b + L.base,
                                L.ws32 - L.base, tuning, stats ? stats + 1 : nullptr, true, stream,
                                /*certify=*/true, /*pre_staged=*/true, nullptr,
                                /*full_first_batch=*/0); // no early check: the FP32 field is not within tol
}

int eik_forward_batched(int32_t n_grids, const eik_grid *grids, int32_t dtype, const int32_t *src_idx,
                        const void *src_t, const void *M, const void *omega, const void *T_init, double tol,
                        int32_t max_rounds, int32_t flags, void *T, uint8_t *parent, int32_t *level, void *ws,
                        size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats, hipStream_t stream)
{
    if (!src_idx) return fail(EIK_EINVAL, "src_idx is NULL");
    int rc = check_ptrs(M, omega, T, parent);
    if (rc) return rc;
    if (!(tol >= 0.0)) return fail(EIK_EINVAL, "tol must be >= 0");
    if (max_rounds < 1) return fail(EIK_EINVAL, "max_rounds must be >= 1");
    if (dtype == EIK_F64)
        return forward_impl<double>(n_grids, grids, src_idx, src_t, M, omega, T_init, tol, max_rounds, flags, T,
                                    parent, level, ws, ws_bytes, tuning, stats, false, stream);
    if (dtype == EIK_F32)
        return forward_impl<float>(n_grids, grids, src_idx, src_t, M, omega, T_init, tol, max_rounds, flags, T,
                                   parent, level, ws, ws_bytes, tuning, stats, false, stream);
    return fail(EIK_EINVAL, "dtype %d", dtype);
}

int eik_forward_batched_mixed(int32_t n_grids, const eik_grid *grids, const int32_t *src_idx, const double *src_t,
                              const double *M, const double *omega, double tol32, double tol, int32_t max_rounds,
                              int32_t flags, double *T, uint8_t *parent, int32_t *level, void *ws, size_t ws_bytes,
                              const eik_tuning *tuning32, const eik_tuning *tuning, eik_stats *stats,
                              hipStream_t stream)
{
    if (!src_idx) return fail(EIK_EINVAL, "src_idx is NULL");
    int rc = check_ptrs(M, omega, T, parent);
    if (rc) return rc;
    if (!(tol >= 0.0) || !(tol32 >= 0.0)) return fail(EIK_EINVAL, "tolerances must be >= 0");
    if (max_rounds < 1) return fail(EIK_EINVAL, "max_rounds must be >= 1");
    if (tuning_or_default(tuning32).tile_height != tuning_or_default(tuning).tile_height)
        return fail(EIK_EINVAL, "both phases must use the tile height of the plan");
    Extent e;
    rc = extent_of(n_grids, grids, EIK_F64, e);
    if (rc) return rc;
    const MixedLayout L = mixed_layout(e);
    if (!ws || ws_bytes < L.total) return fail(EIK_EWORKSPACE, "workspace %zu bytes, %zu needed", ws_bytes, L.total);
    char *b = (char *)ws;
    float *M32 = (float *)(b + L.M32), *om32 = (float *)(b + L.om32), *T32 = (float *)(b + L.T32);
    float *src32 = src_t ? (float *)(b + L.src32) : nullptr;
    // the FP32 copies of M and omega are made by the FP32 staging itself,
    // unless the feasibility check must read them before it
    const bool fused = !(flags & EIK_CHECK_FEASIBLE);
    if (!fused) {
        launch_cast_f64_f32(3 * e.nodes, M, M32, stream);
        launch_cast_f64_f32(2 * e.nodes, omega, om32, stream);
    }
    if (src_t) launch_cast_f64_f32(e.n_src, src_t, src32, stream);
    HIP_OK(hipGetLastError());
    // FP32 sweeps from the cold start (not reaching tol32 is no error here),
    // then FP64 sweeps from that field in place in T
    rc = forward_impl<float>(n_grids, grids, src_idx, src32, M32, om32, nullptr, tol32, max_rounds, flags, T32,
                             parent, nullptr, b + L.base, ws_bytes - L.base, tuning32, stats, false, stream,
                             /*certify=*/false, /*pre_staged=*/false, nullptr, -1, fused ? M : nullptr,
                             fused ? omega : nullptr);
    if (rc < 0) return rc;
    launch_cast_f32_f64(e.nodes, T32, T, stream);
    HIP_OK(hipGetLastError());
    return forward_impl<double>(n_grids, grids, src_idx, src_t, M, omega, T, tol, max_rounds,
                                flags & ~(EIK_CHECK_FEASIBLE | EIK_WARM_FALLBACK), T, parent, level, b + L.base,
                                ws_bytes - L.base, tuning, stats ? stats + 1 : nullptr, false, stream);
}

int eik_backward_batched_mixed(int32_t n_grids, const eik_grid *grids, const int32_t *src_idx, const double *M,
                               const double *omega, const double *T, const uint8_t *parent, const int32_t *level,
                               const double *dLdT, double *dLdM, double *dLdomega, double *dLdsrc, void *ws,
                               size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats, hipStream_t stream)
{
    if (!src_idx || !M || !omega || !T || !parent || !dLdT || !dLdM || !dLdomega || !dLdsrc)
        return fail(EIK_EINVAL, "NULL pointer argument");
    Extent e;
    int rc = extent_of(n_grids, grids, EIK_F64, e);
    if (rc) return rc;
    const MixedLayout L = mixed_layout(e);
    if (!ws || ws_bytes < L.total) return fail(EIK_EWORKSPACE, "workspace %zu bytes, %zu needed", ws_bytes, L.total);
    char *b = (char *)ws;
    const Relax32 r32 = {(float *)(b + L.M32), (float *)(b + L.om32), (float *)(b + L.T32)};
    return backward_impl<double>(n_grids, grids, src_idx, M, omega, T, parent, level, dLdT, dLdM, dLdomega, dLdsrc,
                                 b + L.base, ws_bytes - L.base, tuning, false, stats, stream, &r32);
}

int eik_backward(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, const void *T,
                 const uint8_t *parent, const int32_t *level, const void *dLdT, void *dLdM, void *dLdomega,
                 void *dLdsrc, void *ws, size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats,
                 hipStream_t stream)
{
    if (!grid) return fail(EIK_EINVAL, "grid is NULL");
    if (dtype != EIK_F32 && dtype != EIK_F64) return fail(EIK_EINVAL, "dtype %d", dtype);
    int rc = check_one(grid, 0);
    if (rc) return rc;
    if (!grid->src_idx) return fail(EIK_EINVAL, "src_idx is NULL");
    if (!M || !omega || !T || !parent || !dLdT || !dLdM || !dLdomega || !dLdsrc)
        return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        return backward_impl<double>(1, grid, grid->src_idx, M, omega, T, parent, level, dLdT, dLdM, dLdomega,
                                     dLdsrc, ws, ws_bytes, tuning, true, stats, stream);
    return backward_impl<float>(1, grid, grid->src_idx, M, omega, T, parent, level, dLdT, dLdM, dLdomega, dLdsrc,
                                ws, ws_bytes, tuning, true, stats, stream);
}

int eik_backward_mixed(const eik_grid *grid, const double *M, const double *omega, const double *T,
                       const uint8_t *parent, const int32_t *level, const double *dLdT, double *dLdM,
                       double *dLdomega, double *dLdsrc, void *ws, size_t ws_bytes, const eik_tuning *tuning,
                       eik_stats *stats, hipStream_t stream)
{
    if (!grid) return fail(EIK_EINVAL, "grid is NULL");
    int rc = check_one(grid, 0);
    if (rc) return rc;
    if (!grid->src_idx) return fail(EIK_EINVAL, "src_idx is NULL");
    if (!M || !omega || !T || !parent || !dLdT || !dLdM || !dLdomega || !dLdsrc)
        return fail(EIK_EINVAL, "NULL pointer argument");
    Extent e;
    rc = extent_of(1, grid, EIK_F64, e);
    if (rc) return rc;
    const MixedLayout L = mixed_layout(e);
    if (!ws || ws_bytes < L.total)
        return fail(EIK_EWORKSPACE, "workspace %zu bytes, %zu needed", ws_bytes, L.total);
    char *b = (char *)ws;
    const Relax32 r32 = {(float *)(b + L.M32), (float *)(b + L.om32), (float *)(b + L.T32)};
    return backward_impl<double>(1, grid, grid->src_idx, M, omega, T, parent, level, dLdT, dLdM, dLdomega, dLdsrc,
                                 b + L.base, ws_bytes - L.base, tuning, true, stats, stream, &r32);
}

int eik_backward_batched(int32_t n_grids, const eik_grid *grids, int32_t dtype, const int32_t *src_idx,
                         const void *M, const void *omega, const void *T, const uint8_t *parent,
                         const int32_t *level, const void *dLdT, void *dLdM, void *dLdomega, void *dLdsrc, void *ws,
                         size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats, hipStream_t stream)
{
    if (!src_idx || !M || !omega || !T || !parent || !dLdT || !dLdM || !dLdomega || !dLdsrc)
        return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        return backward_impl<double>(n_grids, grids, src_idx, M, omega, T, parent, level, dLdT, dLdM, dLdomega,
                                     dLdsrc, ws, ws_bytes, tuning, false, stats, stream);
    if (dtype == EIK_F32)
        return backward_impl<float>(n_grids, grids, src_idx, M, omega, T, parent, level, dLdT, dLdM, dLdomega,
                                    dLdsrc, ws, ws_bytes, tuning, false, stats, stream);
    return fail(EIK_EINVAL, "dtype %d", dtype);
}

int eik_project(int64_t n, int32_t dtype, const void *M_in, const void *omega_in, void *M_out, void *omega_out,
                const eik_project_params *p, hipStream_t stream)
{
    if (n < 0) return fail(EIK_EINVAL, "n < 0");
    if (n == 0) return EIK_OK;
    if (!M_in || !omega_in || !M_out || !omega_out) return fail(EIK_EINVAL, "NULL pointer argument");
    eik_project_params d = {1e-3, 1e3, 1e3, 0.95};
    if (p) d = *p;
    if (!(d.eig_min > 0 && d.eig_max >= d.eig_min && d.eucl_clip > 0 && d.rho_max > 0 && d.rho_max < 1))
        return fail(EIK_EINVAL, "projection parameters out of range");
    if (dtype == EIK_F64)
        launch_project<double>(n, M_in, omega_in, M_out, omega_out, d.eig_min, d.eig_max, d.eucl_clip, d.rho_max,
                               stream);
    else if (dtype == EIK_F32)
        launch_project<float>(n, M_in, omega_in, M_out, omega_out, d.eig_min, d.eig_max, d.eucl_clip, d.rho_max,
                              stream);
    else
        return fail(EIK_EINVAL, "dtype %d", dtype);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

int eik_project_backward(int64_t n, int32_t dtype, const void *M_in, const void *omega_in, const void *gM_out,
                         const void *gomega_out, void *gM_in, void *gomega_in, const eik_project_params *p,
                         hipStream_t stream)
{
    if (n < 0) return fail(EIK_EINVAL, "n < 0");
    if (n == 0) return EIK_OK;
    if (!M_in || !omega_in || !gM_out || !gomega_out || !gM_in || !gomega_in)
        return fail(EIK_EINVAL, "NULL pointer argument");
    eik_project_params d = {1e-3, 1e3, 1e3, 0.95};
    if (p) d = *p;
    if (!(d.eig_min > 0 && d.eig_max >= d.eig_min && d.eucl_clip > 0 && d.rho_max > 0 && d.rho_max < 1))
        return fail(EIK_EINVAL, "projection parameters out of range");
    if (dtype == EIK_F64)
        launch_project_backward<double>(n, M_in, omega_in, gM_out, gomega_out, gM_in, gomega_in, d.eig_min,
                                        d.eig_max, d.eucl_clip, d.rho_max, stream);
    else if (dtype == EIK_F32)
        launch_project_backward<float>(n, M_in, omega_in, gM_out, gomega_out, gM_in, gomega_in, d.eig_min,
                                       d.eig_max, d.eucl_clip, d.rho_max, stream);
    else
        return fail(EIK_EINVAL, "dtype %d", dtype);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

int eik_batch_pending(int32_t n_grids, const eik_grid *grids, int32_t dtype, const void *ws, size_t ws_bytes,
                      int64_t pending[3], hipStream_t stream)
{
    if (!pending) return fail(EIK_EINVAL, "pending is NULL");
    if (dtype == EIK_MIXED) {
        Extent e;
        int rc = extent_of(n_grids, grids, EIK_F64, e);
        if (rc) return rc;
        const MixedLayout L = mixed_layout(e);
        if (!ws || ws_bytes < L.total) return fail(EIK_EWORKSPACE, "workspace %zu bytes, %zu needed", ws_bytes, L.total);
        return eik_batch_pending(n_grids, grids, EIK_F64, (const char *)ws + L.base, ws_bytes - L.base, pending,
                                 stream);
    }
    Extent e;
    int rc = extent_of(n_grids, grids, dtype, e);
    if (rc) return rc;
    Ws w;
    rc = carve(e, dtype, const_cast<void *>(ws), ws_bytes, w);
    if (rc) return rc;
    unsigned long long c[3]; // sweep, level, adjoint
    HIP_OK(hipMemcpyAsync(c, w.ctr + kCtrSweepPending, sizeof c, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    for (int k = 0; k < 3; ++k) pending[k] = (int64_t)c[k];
    return EIK_OK;
}

size_t eik_inv_scratch_bytes(void) { return (size_t)kInvBlocks * sizeof(double); }

int eik_tv(int32_t nx, int32_t ny, int32_t n_planes, int32_t dtype, const void *F, const double *weights,
           double scale, void *grad, double *value, void *scratch, hipStream_t stream)
{
    if (nx < 1 || ny < 1 || n_planes < 1 || n_planes > 4) return fail(EIK_EINVAL, "sizes %d x %d x %d", nx, ny, n_planes);
    if ((int64_t)nx * ny >= ((int64_t)1 << 40)) return fail(EIK_EINVAL, "field too large");
    if (!F || !weights || !grad || !value || !scratch) return fail(EIK_EINVAL, "NULL pointer argument");
    for (int c = 0; c < n_planes; ++c)
        if (!(weights[c] >= 0.0)) return fail(EIK_EINVAL, "plane weight %d is negative", c);
    if (dtype == EIK_F64)
        launch_tv<double>(nx, ny, n_planes, F, weights, scale, grad, value, (double *)scratch, stream);
    else if (dtype == EIK_F32)
        launch_tv<float>(nx, ny, n_planes, F, weights, scale, grad, value, (double *)scratch, stream);
    else
        return fail(EIK_EINVAL, "dtype %d", dtype);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

size_t eik_tv_log_euclid_work_bytes(int32_t nx, int32_t ny, int32_t dtype)
{
    if (nx < 1 || ny < 1 || (dtype != EIK_F32 && dtype != EIK_F64)) return 0;
    return 6 * (size_t)nx * (size_t)ny * (dtype == EIK_F64 ? 8 : 4);
}

int eik_tv_log_euclid(int32_t nx, int32_t ny, int32_t dtype, const void *M, double scale, void *grad,
                      double *value, void *work, void *scratch, hipStream_t stream)
{
    if (nx < 1 || ny < 1) return fail(EIK_EINVAL, "sizes %d x %d", nx, ny);
    if ((int64_t)nx * ny >= ((int64_t)1 << 40)) return fail(EIK_EINVAL, "field too large");
    if (!M || !grad || !value || !work || !scratch) return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        launch_tv_log_euclid<double>(nx, ny, M, scale, grad, value, work, (double *)scratch, stream);
    else if (dtype == EIK_F32)
        launch_tv_log_euclid<float>(nx, ny, M, scale, grad, value, work, (double *)scratch, stream);
    else
        return fail(EIK_EINVAL, "dtype %d", dtype);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

int eik_obs_loss(int64_t n, int32_t dtype, const void *T, const void *T_obs, const uint8_t *mask, void *dLdT,
                 double *value, void *scratch, hipStream_t stream)
{
    if (n < 1) return fail(EIK_EINVAL, "n < 1");
    if (!T || !T_obs || !mask || !dLdT || !value || !scratch) return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        launch_obs_loss<double>(n, T, T_obs, mask, dLdT, value, (double *)scratch, stream);
    else if (dtype == EIK_F32)
        launch_obs_loss<float>(n, T, T_obs, mask, dLdT, value, (double *)scratch, stream);
    else
        return fail(EIK_EINVAL, "dtype %d", dtype);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

int eik_sum_sq(int64_t n, int32_t dtype, const void *x, double *acc, void *scratch, hipStream_t stream)
{
    if (n < 1) return fail(EIK_EINVAL, "n < 1");
    if (!x || !acc || !scratch) return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        launch_sum_sq<double>(n, x, acc, (double *)scratch, stream);
    else if (dtype == EIK_F32)
        launch_sum_sq<float>(n, x, acc, (double *)scratch, stream);
    else
        return fail(EIK_EINVAL, "dtype %d", dtype);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

int eik_param_step(int64_t n, int32_t dtype, int32_t method, void *p, const void *g, void *m, void *v, double lr,
                   double beta1, double beta2, double eps, int32_t t, double max_norm, const double *grad_sq,
                   hipStream_t stream)
{
    if (n < 1) return fail(EIK_EINVAL, "n < 1");
    if (method != 0 && method != 1) return fail(EIK_EINVAL, "method %d", method);
    if (!p || !g) return fail(EIK_EINVAL, "NULL pointer argument");
    if (method == 1 && (!m || !v || t < 1 || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps >= 0)))
        return fail(EIK_EINVAL, "Adam needs state arrays, t >= 1, betas in [0, 1) and eps >= 0");
    if (max_norm > 0 && !grad_sq) return fail(EIK_EINVAL, "clipping needs grad_sq");
    if (dtype == EIK_F64)
        launch_param_step<double>(n, method, p, g, m, v, lr, beta1, beta2, eps, t, max_norm, grad_sq, stream);
    else if (dtype == EIK_F32)
        launch_param_step<float>(n, method, p, g, m, v, lr, beta1, beta2, eps, t, max_norm, grad_sq, stream);
    else
        return fail(EIK_EINVAL, "dtype %d", dtype);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

int eik_tie_isotropic(int64_t n, int32_t dtype, void *M, hipStream_t stream)
{
    if (n < 1) return fail(EIK_EINVAL, "n < 1");
    if (!M) return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        launch_tie_isotropic<double>(n, M, stream);
    else if (dtype == EIK_F32)
        launch_tie_isotropic<float>(n, M, stream);
    else
        return fail(EIK_EINVAL, "dtype %d", dtype);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

// ---------------------------------------------------------------------------
// Covariate encoder (include/eik_encoder.h)

int eik_enc_dense(int32_t B, int32_t Cin, int32_t Cout, const float *x, const float *W, const float *b, int32_t relu,
                  float *y, hipStream_t stream)
{
    if (B < 1 || Cin < 1 || Cout < 1 || (int64_t)B * Cout > (1 << 24)) return fail(EIK_EINVAL, "dense sizes");
    if (!x || !W || !y) return fail(EIK_EINVAL, "NULL pointer argument");
    launch_enc_dense(B, Cin, Cout, x, W, b, relu, y, stream);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

int eik_enc_dense_backward(int32_t B, int32_t Cin, int32_t Cout, const float *x, const float *W, const float *y,
                           int32_t relu, const float *dy, float *dx, float *dW, float *db, hipStream_t stream)
{
    if (B < 1 || Cin < 1 || Cout < 1 || (int64_t)B * Cin > (1 << 24) || (int64_t)Cout * (Cin + 1) > (1 << 24))
        return fail(EIK_EINVAL, "dense sizes");
    if (!x || !W || !y || !dy || !dW) return fail(EIK_EINVAL, "NULL pointer argument");
    launch_enc_dense_backward(B, Cin, Cout, x, W, y, relu, dy, dx, dW, db, stream);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

int eik_enc_combine(int32_t B, int64_t n, int32_t dtype, double alpha, const float *base, const float *local,
                    void *M, void *omega, hipStream_t stream)
{
    if (B < 1 || B > kEncMaxScenes || n < 1) return fail(EIK_EINVAL, "B = %d, n = %lld", B, (long long)n);
    if (!base || !local || !M || !omega) return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        launch_enc_combine<double>(B, n, alpha, base, local, M, omega, stream);
    else if (dtype == EIK_F32)
        launch_enc_combine<float>(B, n, alpha, base, local, M, omega, stream);
    else
        return fail(EIK_EINVAL, "dtype %d", dtype);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

size_t eik_enc_scratch_bytes(int32_t B)
{
    if (B < 1 || B > kEncMaxScenes) return 0;
    return sizeof(double) * (size_t)kEncPlanes * (size_t)B * kInvBlocks;
}

int eik_enc_combine_backward(int32_t B, int64_t n, int32_t dtype, double alpha, const void *dM, const void *domega,
                             float *dlocal, float *dbase, void *scratch, hipStream_t stream)
{
    if (B < 1 || B > kEncMaxScenes || n < 1) return fail(EIK_EINVAL, "B = %d, n = %lld", B, (long long)n);
    if (!dM || !domega || !dlocal || !dbase || !scratch) return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        launch_enc_combine_backward<double>(B, n, alpha, dM, domega, dlocal, dbase, (double *)scratch, stream);
    else if (dtype == EIK_F32)
        launch_enc_combine_backward<float>(B, n, alpha, dM, domega, dlocal, dbase, (double *)scratch, stream);
    else
        return fail(EIK_EINVAL, "dtype %d", dtype);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

const char *eik_last_error(void) { return g_last_error.c_str(); }

size_t eik_soft_workspace_bytes(const eik_grid *grid, int32_t dtype)
{
    return eik_soft_batch_workspace_bytes(1, grid, dtype);
}

size_t eik_soft_batch_workspace_bytes(int32_t n_grids, const eik_grid *grids, int32_t dtype)
{
    if (!grids || n_grids < 1 || (dtype != EIK_F32 && dtype != EIK_F64)) return 0;
    int64_t n = 0;
    for (int g = 0; g < n_grids; ++g) {
        if (grids[g].nx < 1 || grids[g].ny < 1) return 0;
        n += (int64_t)grids[g].nx * grids[g].ny;
    }
    return soft_layout(n_grids, n, dtype).total;
}

int eik_soft_forward_batched(int32_t n_grids, const eik_grid *grids, int32_t dtype, const int32_t *src_idx,
                             const void *src_t, const void *M, const void *omega, double tau, double tol,
                             int32_t max_cycles, void *T, void *ws, size_t ws_bytes, int32_t *cycles,
                             double *cycle_ms, hipStream_t stream)
{
    int64_t n, max_n;
    int rc = soft_check(n_grids, grids, dtype, src_idx, tau, tol, max_cycles, ws, ws_bytes, n, max_n);
    if (rc) return rc;
    if (!M || !omega || !T) return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        return soft_forward_impl<double>(n_grids, grids, src_idx, src_t, M, omega, tau, tol, max_cycles, T, ws, n,
                                         max_n, cycles, cycle_ms, stream);
    return soft_forward_impl<float>(n_grids, grids, src_idx, src_t, M, omega, tau, tol, max_cycles, T, ws, n, max_n,
                                    cycles, cycle_ms, stream);
}

int eik_soft_backward_batched(int32_t n_grids, const eik_grid *grids, int32_t dtype, const int32_t *src_idx,
                              const void *M, const void *omega, const void *T, double tau, const void *dLdT,
                              double tol, int32_t max_cycles, void *dLdM, void *dLdomega, void *dLdsrc, void *ws,
                              size_t ws_bytes, int32_t *cycles, double *cycle_ms, hipStream_t stream)
{
    int64_t n, max_n;
    int rc = soft_check(n_grids, grids, dtype, src_idx, tau, tol, max_cycles, ws, ws_bytes, n, max_n);
    if (rc) return rc;
    if (!M || !omega || !T || !dLdT || !dLdM || !dLdomega || !dLdsrc) return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        return soft_backward_impl<double>(n_grids, grids, src_idx, M, omega, T, tau, dLdT, tol, max_cycles, dLdM,
                                          dLdomega, dLdsrc, ws, n, max_n, cycles, cycle_ms, stream);
    return soft_backward_impl<float>(n_grids, grids, src_idx, M, omega, T, tau, dLdT, tol, max_cycles, dLdM, dLdomega,
                                     dLdsrc, ws, n, max_n, cycles, cycle_ms, stream);
}

int eik_soft_forward(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, double tau, double tol,
                     int32_t max_cycles, void *T, void *ws, size_t ws_bytes, int32_t *cycles, hipStream_t stream)
{
    if (!grid) return fail(EIK_EINVAL, "grid is NULL");
    return eik_soft_forward_batched(1, grid, dtype, grid->src_idx, grid->src_t, M, omega, tau, tol, max_cycles, T, ws,
                                    ws_bytes, cycles, nullptr, stream);
}

int eik_soft_backward(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, const void *T,
                      double tau, const void *dLdT, double tol, int32_t max_cycles, void *dLdM, void *dLdomega,
                      void *dLdsrc, void *ws, size_t ws_bytes, int32_t *cycles, hipStream_t stream)
{
    if (!grid) return fail(EIK_EINVAL, "grid is NULL");
    return eik_soft_backward_batched(1, grid, dtype, grid->src_idx, M, omega, T, tau, dLdT, tol, max_cycles, dLdM,
                                     dLdomega, dLdsrc, ws, ws_bytes, cycles, nullptr, stream);
}

} // extern "C"
