// eik_api.hip -- the C ABI declared in include/eik.h: argument checks,
// workspace layout, and the order of kernel launches on the caller's stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/eik.h"
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

struct Layout {
    size_t act, act_count, ctr, lam, w1, counts, cursor, list, total;
};

constexpr int kDefaultTH = 64;

GridArgs make_grid(const eik_grid *g, int th)
{
    GridArgs a;
    a.nx = g->nx;
    a.ny = g->ny;
    a.h = g->h;
    a.n_src = g->n_src;
    a.th = th;
    a.ntx = (g->nx + 63) / 64;
    a.nty = (g->ny + th - 1) / th;
    a.n_tiles = a.ntx * a.nty;
    return a;
}

Layout layout(const eik_grid *g, int dtype)
{
    const size_t n = (size_t)g->nx * (size_t)g->ny;
    const size_t rs = dtype == EIK_F64 ? 8 : 4;
    // tile counts for the smallest tile height (largest count)
    const size_t tiles = (size_t)((g->nx + 63) / 64) * (size_t)((g->ny + 31) / 32);
    Layout L;
    size_t o = 0;
    L.act = o;       o += align256(2 * tiles * 4);
    L.act_count = o; o += align256((size_t)(kMaxRounds + 2) * 4);
    L.ctr = o;       o += align256(kCtrCount * 8);
    L.lam = o;       o += align256(n * rs);
    L.w1 = o;        o += align256(n * rs);
    L.counts = o;    o += align256((n + 2) * 4);
    L.cursor = o;    o += align256((n + 2) * 4);
    L.list = o;      o += align256(n * 4);
    L.total = o;
    return L;
}

int check_grid(const eik_grid *g, int dtype)
{
    if (!g) return fail(EIK_EINVAL, "grid is NULL");
    if (g->nx < 1 || g->ny < 1) return fail(EIK_EINVAL, "grid size %d x %d", g->nx, g->ny);
    if ((int64_t)g->nx * g->ny >= ((int64_t)1 << 31)) return fail(EIK_EINVAL, "grid has 2^31 nodes or more");
    if (!(g->h > 0.0)) return fail(EIK_EINVAL, "grid spacing h must be positive");
    if (g->n_src < 1 || !g->src_idx) return fail(EIK_EINVAL, "at least one source index is required");
    if (dtype != EIK_F32 && dtype != EIK_F64) return fail(EIK_EINVAL, "dtype %d", dtype);
    return EIK_OK;
}

struct Ws {
    int32_t *act, *act_count, *counts, *cursor, *list;
    unsigned long long *ctr;
    void *lam, *w1;
};

int carve(const eik_grid *g, int dtype, void *ws, size_t ws_bytes, Ws &w)
{
    const Layout L = layout(g, dtype);
    if (!ws || ws_bytes < L.total)
        return fail(EIK_EWORKSPACE, "workspace %zu bytes, %zu needed", ws_bytes, L.total);
    char *b = (char *)ws;
    w.act = (int32_t *)(b + L.act);
    w.act_count = (int32_t *)(b + L.act_count);
    w.ctr = (unsigned long long *)(b + L.ctr);
    w.lam = b + L.lam;
    w.w1 = b + L.w1;
    w.counts = (int32_t *)(b + L.counts);
    w.cursor = (int32_t *)(b + L.cursor);
    w.list = (int32_t *)(b + L.list);
    return EIK_OK;
}

eik_tuning tuning_or_default(const eik_tuning *t)
{
    eik_tuning d;
    d.max_local_cycles = 4;
    d.rounds_per_check = 8;
    d.adjoint_single_wg_max_cells = 1 << 18;
    if (t) {
        if (t->max_local_cycles >= 1) d.max_local_cycles = t->max_local_cycles;
        if (t->rounds_per_check >= 1) d.rounds_per_check = t->rounds_per_check;
        if (t->adjoint_single_wg_max_cells >= 0) d.adjoint_single_wg_max_cells = t->adjoint_single_wg_max_cells;
    }
    return d;
}

// Run tile rounds until a round flags nothing or max_rounds is reached.
// round_fn(r, act_in, act_out, count_next) enqueues round r.
// Optional per-launch timing with HIP events recorded on the launch stream.
struct LaunchTimer {
    std::vector<hipEvent_t> ev;
    int used = 0;
    double ms = 0.0;
    bool on = false;
    ~LaunchTimer()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    int init(bool enable, int per_batch)
    {
        on = enable;
        if (!on) return EIK_OK;
        ev.resize(2 * per_batch);
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
    // after the stream has been synchronised
    void collect()
    {
        for (int b = 0; b < used; ++b) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[2 * b], ev[2 * b + 1]) == hipSuccess) ms += t;
        }
        used = 0;
    }
};

template <typename F>
int run_rounds(int32_t *act, int32_t *act_count, int n_tiles, int max_rounds, int per_check, hipStream_t st,
               F round_fn, int *rounds_done, bool *converged, LaunchTimer *timer = nullptr)
{
    int r = 0;
    *converged = false;
    while (r < max_rounds) {
        const int batch = std::min(per_check, max_rounds - r);
        for (int b = 0; b < batch; ++b, ++r) {
            if (timer) timer->before(st);
            round_fn(act + (r & 1) * n_tiles, act + ((r + 1) & 1) * n_tiles, act_count + r + 1);
            if (timer) timer->after(st);
        }
        int32_t cnt = 0;
        HIP_OK(hipMemcpyAsync(&cnt, act_count + r, sizeof cnt, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (timer) timer->collect();
        if (cnt == 0) {
            *converged = true;
            break;
        }
    }
    *rounds_done = r;
    return EIK_OK;
}

template <typename R>
int forward_impl(const eik_grid *grid, const void *M, const void *om, const void *T_init, double tol,
                 int max_rounds, int flags, void *T, uint8_t *parent, int32_t *level, void *ws, size_t ws_bytes,
                 const eik_tuning *tun, eik_stats *stats, hipStream_t st)
{
    const int dtype = sizeof(R) == 8 ? EIK_F64 : EIK_F32;
    Ws w;
    int rc = carve(grid, dtype, ws, ws_bytes, w);
    if (rc) return rc;
    const eik_tuning tn = tuning_or_default(tun);
    GridArgs g = make_grid(grid, kDefaultTH);
    const int64_t n = (int64_t)g.nx * g.ny;
    max_rounds = std::max(1, std::min(max_rounds, kMaxRounds));

    launch_fill_u64(w.ctr, kCtrCount, st);
    launch_fill_i32(w.act, 2 * (int64_t)g.n_tiles, 0, st);
    launch_fill_i32(w.act_count, kMaxRounds + 2, 0, st);
    HIP_OK(hipGetLastError());
    if (flags & EIK_CHECK_FEASIBLE) {
        launch_check_feasible<R>(n, M, om, w.ctr, st);
        unsigned long long bad = 0;
        HIP_OK(hipMemcpyAsync(&bad, w.ctr + kCtrInfeasible, 8, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (bad) return fail(EIK_EINFEASIBLE, "metric not SPD or |omega|_{M^-1} >= 1 somewhere");
    }
    launch_init<R>(g, T_init, T, parent, level, grid->src_idx, grid->src_t, w.act, w.act_count, w.ctr,
                   T_init != nullptr, st);
    HIP_OK(hipGetLastError());

    int rounds = 0;
    bool conv = false;
    LaunchTimer timer;
    rc = timer.init((flags & EIK_TIME_KERNELS) != 0, tn.rounds_per_check);
    if (rc) return rc;
    rc = run_rounds(
        w.act, w.act_count, g.n_tiles, max_rounds, tn.rounds_per_check, st,
        [&](int32_t *ain, int32_t *aout, int32_t *cnt) {
            launch_sweep_round<R>(g, M, om, T, parent, ain, aout, cnt, w.ctr, tol, tn.max_local_cycles, st);
        },
        &rounds, &conv, &timer);
    if (rc) return rc;
    HIP_OK(hipGetLastError());

    // active stencils and levels
    launch_parents<R>(g, M, om, T, parent, level, st);
    launch_fill_i32(w.act, 2 * (int64_t)g.n_tiles, 0, st);
    launch_fill_i32(w.act_count, kMaxRounds + 2, 0, st);
    launch_level_prep(g, w.act, w.act_count, st);
    int lrounds = 0;
    bool lconv = false;
    rc = run_rounds(
        w.act, w.act_count, g.n_tiles, kMaxRounds, tn.rounds_per_check, st,
        [&](int32_t *ain, int32_t *aout, int32_t *cnt) {
            launch_level_round(g, parent, level, ain, aout, cnt, tn.max_local_cycles, st);
        },
        &lrounds, &lconv);
    if (rc) return rc;
    if (!lconv) return fail(EIK_EDEVICE, "dependency levels did not settle");
    launch_max_level(n, level, w.ctr, st);
    HIP_OK(hipGetLastError());

    unsigned long long ctr[kCtrCount];
    HIP_OK(hipMemcpyAsync(ctr, w.ctr, sizeof ctr, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    int status = conv ? EIK_OK : EIK_NOT_CONVERGED;
    if (ctr[kCtrBadSource]) status = fail(EIK_EINVAL, "%llu source indices out of range", ctr[kCtrBadSource]);
    else if (!conv) fail(EIK_NOT_CONVERGED, "tolerance not reached in %d rounds", rounds);
    if (stats) {
        stats->rounds = rounds;
        stats->converged = conv ? 1 : 0;
        stats->cell_updates = (int64_t)ctr[kCtrCellUpdates];
        stats->n_levels = (int32_t)ctr[kCtrMaxLevel] + 1;
        stats->status = status;
        stats->sweep_launches = rounds;
        stats->sweep_ms = timer.ms;
    }
    return status;
}

template <typename R>
int backward_impl(const eik_grid *grid, const void *M, const void *om, const void *T, const uint8_t *parent,
                  const int32_t *level, const void *dLdT, void *dLdM, void *dLdom, void *dLdsrc, void *ws,
                  size_t ws_bytes, const eik_tuning *tun, hipStream_t st)
{
    const int dtype = sizeof(R) == 8 ? EIK_F64 : EIK_F32;
    Ws w;
    int rc = carve(grid, dtype, ws, ws_bytes, w);
    if (rc) return rc;
    const eik_tuning tn = tuning_or_default(tun);
    GridArgs g = make_grid(grid, kDefaultTH);
    const int64_t n = (int64_t)g.nx * g.ny;

    launch_fill_u64(w.ctr, kCtrCount, st);
    launch_fill_i32(w.counts, n + 2, 0, st);
    launch_max_level(n, level, w.ctr, st);
    launch_adj_prep<R>(g, M, om, T, parent, level, w.w1, w.counts, dLdM, dLdom, st);
    launch_scan_levels(w.counts, w.counts /*offsets in place*/, w.cursor, w.ctr, st);
    launch_scatter_levels(n, level, w.cursor, w.list, st);
    HIP_OK(hipGetLastError());
    if (n <= tn.adjoint_single_wg_max_cells) {
        launch_adj_levels<R>(g, -1, 0, true, w.ctr, w.counts, w.list, parent, w.w1, dLdT, M, w.lam, dLdM, dLdom,
                             st);
    } else {
        unsigned long long lmax = 0;
        HIP_OK(hipMemcpyAsync(&lmax, w.ctr + kCtrMaxLevel, 8, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        for (int L = (int)lmax; L >= 0; --L)
            launch_adj_levels<R>(g, L, L, false, w.ctr, w.counts, w.list, parent, w.w1, dLdT, M, w.lam, dLdM,
                                 dLdom, st);
    }
    launch_dsrc<R>(g, grid->src_idx, w.lam, dLdsrc, st);
    HIP_OK(hipGetLastError());
    return EIK_OK;
}

} // namespace

extern "C" {

size_t eik_workspace_bytes(const eik_grid *grid, int32_t dtype)
{
    if (check_grid(grid, dtype)) return 0;
    return layout(grid, dtype).total;
}

int eik_forward(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, const void *T_init,
                double tol, int32_t max_rounds, int32_t flags, void *T, uint8_t *parent, int32_t *level, void *ws,
                size_t ws_bytes, const eik_tuning *tuning, eik_stats *stats, hipStream_t stream)
{
    int rc = check_grid(grid, dtype);
    if (rc) return rc;
    if (!M || !omega || !T || !parent || !level) return fail(EIK_EINVAL, "NULL field or output pointer");
    if (!(tol >= 0.0)) return fail(EIK_EINVAL, "tol must be >= 0");
    if (max_rounds < 1) return fail(EIK_EINVAL, "max_rounds must be >= 1");
    if (dtype == EIK_F64)
        return forward_impl<double>(grid, M, omega, T_init, tol, max_rounds, flags, T, parent, level, ws, ws_bytes,
                                    tuning, stats, stream);
    return forward_impl<float>(grid, M, omega, T_init, tol, max_rounds, flags, T, parent, level, ws, ws_bytes,
                               tuning, stats, stream);
}

int eik_backward(const eik_grid *grid, int32_t dtype, const void *M, const void *omega, const void *T,
                 const uint8_t *parent, const int32_t *level, const void *dLdT, void *dLdM, void *dLdomega,
                 void *dLdsrc, void *ws, size_t ws_bytes, const eik_tuning *tuning, hipStream_t stream)
{
    int rc = check_grid(grid, dtype);
    if (rc) return rc;
    if (!M || !omega || !T || !parent || !level || !dLdT || !dLdM || !dLdomega || !dLdsrc)
        return fail(EIK_EINVAL, "NULL pointer argument");
    if (dtype == EIK_F64)
        return backward_impl<double>(grid, M, omega, T, parent, level, dLdT, dLdM, dLdomega, dLdsrc, ws, ws_bytes,
                                     tuning, stream);
    return backward_impl<float>(grid, M, omega, T, parent, level, dLdT, dLdM, dLdomega, dLdsrc, ws, ws_bytes,
                                tuning, stream);
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

const char *eik_last_error(void) { return g_last_error.c_str(); }

} // extern "C"
