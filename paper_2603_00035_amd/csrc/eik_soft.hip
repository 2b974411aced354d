// eik_soft.hip -- the soft-min mode, the smooth alternative to stencil
// selection named in Sec. 3.3: each stencil contributes the minimum of the
// Hopf-Lax objective over its segment (its two-point value of Eq. two_point
// when both barycentric weights are >= 0, else the smaller one-point value of
// Eq. one_point at its finite endpoints; no causality test), and a node takes
// the soft minimum T = -tau log sum_k exp(-H_k / tau) over its eight stencils.
// The update is continuously differentiable, and it makes a node depend on
// every neighbour (later ones too), so the adjoint system is not triangular:
// it is relaxed until it settles.
//
// Layout of the work: one workgroup per grid of a batch sweeps its grid line
// by line, rows up, rows down, columns up, columns down (the paper's
// column/row sweeps): the nodes of a line are updated in parallel from the
// current values (all reads of a line before its writes), the lines one after
// the other. A grid whose cycle of four directions changes no value beyond the
// tolerance is done: later cycle launches skip it, so its result does not
// depend on the rest of the batch. Lines are at most kSoftMaxLine nodes long.
// Arrays are packed grid after grid as in the batched hard solve.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "eik_device.h"
#include "eik_internal.h"

namespace eik {

// Workgroup shapes of the line sweeps: NT threads, PER nodes of a line per
// thread. The host takes the smallest that covers the batch's longest line:
// one wave per grid for grids up to 64 nodes wide (many grids per CU), up to
// 512 threads with 8 nodes each for lines up to kSoftMaxLine.
constexpr int kSoftWideThreads = 512;
constexpr int kSoftWidePer = kSoftMaxLine / kSoftWideThreads;

// Segment minimum of stencil S: value, the code of the piece that attains it
// (S for the interior two-point value, 8 + k for the one-point value of
// neighbour k, kUnreached when neither donor is finite) and the weight w1 of
// the stencil's first donor for the interior piece.
template <typename R, int S>
__device__ __forceinline__ R stencil_hl(const NodeConst<R> &k, const R Tn[8], int &code, R &w1)
{
    constexpr int Q = (S + 1) & 7;
    const R inf = inf_v<R>();
    const R Tp = Tn[S], Tq = Tn[Q];
    R best = inf;
    code = kUnreached;
    w1 = R(1);
    if (Tp < inf && Tq < inf) {
        R t, mu1, mu2;
        if (two_point_root(k, S, Tp, Tq, t, mu1, mu2) && mu1 >= R(0) && mu2 >= R(0) && mu1 + mu2 > R(0)) {
            best = t;
            code = S;
            w1 = mu1 / (mu1 + mu2);
        }
    }
    const R op = Tp + k.c1[S], oq = Tq + k.c1[Q]; // +inf for an unreached donor
    if (op < best) {
        best = op;
        code = 8 + S;
        w1 = R(1);
    }
    if (oq < best) {
        best = oq;
        code = 8 + Q;
        w1 = R(1);
    }
    return best;
}

template <typename R>
__device__ __forceinline__ void all_stencils(const NodeConst<R> &k, const R Tn[8], R H[8], int code[8], R w1[8])
{
    H[0] = stencil_hl<R, 0>(k, Tn, code[0], w1[0]);
    H[1] = stencil_hl<R, 1>(k, Tn, code[1], w1[1]);
    H[2] = stencil_hl<R, 2>(k, Tn, code[2], w1[2]);
    H[3] = stencil_hl<R, 3>(k, Tn, code[3], w1[3]);
    H[4] = stencil_hl<R, 4>(k, Tn, code[4], w1[4]);
    H[5] = stencil_hl<R, 5>(k, Tn, code[5], w1[5]);
    H[6] = stencil_hl<R, 6>(k, Tn, code[6], w1[6]);
    H[7] = stencil_hl<R, 7>(k, Tn, code[7], w1[7]);
}

// -tau log sum exp(-H_k / tau), shifted by the smallest H for range; +inf when
// no stencil has a finite donor. inv_tau = 1 / tau (a multiply per stencil in
// place of a division).
template <typename R>
__device__ __forceinline__ R soft_min(const R H[8], R tau, R inv_tau)
{
    const R inf = inf_v<R>();
    R m = inf;
#pragma unroll
    for (int s = 0; s < 8; ++s) m = H[s] < m ? H[s] : m;
    if (!(m < inf)) return inf;
    R sum = R(0);
#pragma unroll
    for (int s = 0; s < 8; ++s)
        if (H[s] < inf) sum += exp((m - H[s]) * inv_tau);
    return m - tau * log(sum);
}

// One grid of a batch, as the device sees it.
struct SoftDesc {
    int64_t off; // first node in the packed node arrays
    double h;
    int32_t nx, ny;
    int32_t n_src, src_base;
};
static_assert(sizeof(SoftDesc) == kSoftDescBytes, "descriptor size shared with the host layout");

// Neighbour times of node (i, j) from a row-major field of pitch tp (+inf
// outside the grid).
template <typename R>
__device__ __forceinline__ void neighbour_times(const SoftDesc &g, const R *T, int tp, int i, int j, R Tn[8])
{
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const int a = i + nb_dx(d), b = j + nb_dy(d);
        Tn[d] = (a < 0 || a >= g.nx || b < 0 || b >= g.ny) ? inf_v<R>() : T[b * tp + a];
    }
}

// Node e of line `line` in direction dir: 0 rows up, 1 rows down, 2 columns
// up, 3 columns down.
__device__ __forceinline__ void line_node(int dir, int line, int e, int &i, int &j)
{
    if (dir < 2) {
        i = e;
        j = line;
    } else {
        i = line;
        j = e;
    }
}

// Pitch of a grid held in LDS: odd, so that a column of values falls in
// distinct banks.
__host__ __device__ inline int soft_pitch(int nx) { return nx | 1; }

// Whether a value's move from a to b keeps the iteration going: any change
// between finite and infinite, else |b - a| > tol max(|b|, scale), where scale
// is the largest finite magnitude of the previous cycle (a floor that keeps
// values near zero from holding the iteration on their last bits).
template <typename R>
__device__ __forceinline__ bool soft_change(R a, R b, R tol, R scale)
{
    if (a == b) return false;
    const R inf = inf_v<R>();
    if (a == inf || b == inf) return true;
    const R d = fabs(b - a), m = fabs(b);
    return d > tol * (m > scale ? m : scale);
}

// Largest value over the workgroup of NT threads; every thread must call it.
template <typename R, int NT>
__device__ R block_max(R v, R *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    return red[0];
}

// Per-grid state of an iteration (caller's workspace): the scale of
// soft_change carried from cycle to cycle, whether the grid is done, and its
// cycle count.
template <typename R>
struct SoftState {
    R *scale;
    int32_t *done, *cycles;
};

// The end of one cycle: flag and scale over the workgroup. Returns whether
// the cycle changed anything; every thread must call it.
template <typename R, int NT>
__device__ __forceinline__ bool cycle_end(bool ch, R &vmax, int *s_changed, R *s_red)
{
    if (ch) atomicOr(s_changed, 1);
    vmax = block_max<R, NT>(vmax, s_red); // its barriers also order s_changed
    const bool changed = *s_changed != 0;
    __syncthreads(); // every thread has read the flag and the maximum before the next cycle resets them
    return changed;
}

// Up to ncyc cycles of the four directional sweeps of the soft update over
// grid blockIdx.x, stopping after the first quiet one (skipped once the grid
// is done). LDS: the grid's times and source marks live in LDS for the
// launch (row-major, odd pitch), else the sweeps work on the global field.
// Rows read the parameters row-major (M, om), columns from the transposed
// copy Pt ([5][nx][ny]), so that the nodes of a line are contiguous either way.
template <typename R, int NT, int PER, bool LDS>
__global__ __launch_bounds__(NT) void k_soft_cycle(const SoftDesc *__restrict__ descs,
                                                  const R *__restrict__ Mall, const R *__restrict__ omall,
                                                  const R *__restrict__ Ptall, R *Tall,
                                                  const uint8_t *__restrict__ markall, R tau, R tol, int ncyc,
                                                  SoftState<R> st)
{
    extern __shared__ __align__(16) unsigned char soft_lds[];
    const int gi = blockIdx.x;
    if (st.done[gi]) return; // uniform over the workgroup
    const SoftDesc g = descs[gi];
    const int n = g.nx * g.ny;
    const R *M = Mall + 3 * g.off, *om = omall + 2 * g.off, *Pt = Ptall + 5 * g.off;
    R *Tg = Tall + g.off;
    const uint8_t *markg = markall + g.off;
    const int tp = LDS ? soft_pitch(g.nx) : g.nx;
    R *T = LDS ? (R *)soft_lds : Tg;
    uint8_t *mark = LDS ? soft_lds + (size_t)g.ny * tp * sizeof(R) : (uint8_t *)markg;
    const R h = R(g.h), inv_h = R(1) / h, inv_tau = R(1) / tau;
    __shared__ int s_changed;
    __shared__ R s_red[NT];
    if (LDS) {
        for (int c = threadIdx.x; c < n; c += NT) {
            const int i = c % g.nx, j = c / g.nx;
            T[j * tp + i] = Tg[c];
            mark[j * tp + i] = markg[c];
        }
    }
    R scale = st.scale[gi];
    int cyc = 0;
    bool quiet = false;
    while (cyc < ncyc && !quiet) {
        if (threadIdx.x == 0) s_changed = 0;
        __syncthreads();
        bool ch = false;
        R vmax = R(0);
        for (int dir = 0; dir < 4; ++dir) {
            const int len = dir < 2 ? g.ny : g.nx, span = dir < 2 ? g.nx : g.ny;
            const R *P = dir < 2 ? M : Pt;
            const R *O = dir < 2 ? om : Pt + 3 * n;
            // the parameters of the next line load while a line is updated
            // (c: the node in the layout P and O follow; lanes past the line
            // read its last node)
            auto fetch = [&](int s, R (*p)[5]) {
                const int line = (dir & 1) ? len - 1 - s : s;
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int e = min(threadIdx.x + q * NT, span - 1);
                    const int c = line * span + e;
                    p[q][0] = P[c];
                    p[q][1] = P[n + c];
                    p[q][2] = P[2 * n + c];
                    p[q][3] = O[c];
                    p[q][4] = O[n + c];
                }
            };
            // one line ahead with one node per thread; wide workgroups (8 nodes
            // per thread) load each line as it comes, to stay within registers
            constexpr bool AHEAD = PER == 1;
            R pc[PER][5], pn[AHEAD ? PER : 1][5];
            if (AHEAD) fetch(0, pc);
            for (int s = 0; s < len; ++s) {
                const int line = (dir & 1) ? len - 1 - s : s;
                if (!AHEAD) fetch(s, pc);
                else if (s + 1 < len) fetch(s + 1, pn); // uniform over the workgroup
                R v[PER];
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int e = threadIdx.x + q * NT;
                    if (e >= span) continue;
                    int i, j;
                    line_node(dir, line, e, i, j);
                    const int at = j * tp + i;
                    if (mark[at] == kSource) {
                        v[q] = T[at];
                        continue;
                    }
                    NodeConst<R> k;
                    node_const<R>(pc[q][0], pc[q][1], pc[q][2], pc[q][3], pc[q][4], h, inv_h, k);
                    R Tn[8], H[8], w1[8];
                    int code[8];
                    neighbour_times<R>(g, T, tp, i, j, Tn);
                    all_stencils<R>(k, Tn, H, code, w1);
                    v[q] = soft_min<R>(H, tau, inv_tau);
                }
                __syncthreads(); // every read of the line before its writes
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int e = threadIdx.x + q * NT;
                    if (e >= span) continue;
                    int i, j;
                    line_node(dir, line, e, i, j);
                    const int at = j * tp + i;
                    ch |= soft_change<R>(T[at], v[q], tol, scale);
                    if (v[q] < inf_v<R>()) vmax = fmax(vmax, fabs(v[q]));
                    T[at] = v[q];
                }
                if (AHEAD) {
#pragma unroll
                    for (int a = 0; a < 5; ++a) pc[0][a] = pn[0][a];
                }
                __syncthreads(); // the line's values before the next line reads them
            }
        }
        quiet = !cycle_end<R, NT>(ch, vmax, &s_changed, s_red);
        scale = vmax;
        ++cyc;
    }
    if (LDS) {
        for (int c = threadIdx.x; c < n; c += NT) Tg[c] = T[(c / g.nx) * tp + c % g.nx];
    }
    if (threadIdx.x == 0) {
        if (quiet) st.done[gi] = 1;
        st.scale[gi] = scale;
        st.cycles[gi] += cyc;
    }
}

template <typename R>
__global__ void k_soft_init(int64_t n, R *__restrict__ T, uint8_t *__restrict__ mark, int32_t *__restrict__ bad)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *bad = 0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        if (T) T[c] = inf_v<R>();
        mark[c] = 0;
    }
}

// Sources of grid blockIdx.x: T = t_s (0 without times), marked; indices
// outside the grid are counted in *bad. Also resets the grid's iteration state.
template <typename R>
__global__ void k_soft_sources(const SoftDesc *__restrict__ descs, const int32_t *__restrict__ src,
                               const R *__restrict__ src_t, R *__restrict__ T, uint8_t *__restrict__ mark,
                               int32_t *__restrict__ bad, SoftState<R> st)
{
    const int gi = blockIdx.x;
    const SoftDesc g = descs[gi];
    if (threadIdx.x == 0) {
        st.scale[gi] = R(0);
        st.done[gi] = 0;
        st.cycles[gi] = 0;
    }
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int s = threadIdx.x; s < g.n_src; s += blockDim.x) {
        const int32_t c = src[g.src_base + s];
        if (c < 0 || (int64_t)c >= n) {
            atomicAdd(bad, 1);
            continue;
        }
        mark[g.off + c] = kSource;
        if (T) T[g.off + c] = src_t ? src_t[g.src_base + s] : R(0);
    }
}

// Transposed copy of a grid's five parameter planes ([5][nx][ny]) for the
// column sweeps; grid blockIdx.y.
template <typename R>
__global__ void k_soft_transpose(const SoftDesc *__restrict__ descs, const R *__restrict__ Mall,
                                 const R *__restrict__ omall, R *__restrict__ Ptall)
{
    const SoftDesc g = descs[blockIdx.y];
    const int n = g.nx * g.ny;
    const R *M = Mall + 3 * g.off, *om = omall + 2 * g.off;
    R *Pt = Ptall + 5 * g.off;
    for (int ct = blockIdx.x * blockDim.x + threadIdx.x; ct < n; ct += gridDim.x * blockDim.x) {
        const int j = ct % g.ny, i = ct / g.ny, c = j * g.nx + i; // consecutive threads write consecutive ct
        Pt[ct] = M[c];
        Pt[n + ct] = M[n + c];
        Pt[2 * n + ct] = M[2 * n + c];
        Pt[3 * n + ct] = om[c];
        Pt[4 * n + ct] = om[n + c];
    }
}

// Partial derivatives of each node's soft update at the field T, stored for
// the adjoint as incoming weights: win[d][x] (row-major) and winT[d][x]
// (transposed) hold the derivative of neighbour nb_d(x)'s update with respect
// to T_x, so that lambda_x = g_x + sum_d win[d][x] lambda_{nb_d(x)}; node c
// writes its coefficient for neighbour d into entry (opp d, nb_d(c)), one
// writer per entry, and entries towards nodes outside the grid are never read.
// dth[a] (planes per grid at 5 off) holds the derivative with respect to the
// node's stored m11, m12, m22, bx, by; coefficients and dth are zero at
// sources and unreached nodes (their values do not follow the update). Also
// writes the transposed dL/dT (gt), clears lambda and the iteration state.
// Grid blockIdx.y.
template <typename R>
__global__ __launch_bounds__(256) void k_soft_coef(const SoftDesc *__restrict__ descs, const R *__restrict__ Mall,
                                                   const R *__restrict__ omall, const R *__restrict__ Tall,
                                                   const uint8_t *__restrict__ markall, const R *__restrict__ gall,
                                                   R tau, R *__restrict__ winall, R *__restrict__ wintall,
                                                   R *__restrict__ dthall, R *__restrict__ gtall,
                                                   R *__restrict__ lamall, SoftState<R> st)
{
    const int gi = blockIdx.y;
    const SoftDesc g = descs[gi];
    const int n = g.nx * g.ny;
    const R *M = Mall + 3 * g.off, *om = omall + 2 * g.off, *T = Tall + g.off, *gT = gall + g.off;
    const uint8_t *mark = markall + g.off;
    R *win = winall + 8 * g.off, *wint = wintall + 8 * g.off, *dth = dthall + 5 * g.off, *gt = gtall + g.off;
    R *lam = lamall + g.off;
    const R h = R(g.h), inv_tau = R(1) / tau;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.scale[gi] = R(0);
        st.done[gi] = 0;
        st.cycles[gi] = 0;
    }
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const int i = c % g.nx, j = c / g.nx;
        lam[c] = R(0);
        gt[i * g.ny + j] = gT[c];
        R cf[8], dt[5];
#pragma unroll
        for (int d = 0; d < 8; ++d) cf[d] = R(0);
#pragma unroll
        for (int a = 0; a < 5; ++a) dt[a] = R(0);
        if (mark[c] != kSource && T[c] < inf_v<R>()) {
            NodeConst<R> k;
            node_const<R>(M[c], M[n + c], M[2 * n + c], om[c], om[n + c], h, R(1) / h, k);
            R Tn[8], H[8], w1[8];
            int code[8];
            neighbour_times<R>(g, T, g.nx, i, j, Tn);
            all_stencils<R>(k, Tn, H, code, w1);
            const R v = soft_min<R>(H, tau, inv_tau);
            const R m11 = M[c], m12 = M[n + c], m22 = M[2 * n + c];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                if (!(H[s] < inf_v<R>())) continue;
                const R p = exp((v - H[s]) * inv_tau); // soft-min weight of stencil s
                if (code[s] < 8) {
                    cf[s] += p * w1[s];
                    cf[(s + 1) & 7] += p * (R(1) - w1[s]);
                } else {
                    cf[code[s] - 8] += p;
                }
                R f[5];
                param_derivs<R>(code[s], w1[s], m11, m12, m22, h, f);
#pragma unroll
                for (int a = 0; a < 5; ++a) dt[a] += p * f[a];
            }
        }
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int a = i + nb_dx(d), b = j + nb_dy(d);
            if (a < 0 || a >= g.nx || b < 0 || b >= g.ny) continue;
            const int o = (d + 4) & 7;
            win[o * n + b * g.nx + a] = cf[d];
            wint[o * n + a * g.ny + b] = cf[d];
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) dth[a * n + c] = dt[a];
    }
}

// Up to ncyc cycles of the adjoint relaxation lambda_x = g_x + sum_d win[d][x]
// lambda_{nb_d(x)} over grid blockIdx.x, with the line order of the forward,
// stopping after the first quiet cycle (unreached nodes keep lambda = 0). Rows
// read win and g row-major, columns the transposed copies. LDS: lambda and the
// reached flags live in LDS for the launch.
template <typename R, int NT, int PER, bool LDS>
__global__ __launch_bounds__(NT) void k_soft_adj_cycle(const SoftDesc *__restrict__ descs,
                                                      const R *__restrict__ winall, const R *__restrict__ wintall,
                                                      const R *__restrict__ gall, const R *__restrict__ gtall,
                                                      const R *__restrict__ Tall, R *lamall, R tol, int ncyc,
                                                      SoftState<R> st)
{
    extern __shared__ __align__(16) unsigned char soft_lds[];
    const int gi = blockIdx.x;
    if (st.done[gi]) return;
    const SoftDesc g = descs[gi];
    const int n = g.nx * g.ny;
    const R *win = winall + 8 * g.off, *wint = wintall + 8 * g.off, *gg = gall + g.off, *gt = gtall + g.off;
    const R *Tg = Tall + g.off;
    R *lamg = lamall + g.off;
    const int tp = LDS ? soft_pitch(g.nx) : g.nx;
    R *lam = LDS ? (R *)soft_lds : lamg;
    uint8_t *reach = LDS ? soft_lds + (size_t)g.ny * tp * sizeof(R) : nullptr;
    __shared__ int s_changed;
    __shared__ R s_red[NT];
    if (LDS) {
        for (int c = threadIdx.x; c < n; c += NT) {
            const int at = (c / g.nx) * tp + c % g.nx;
            lam[at] = lamg[c];
            reach[at] = Tg[c] < inf_v<R>();
        }
    }
    R scale = st.scale[gi];
    int cyc = 0;
    bool quiet = false;
    while (cyc < ncyc && !quiet) {
        if (threadIdx.x == 0) s_changed = 0;
        __syncthreads();
        bool ch = false;
        R vmax = R(0);
        for (int dir = 0; dir < 4; ++dir) {
            const int len = dir < 2 ? g.ny : g.nx, span = dir < 2 ? g.nx : g.ny;
            const R *W = dir < 2 ? win : wint;
            const R *G = dir < 2 ? gg : gt;
            // the weights and dL/dT of the next line load while a line is
            // updated (c: the node in the layout W and G follow; lanes past
            // the line read its last node)
            auto fetch = [&](int s, R (*w)[9]) {
                const int line = (dir & 1) ? len - 1 - s : s;
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int e = min(threadIdx.x + q * NT, span - 1);
                    const int c = line * span + e;
#pragma unroll
                    for (int d = 0; d < 8; ++d) w[q][d] = W[d * n + c];
                    w[q][8] = G[c];
                }
            };
            constexpr bool AHEAD = PER == 1; // as in the forward
            R wc[PER][9], wn[AHEAD ? PER : 1][9];
            if (AHEAD) fetch(0, wc);
            for (int s = 0; s < len; ++s) {
                const int line = (dir & 1) ? len - 1 - s : s;
                if (!AHEAD) fetch(s, wc);
                else if (s + 1 < len) fetch(s + 1, wn); // uniform over the workgroup
                R v[PER];
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int e = threadIdx.x + q * NT;
                    if (e >= span) continue;
                    int i, j;
                    line_node(dir, line, e, i, j);
                    const bool reached = LDS ? reach[j * tp + i] != 0 : Tg[j * g.nx + i] < inf_v<R>();
                    if (!reached) {
                        v[q] = R(0);
                        continue;
                    }
                    R acc = wc[q][8];
#pragma unroll
                    for (int d = 0; d < 8; ++d) {
                        const int a = i + nb_dx(d), b = j + nb_dy(d);
                        if (a < 0 || a >= g.nx || b < 0 || b >= g.ny) continue;
                        acc += wc[q][d] * lam[b * tp + a];
                    }
                    v[q] = acc;
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int e = threadIdx.x + q * NT;
                    if (e >= span) continue;
                    int i, j;
                    line_node(dir, line, e, i, j);
                    const int at = j * tp + i;
                    ch |= soft_change<R>(lam[at], v[q], tol, scale);
                    vmax = fmax(vmax, fabs(v[q]));
                    lam[at] = v[q];
                }
                if (AHEAD) {
#pragma unroll
                    for (int d = 0; d < 9; ++d) wc[0][d] = wn[0][d];
                }
                __syncthreads();
            }
        }
        quiet = !cycle_end<R, NT>(ch, vmax, &s_changed, s_red);
        scale = vmax;
        ++cyc;
    }
    if (LDS) {
        for (int c = threadIdx.x; c < n; c += NT) lamg[c] = lam[(c / g.nx) * tp + c % g.nx];
    }
    if (threadIdx.x == 0) {
        if (quiet) st.done[gi] = 1;
        st.scale[gi] = scale;
        st.cycles[gi] += cyc;
    }
}

// dL/dtheta_i = lambda_i dth_i (zero at sources and unreached nodes: their dth
// is zero), grid blockIdx.y.
template <typename R>
__global__ void k_soft_params(const SoftDesc *__restrict__ descs, const R *__restrict__ lamall,
                              const R *__restrict__ dthall, R *__restrict__ dMall, R *__restrict__ domall)
{
    const SoftDesc g = descs[blockIdx.y];
    const int64_t n = (int64_t)g.nx * g.ny;
    const R *lam = lamall + g.off, *dth = dthall + 5 * g.off;
    R *dM = dMall + 3 * g.off, *dom = domall + 2 * g.off;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const R l = lam[c];
        dM[c] = l * dth[c];
        dM[n + c] = l * dth[n + c];
        dM[2 * n + c] = l * dth[2 * n + c];
        dom[c] = l * dth[3 * n + c];
        dom[n + c] = l * dth[4 * n + c];
    }
}

// dL/dt_s = lambda_s, grid blockIdx.x.
template <typename R>
__global__ void k_soft_dsrc(const SoftDesc *__restrict__ descs, const int32_t *__restrict__ src,
                            const R *__restrict__ lamall, R *__restrict__ dsrc)
{
    const SoftDesc g = descs[blockIdx.x];
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int s = threadIdx.x; s < g.n_src; s += blockDim.x) {
        const int32_t c = src[g.src_base + s];
        dsrc[g.src_base + s] = (c >= 0 && (int64_t)c < n) ? lamall[g.off + c] : R(0);
    }
}

// 2-D launch over the nodes of every grid: y = grid, x = enough blocks of 256
// for the largest grid (at most 1024).
static inline dim3 soft_node_grid(int n_grids, int64_t max_nodes)
{
    return dim3((unsigned)std::min<int64_t>((max_nodes + 255) / 256, 1024), (unsigned)n_grids);
}

template <typename R>
static SoftState<R> soft_state(const SoftBatch &b)
{
    return SoftState<R>{(R *)b.scale, b.done, b.cycles};
}

// LDS bytes of the largest grid held in LDS by the cycle kernels (values and
// one byte per node at the odd pitch); 0 when the batch's largest grid does
// not fit the budget and the sweeps work on the global arrays.
template <typename R>
static size_t soft_lds_bytes(const SoftBatch &b)
{
    const size_t need = (size_t)b.max_rows * soft_pitch(b.max_cols) * (sizeof(R) + 1);
    return need <= kSoftLdsBudget ? need : 0;
}

template <typename R>
void launch_soft_init(const SoftBatch &b, const int32_t *src, const void *src_t, void *T, const void *M,
                      const void *om, hipStream_t st)
{
    hipLaunchKernelGGL(k_soft_init<R>, dim3((unsigned)std::min<int64_t>((b.n_nodes + 255) / 256, 4096)), dim3(256), 0,
                       st, b.n_nodes, (R *)T, b.mark, b.bad);
    hipLaunchKernelGGL(k_soft_sources<R>, dim3(b.n_grids), dim3(256), 0, st, (const SoftDesc *)b.descs, src,
                       (const R *)src_t, (R *)T, b.mark, b.bad, soft_state<R>(b));
    if (M)
        hipLaunchKernelGGL(k_soft_transpose<R>, soft_node_grid(b.n_grids, b.max_nodes), dim3(256), 0, st,
                           (const SoftDesc *)b.descs, (const R *)M, (const R *)om, (R *)b.Pt);
}

template <typename R, int NT, int PER>
static void soft_cycle_nt(const SoftBatch &b, const void *M, const void *om, void *T, double tau, double tol, int ncyc,
                          hipStream_t st)
{
    const size_t lds = soft_lds_bytes<R>(b);
    if (lds)
        hipLaunchKernelGGL((k_soft_cycle<R, NT, PER, true>), dim3(b.n_grids), dim3(NT), lds, st,
                           (const SoftDesc *)b.descs, (const R *)M, (const R *)om, (const R *)b.Pt, (R *)T, b.mark,
                           R(tau), R(tol), ncyc, soft_state<R>(b));
    else
        hipLaunchKernelGGL((k_soft_cycle<R, NT, PER, false>), dim3(b.n_grids), dim3(NT), 0, st,
                           (const SoftDesc *)b.descs, (const R *)M, (const R *)om, (const R *)b.Pt, (R *)T, b.mark,
                           R(tau), R(tol), ncyc, soft_state<R>(b));
}

template <typename R>
void launch_soft_cycles(const SoftBatch &b, const void *M, const void *om, void *T, double tau, double tol, int ncyc,
                        hipStream_t st)
{
    if (b.max_line <= 64) soft_cycle_nt<R, 64, 1>(b, M, om, T, tau, tol, ncyc, st);
    else if (b.max_line <= 128) soft_cycle_nt<R, 128, 1>(b, M, om, T, tau, tol, ncyc, st);
    else if (b.max_line <= 256) soft_cycle_nt<R, 256, 1>(b, M, om, T, tau, tol, ncyc, st);
    else soft_cycle_nt<R, kSoftWideThreads, kSoftWidePer>(b, M, om, T, tau, tol, ncyc, st);
}

template <typename R>
void launch_soft_coef(const SoftBatch &b, const void *M, const void *om, const void *T, const void *gT, double tau,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_soft_coef<R>, soft_node_grid(b.n_grids, b.max_nodes), dim3(256), 0, st,
                       (const SoftDesc *)b.descs, (const R *)M, (const R *)om, (const R *)T, b.mark, (const R *)gT,
                       R(tau), (R *)b.win, (R *)b.wint, (R *)b.dth, (R *)b.gt, (R *)b.lam, soft_state<R>(b));
}

template <typename R, int NT, int PER>
static void soft_adj_cycle_nt(const SoftBatch &b, const void *gT, const void *T, double tol, int ncyc, hipStream_t st)
{
    const size_t lds = soft_lds_bytes<R>(b);
    if (lds)
        hipLaunchKernelGGL((k_soft_adj_cycle<R, NT, PER, true>), dim3(b.n_grids), dim3(NT), lds, st,
                           (const SoftDesc *)b.descs, (const R *)b.win, (const R *)b.wint, (const R *)gT,
                           (const R *)b.gt, (const R *)T, (R *)b.lam, R(tol), ncyc, soft_state<R>(b));
    else
        hipLaunchKernelGGL((k_soft_adj_cycle<R, NT, PER, false>), dim3(b.n_grids), dim3(NT), 0, st,
                           (const SoftDesc *)b.descs, (const R *)b.win, (const R *)b.wint, (const R *)gT,
                           (const R *)b.gt, (const R *)T, (R *)b.lam, R(tol), ncyc, soft_state<R>(b));
}

template <typename R>
void launch_soft_adj_cycles(const SoftBatch &b, const void *gT, const void *T, double tol, int ncyc, hipStream_t st)
{
    if (b.max_line <= 64) soft_adj_cycle_nt<R, 64, 1>(b, gT, T, tol, ncyc, st);
    else if (b.max_line <= 128) soft_adj_cycle_nt<R, 128, 1>(b, gT, T, tol, ncyc, st);
    else if (b.max_line <= 256) soft_adj_cycle_nt<R, 256, 1>(b, gT, T, tol, ncyc, st);
    else soft_adj_cycle_nt<R, kSoftWideThreads, kSoftWidePer>(b, gT, T, tol, ncyc, st);
}

template <typename R>
void launch_soft_params(const SoftBatch &b, const int32_t *src, void *dM, void *dom, void *dsrc, hipStream_t st)
{
    hipLaunchKernelGGL(k_soft_params<R>, soft_node_grid(b.n_grids, b.max_nodes), dim3(256), 0, st,
                       (const SoftDesc *)b.descs, (const R *)b.lam, (const R *)b.dth, (R *)dM, (R *)dom);
    hipLaunchKernelGGL(k_soft_dsrc<R>, dim3(b.n_grids), dim3(256), 0, st, (const SoftDesc *)b.descs, src,
                       (const R *)b.lam, (R *)dsrc);
}

void write_soft_desc(int64_t off, double h, int32_t nx, int32_t ny, int32_t n_src, int32_t src_base, void *dst)
{
    SoftDesc d;
    d.off = off;
    d.h = h;
    d.nx = nx;
    d.ny = ny;
    d.n_src = n_src;
    d.src_base = src_base;
    memcpy(dst, &d, sizeof d);
}

#define EIK_SOFT_INST(R)                                                                                           \
    template void launch_soft_init<R>(const SoftBatch &, const int32_t *, const void *, void *, const void *,       \
                                      const void *, hipStream_t);                                                  \
    template void launch_soft_cycles<R>(const SoftBatch &, const void *, const void *, void *, double, double, int, \
                                        hipStream_t);                                                              \
    template void launch_soft_coef<R>(const SoftBatch &, const void *, const void *, const void *, const void *,    \
                                      double, hipStream_t);                                                        \
    template void launch_soft_adj_cycles<R>(const SoftBatch &, const void *, const void *, double, int,            \
                                            hipStream_t);                                                          \
    template void launch_soft_params<R>(const SoftBatch &, const int32_t *, void *, void *, void *, hipStream_t);
EIK_SOFT_INST(float)
EIK_SOFT_INST(double)
#undef EIK_SOFT_INST

} // namespace eik
