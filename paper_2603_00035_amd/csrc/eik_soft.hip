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
// Layout of the work: one workgroup per grid sweeps the grid line by line,
// rows up, rows down, columns up, columns down (the paper's column/row
// sweeps): the nodes of a line are updated in parallel from the current
// values (all reads of a line before its writes), the lines one after the
// other. A cycle of four directions that changes no value beyond the
// tolerance ends the solve. Lines are at most kSoftMaxLine nodes long.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eik_device.h"
#include "eik_internal.h"

namespace eik {

constexpr int kSoftThreads = 512; // 2 waves per SIMD: room for the FP64 update's registers
constexpr int kSoftPer = kSoftMaxLine / kSoftThreads; // nodes of a line per thread

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
// no stencil has a finite donor.
template <typename R>
__device__ __forceinline__ R soft_min(const R H[8], R tau)
{
    const R inf = inf_v<R>();
    R m = inf;
#pragma unroll
    for (int s = 0; s < 8; ++s) m = H[s] < m ? H[s] : m;
    if (!(m < inf)) return inf;
    R sum = R(0);
#pragma unroll
    for (int s = 0; s < 8; ++s)
        if (H[s] < inf) sum += exp((m - H[s]) / tau);
    return m - tau * log(sum);
}

struct SoftGrid {
    int32_t nx, ny;
    double h;
};

template <typename R>
__device__ __forceinline__ void node_inputs(const SoftGrid &g, const R *__restrict__ M, const R *__restrict__ om,
                                            const R *T, int i, int j, NodeConst<R> &k, R Tn[8])
{
    const int64_t n = (int64_t)g.nx * g.ny, c = (int64_t)j * g.nx + i;
    const R h = R(g.h);
    node_const<R>(M[c], M[n + c], M[2 * n + c], om[c], om[n + c], h, R(1) / h, k);
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const int a = i + nb_dx(d), b = j + nb_dy(d);
        Tn[d] = (a < 0 || a >= g.nx || b < 0 || b >= g.ny) ? inf_v<R>() : T[(int64_t)b * g.nx + a];
    }
}

// Node e of line `line` in direction dir: 0 rows up, 1 rows down, 2 columns
// up, 3 columns down.
__device__ __forceinline__ void line_node(const SoftGrid &g, int dir, int line, int e, int &i, int &j)
{
    if (dir < 2) {
        i = e;
        j = line;
    } else {
        i = line;
        j = e;
    }
}

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

// Largest value over the workgroup; every thread must call it.
template <typename R>
__device__ R block_max(R v, R *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kSoftThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    return red[0];
}

// One cycle of the four directional sweeps of the soft update. changed
// receives 1 when some value moved (soft_change); ctl_scale carries the scale
// of soft_change from cycle to cycle (0 before the first).
template <typename R>
__global__ __launch_bounds__(kSoftThreads) void k_soft_cycle(SoftGrid g, const R *__restrict__ M,
                                                            const R *__restrict__ om, R *T,
                                                            const uint8_t *__restrict__ mark, R tau, R tol,
                                                            int32_t *__restrict__ changed, R *ctl_scale)
{
    __shared__ int s_changed;
    __shared__ R s_red[kSoftThreads];
    if (threadIdx.x == 0) s_changed = 0;
    const R scale = *ctl_scale;
    __syncthreads();
    bool ch = false;
    R vmax = R(0);
    for (int dir = 0; dir < 4; ++dir) {
        const int len = dir < 2 ? g.ny : g.nx, span = dir < 2 ? g.nx : g.ny;
        for (int s = 0; s < len; ++s) {
            const int line = (dir & 1) ? len - 1 - s : s;
            R v[kSoftPer];
#pragma unroll
            for (int q = 0; q < kSoftPer; ++q) {
                const int e = threadIdx.x + q * kSoftThreads;
                if (e >= span) continue;
                int i, j;
                line_node(g, dir, line, e, i, j);
                const int64_t c = (int64_t)j * g.nx + i;
                if (mark[c] == kSource) {
                    v[q] = T[c];
                    continue;
                }
                NodeConst<R> k;
                R Tn[8], H[8], w1[8];
                int code[8];
                node_inputs<R>(g, M, om, T, i, j, k, Tn);
                all_stencils<R>(k, Tn, H, code, w1);
                v[q] = soft_min<R>(H, tau);
            }
            __syncthreads(); // every read of the line before its writes
#pragma unroll
            for (int q = 0; q < kSoftPer; ++q) {
                const int e = threadIdx.x + q * kSoftThreads;
                if (e >= span) continue;
                int i, j;
                line_node(g, dir, line, e, i, j);
                const int64_t c = (int64_t)j * g.nx + i;
                ch |= soft_change<R>(T[c], v[q], tol, scale);
                if (v[q] < inf_v<R>()) vmax = fmax(vmax, fabs(v[q]));
                T[c] = v[q];
            }
            __syncthreads(); // the line's values before the next line reads them
        }
    }
    if (ch) atomicOr(&s_changed, 1);
    vmax = block_max<R>(vmax, s_red); // its barriers also order s_changed
    if (threadIdx.x == 0) {
        *changed = s_changed;
        *ctl_scale = vmax;
    }
}

template <typename R>
__global__ void k_soft_init(int64_t n, R *__restrict__ T, uint8_t *__restrict__ mark)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        if (T) T[c] = inf_v<R>();
        mark[c] = 0;
    }
}

// Sources: T = t_s (0 without times), marked; out-of-range indices are
// counted in *bad. One workgroup: it also clears *bad and the scale.
template <typename R>
__global__ void k_soft_sources(int64_t n, int n_src, const int32_t *__restrict__ src, const R *__restrict__ src_t,
                               R *__restrict__ T, uint8_t *__restrict__ mark, int32_t *__restrict__ bad,
                               R *__restrict__ ctl_scale)
{
    if (threadIdx.x == 0) {
        *bad = 0;
        *ctl_scale = R(0);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < n_src; s += blockDim.x) {
        const int32_t c = src[s];
        if (c < 0 || (int64_t)c >= n) {
            atomicAdd(bad, 1);
            continue;
        }
        mark[c] = kSource;
        if (T) T[c] = src_t ? src_t[s] : R(0);
    }
}

// Partial derivatives of each node's soft update at the field T: coef[d][c]
// with respect to neighbour d's time (summing to 1), dth[a][c] with respect
// to the node's stored m11, m12, m22, bx, by; zero at sources and unreached
// nodes (their values do not follow the update). Also clears the adjoint
// (lam and the scale of its convergence test).
template <typename R>
__global__ __launch_bounds__(256) void k_soft_coef(SoftGrid g, const R *__restrict__ M, const R *__restrict__ om, const R *__restrict__ T,
                            const uint8_t *__restrict__ mark, R tau, R *__restrict__ coef, R *__restrict__ dth,
                            R *__restrict__ lam, R *__restrict__ ctl_scale)
{
    const int64_t n = (int64_t)g.nx * g.ny;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctl_scale = R(0);
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        lam[c] = R(0);
        R cf[8], dt[5];
#pragma unroll
        for (int d = 0; d < 8; ++d) cf[d] = R(0);
#pragma unroll
        for (int a = 0; a < 5; ++a) dt[a] = R(0);
        if (mark[c] != kSource && T[c] < inf_v<R>()) {
            const int i = (int)(c % g.nx), j = (int)(c / g.nx);
            NodeConst<R> k;
            R Tn[8], H[8], w1[8];
            int code[8];
            node_inputs<R>(g, M, om, T, i, j, k, Tn);
            all_stencils<R>(k, Tn, H, code, w1);
            const R v = soft_min<R>(H, tau);
            const R m11 = M[c], m12 = M[n + c], m22 = M[2 * n + c];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                if (!(H[s] < inf_v<R>())) continue;
                const R p = exp((v - H[s]) / tau); // soft-min weight of stencil s
                if (code[s] < 8) {
                    cf[s] += p * w1[s];
                    cf[(s + 1) & 7] += p * (R(1) - w1[s]);
                } else {
                    cf[code[s] - 8] += p;
                }
                R f[5];
                param_derivs<R>(code[s], w1[s], m11, m12, m22, R(g.h), f);
#pragma unroll
                for (int a = 0; a < 5; ++a) dt[a] += p * f[a];
            }
        }
#pragma unroll
        for (int d = 0; d < 8; ++d) coef[d * n + c] = cf[d];
#pragma unroll
        for (int a = 0; a < 5; ++a) dth[a * n + c] = dt[a];
    }
}

// One cycle of the adjoint relaxation lambda_i = g_i + sum_d coef[opp d][nb_d]
// lambda_{nb_d}, with the same line order as the forward (unreached nodes keep
// lambda = 0).
template <typename R>
__global__ __launch_bounds__(kSoftThreads) void k_soft_adj_cycle(SoftGrid g, const R *__restrict__ coef,
                                                                const R *__restrict__ gT, const R *__restrict__ T,
                                                                R *lam, R tol, int32_t *__restrict__ changed,
                                                                R *ctl_scale)
{
    __shared__ int s_changed;
    __shared__ R s_red[kSoftThreads];
    if (threadIdx.x == 0) s_changed = 0;
    const R scale = *ctl_scale;
    __syncthreads();
    const int64_t n = (int64_t)g.nx * g.ny;
    bool ch = false;
    R vmax = R(0);
    for (int dir = 0; dir < 4; ++dir) {
        const int len = dir < 2 ? g.ny : g.nx, span = dir < 2 ? g.nx : g.ny;
        for (int s = 0; s < len; ++s) {
            const int line = (dir & 1) ? len - 1 - s : s;
            R v[kSoftPer];
#pragma unroll
            for (int q = 0; q < kSoftPer; ++q) {
                const int e = threadIdx.x + q * kSoftThreads;
                if (e >= span) continue;
                int i, j;
                line_node(g, dir, line, e, i, j);
                const int64_t c = (int64_t)j * g.nx + i;
                if (!(T[c] < inf_v<R>())) {
                    v[q] = R(0);
                    continue;
                }
                R acc = gT[c];
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const int a = i + nb_dx(d), b = j + nb_dy(d);
                    if (a < 0 || a >= g.nx || b < 0 || b >= g.ny) continue;
                    const int64_t nc = (int64_t)b * g.nx + a;
                    acc += coef[((d + 4) & 7) * n + nc] * lam[nc]; // neighbour's dependence on this node
                }
                v[q] = acc;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kSoftPer; ++q) {
                const int e = threadIdx.x + q * kSoftThreads;
                if (e >= span) continue;
                int i, j;
                line_node(g, dir, line, e, i, j);
                const int64_t c = (int64_t)j * g.nx + i;
                ch |= soft_change<R>(lam[c], v[q], tol, scale);
                vmax = fmax(vmax, fabs(v[q]));
                lam[c] = v[q];
            }
            __syncthreads();
        }
    }
    if (ch) atomicOr(&s_changed, 1);
    vmax = block_max<R>(vmax, s_red);
    if (threadIdx.x == 0) {
        *changed = s_changed;
        *ctl_scale = vmax;
    }
}

// dL/dtheta_i = lambda_i dth_i (zero at sources and unreached nodes: their dth is
// zero), dL/dt_s = lambda_s.
template <typename R>
__global__ void k_soft_params(int64_t n, const R *__restrict__ lam, const R *__restrict__ dth, R *__restrict__ dM,
                              R *__restrict__ dom)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const R l = lam[c];
        dM[c] = l * dth[c];
        dM[n + c] = l * dth[n + c];
        dM[2 * n + c] = l * dth[2 * n + c];
        dom[c] = l * dth[3 * n + c];
        dom[n + c] = l * dth[4 * n + c];
    }
}

template <typename R>
__global__ void k_soft_dsrc(int n_src, const int32_t *__restrict__ src, const R *__restrict__ lam,
                            R *__restrict__ dsrc, int64_t n)
{
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n_src; s += gridDim.x * blockDim.x) {
        const int32_t c = src[s];
        dsrc[s] = (c >= 0 && (int64_t)c < n) ? lam[c] : R(0);
    }
}

static inline unsigned soft_blocks(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 4096); }

template <typename R>
void launch_soft_init(int32_t nx, int32_t ny, int n_src, const int32_t *src, const void *src_t, void *T,
                      uint8_t *mark, int32_t *bad, void *scale, hipStream_t st)
{
    const int64_t n = (int64_t)nx * ny;
    hipLaunchKernelGGL(k_soft_init<R>, dim3(soft_blocks(n)), dim3(256), 0, st, n, (R *)T, mark);
    hipLaunchKernelGGL(k_soft_sources<R>, dim3(1), dim3(256), 0, st, n, n_src, src, (const R *)src_t, (R *)T, mark,
                       bad, (R *)scale);
}

template <typename R>
void launch_soft_cycle(int32_t nx, int32_t ny, double h, const void *M, const void *om, void *T, const uint8_t *mark,
                       double tau, double tol, int32_t *changed, void *scale, hipStream_t st)
{
    const SoftGrid g{nx, ny, h};
    hipLaunchKernelGGL(k_soft_cycle<R>, dim3(1), dim3(kSoftThreads), 0, st, g, (const R *)M, (const R *)om, (R *)T,
                       mark, R(tau), R(tol), changed, (R *)scale);
}

template <typename R>
void launch_soft_coef(int32_t nx, int32_t ny, double h, const void *M, const void *om, const void *T,
                      const uint8_t *mark, double tau, void *coef, void *dth, void *lam, void *scale, hipStream_t st)
{
    const SoftGrid g{nx, ny, h};
    hipLaunchKernelGGL(k_soft_coef<R>, dim3(soft_blocks((int64_t)nx * ny)), dim3(256), 0, st, g, (const R *)M,
                       (const R *)om, (const R *)T, mark, R(tau), (R *)coef, (R *)dth, (R *)lam, (R *)scale);
}

template <typename R>
void launch_soft_adj_cycle(int32_t nx, int32_t ny, const void *coef, const void *gT, const void *T, void *lam,
                           double tol, int32_t *changed, void *scale, hipStream_t st)
{
    const SoftGrid g{nx, ny, 0.0};
    hipLaunchKernelGGL(k_soft_adj_cycle<R>, dim3(1), dim3(kSoftThreads), 0, st, g, (const R *)coef, (const R *)gT,
                       (const R *)T, (R *)lam, R(tol), changed, (R *)scale);
}

template <typename R>
void launch_soft_params(int32_t nx, int32_t ny, int n_src, const int32_t *src, const void *lam, const void *dth,
                        void *dM, void *dom, void *dsrc, hipStream_t st)
{
    const int64_t n = (int64_t)nx * ny;
    hipLaunchKernelGGL(k_soft_params<R>, dim3(soft_blocks(n)), dim3(256), 0, st, n, (const R *)lam, (const R *)dth,
                       (R *)dM, (R *)dom);
    hipLaunchKernelGGL(k_soft_dsrc<R>, dim3(1), dim3(256), 0, st, n_src, src, (const R *)lam, (R *)dsrc, n);
}

#define EIK_SOFT_INST(R)                                                                                           \
    template void launch_soft_init<R>(int32_t, int32_t, int, const int32_t *, const void *, void *, uint8_t *,       \
                                      int32_t *, void *, hipStream_t);                                             \
    template void launch_soft_cycle<R>(int32_t, int32_t, double, const void *, const void *, void *,                \
                                       const uint8_t *, double, double, int32_t *, void *, hipStream_t);           \
    template void launch_soft_coef<R>(int32_t, int32_t, double, const void *, const void *, const void *,            \
                                      const uint8_t *, double, void *, void *, void *, void *, hipStream_t);        \
    template void launch_soft_adj_cycle<R>(int32_t, int32_t, const void *, const void *, const void *, void *,      \
                                           double, int32_t *, void *, hipStream_t);                                \
    template void launch_soft_params<R>(int32_t, int32_t, int, const int32_t *, const void *, const void *, void *, \
                                        void *, void *, hipStream_t);
EIK_SOFT_INST(float)
EIK_SOFT_INST(double)
#undef EIK_SOFT_INST

} // namespace eik
