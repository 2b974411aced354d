// eik_device.h -- device-side pieces shared by the gfx950 kernels: the
// per-node local update (Sec. 3.2: Eq. two_point, Eq. one_point, validity
// and causality tests of App. solver details) and small helpers.
//
// Every quantity is in grid units: a donor displacement m (receiver minus
// donor) has integer components, E = Mst^T G Mst is the stencil metric of the
// two donors, and for the unimodular stencils used here det E = det G.
// Writing the candidate as T0 = S0 + h tau with S0 the smaller drift-adjusted
// donor time, the quadratic of Eq. two_point multiplied through by det E reads
//   a tau^2 - 2 beta tau + c = 0,  a = |m_p - m_q|_G^2,
//   beta = s1 (E22 - E12) + s2 (E11 - E12),  c = E22 s1^2 + E11 s2^2 - det G,
// where (s1, s2) = (S - S0)/h has one zero entry; the barycentric test
// lambda = Q (T0 1 - S) >= 0 becomes mu = adj(E) (tau 1 - s) >= 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eik {

constexpr uint8_t kSource = 0xFE;
constexpr uint8_t kUnreached = 0xFF;

template <typename R>
__device__ __forceinline__ R inf_v();
template <>
__device__ __forceinline__ float inf_v<float>() { return __builtin_huge_valf(); }
template <>
__device__ __forceinline__ double inf_v<double>() { return __builtin_huge_val(); }

// FP32 uses the hardware square root and reciprocal (about 1 ulp) instead of
// the correctly rounded instruction sequences, which cost ten or more
// instructions each on the sweep's critical path; FP64 keeps the correctly
// rounded forms.
__device__ __forceinline__ float dsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float drcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double drcp(double x) { return 1.0 / x; }

// Neighbour k of (i, j) is (i + nb_dx(k), j + nb_dy(k)), counter-clockwise
// from the upper-left neighbour with +y = +j (Fig. stencil).
__device__ __forceinline__ int nb_dx(int k) { return (k <= 2) ? -1 : ((k == 3 || k == 7) ? 0 : 1); }
__device__ __forceinline__ int nb_dy(int k) { return (k == 0 || k >= 6) ? 1 : ((k == 1 || k == 5) ? 0 : -1); }

// Whether a node's change from a to b keeps the solve going: any change
// between finite and infinite, else |b - a| > tol |b|.
template <typename R>
__device__ __forceinline__ bool counts_as_change(R a, R b, R tol)
{
    if (a == b) return false;
    const R inf = inf_v<R>();
    if (a == inf || b == inf) return true;
    R d = b - a;
    d = d < R(0) ? -d : d;
    const R s = b < R(0) ? -b : b;
    return d > tol * s;
}

// Per-node constants of the 16 candidates.
template <typename R>
struct NodeConst {
    R e[8];    // |m_k|_G^2 for donor k
    R c1[8];   // h (m_k . b + |m_k|_G): one-point increment from donor k
    R hbm[8];  // h m_k . b
    R E12[8];  // m_k^T G m_{k+1}: stencil k cross term
    R a[8];    // |m_{k+1} - m_k|_G^2
    R db[8];   // b . (m_{k+1} - m_k)
    R det, h, inv_h, inv_m11, inv_m22;
};

// The square roots and reciprocals among a node's constants, which depend on
// the metric alone: |(1,0)|_G, |(0,1)|_G, |(1,1)|_G, |(1,-1)|_G, 1/m11, 1/m22.
// The sweeps read them from a copy staged once per solve.
constexpr int kRoots = 6;

template <typename R>
__device__ __forceinline__ void node_roots(R m11, R m12, R m22, R r[kRoots])
{
    const R dp = m11 + R(2) * m12 + m22; // |(1, 1)|_G^2
    const R dm = m11 - R(2) * m12 + m22; // |(1,-1)|_G^2
    r[0] = dsqrt(m11);
    r[1] = dsqrt(m22);
    r[2] = dsqrt(dp);
    r[3] = dsqrt(dm);
    r[4] = drcp(m11);
    r[5] = drcp(m22);
}

// Constants from the metric, the drift and node_roots' values.
template <typename R>
__device__ __forceinline__ void node_const_pre(R m11, R m12, R m22, R bx, R by, const R r[kRoots], R h, R inv_h,
                                               NodeConst<R> &k)
{
    // displacements m_k = -offset_k: (1,-1) (1,0) (1,1) (0,1) (-1,1) (-1,0) (-1,-1) (0,-1)
    const R dp = m11 + R(2) * m12 + m22; // |(1, 1)|_G^2
    const R dm = m11 - R(2) * m12 + m22; // |(1,-1)|_G^2
    const R sx = r[0], sy = r[1], sp = r[2], sm = r[3];
    k.e[0] = dm; k.e[1] = m11; k.e[2] = dp; k.e[3] = m22;
    k.e[4] = dm; k.e[5] = m11; k.e[6] = dp; k.e[7] = m22;
    const R b0 = bx - by, b1 = bx, b2 = bx + by, b3 = by;
    k.hbm[0] = h * b0; k.hbm[1] = h * b1; k.hbm[2] = h * b2; k.hbm[3] = h * b3;
    k.hbm[4] = -k.hbm[0]; k.hbm[5] = -k.hbm[1]; k.hbm[6] = -k.hbm[2]; k.hbm[7] = -k.hbm[3];
    k.c1[0] = h * (b0 + sm); k.c1[1] = h * (b1 + sx); k.c1[2] = h * (b2 + sp); k.c1[3] = h * (b3 + sy);
    k.c1[4] = h * (sm - b0); k.c1[5] = h * (sx - b1); k.c1[6] = h * (sp - b2); k.c1[7] = h * (sy - b3);
    k.E12[0] = m11 - m12; k.E12[1] = m11 + m12; k.E12[2] = m12 + m22; k.E12[3] = m22 - m12;
    k.E12[4] = m11 - m12; k.E12[5] = m11 + m12; k.E12[6] = m12 + m22; k.E12[7] = m22 - m12;
    k.a[0] = m22; k.a[1] = m22; k.a[2] = m11; k.a[3] = m11;
    k.a[4] = m22; k.a[5] = m22; k.a[6] = m11; k.a[7] = m11;
    k.db[0] = by; k.db[1] = by; k.db[2] = -bx; k.db[3] = -bx;
    k.db[4] = -by; k.db[5] = -by; k.db[6] = bx; k.db[7] = bx;
    k.det = m11 * m22 - m12 * m12;
    k.h = h;
    k.inv_h = inv_h;
    k.inv_m11 = r[4];
    k.inv_m22 = r[5];
}

template <typename R>
__device__ __forceinline__ void node_const(R m11, R m12, R m22, R bx, R by, R h, R inv_h, NodeConst<R> &k)
{
    R r[kRoots];
    node_roots<R>(m11, m12, m22, r);
    node_const_pre<R>(m11, m12, m22, bx, by, r, h, inv_h, k);
}

// Two-point candidate of stencil s (donors s and s+1 with times Tp, Tq).
// Returns true when it passes the barycentric and causality tests; t, mu1, mu2
// receive the candidate and the unnormalised barycentric weights.
template <typename R>
__device__ __forceinline__ bool two_point(const NodeConst<R> &k, int s, R Tp, R Tq, R &t, R &mu1, R &mu2)
{
    const int q = (s + 1) & 7;
    const R Ep = k.e[s], Eq = k.e[q], Epq = k.E12[s];
    const R delta = (Tq - Tp) * k.inv_h + k.db[s]; // (S_q - S_p) / h
    const bool base_q = delta < R(0);
    const R s1 = base_q ? -delta : R(0);
    const R s2 = base_q ? R(0) : delta;
    const R S0 = base_q ? Tq + k.hbm[q] : Tp + k.hbm[s];
    const R beta = s1 * (Eq - Epq) + s2 * (Ep - Epq);
    const R c = Eq * s1 * s1 + Ep * s2 * s2 - k.det;
    const R inv_a = (s == 2 || s == 3 || s == 6 || s == 7) ? k.inv_m11 : k.inv_m22;
    const R D = beta * beta - k.a[s] * c;
    if (!(D >= R(0))) return false;
    const R tau = (beta + dsqrt(D)) * inv_a;
    mu1 = Eq * (tau - s1) - Epq * (tau - s2);
    mu2 = Ep * (tau - s2) - Epq * (tau - s1);
    t = S0 + k.h * tau;
    return mu1 >= R(0) && mu2 >= R(0) && t > Tp && t > Tq;
}

// The larger root of stencil s's quadratic and its unnormalised barycentric
// weights, as in two_point but without its validity tests (the soft-min mode
// takes the segment minimum itself). Returns false, leaving the outputs
// unwritten, when the quadratic has no real root.
template <typename R>
__device__ __forceinline__ bool two_point_root(const NodeConst<R> &k, int s, R Tp, R Tq, R &t, R &mu1, R &mu2)
{
    const int q = (s + 1) & 7;
    const R Ep = k.e[s], Eq = k.e[q], Epq = k.E12[s];
    const R delta = (Tq - Tp) * k.inv_h + k.db[s];
    const bool base_q = delta < R(0);
    const R s1 = base_q ? -delta : R(0);
    const R s2 = base_q ? R(0) : delta;
    const R S0 = base_q ? Tq + k.hbm[q] : Tp + k.hbm[s];
    const R beta = s1 * (Eq - Epq) + s2 * (Ep - Epq);
    const R c = Eq * s1 * s1 + Ep * s2 * s2 - k.det;
    const R inv_a = (s == 2 || s == 3 || s == 6 || s == 7) ? k.inv_m11 : k.inv_m22;
    const R D = beta * beta - k.a[s] * c;
    if (!(D >= R(0))) return false;
    const R tau = (beta + dsqrt(D)) * inv_a;
    mu1 = Eq * (tau - s1) - Epq * (tau - s2);
    mu2 = Ep * (tau - s2) - Epq * (tau - s1);
    t = S0 + k.h * tau;
    return true;
}

// two_point for a stencil index known only at run time: one constant-index
// call per case, so the per-node constants stay in registers (an indexed
// access into them would go through scratch memory).
template <typename R>
__device__ __forceinline__ bool two_point_any(const NodeConst<R> &k, int s, R Tp, R Tq, R &t, R &mu1, R &mu2)
{
    switch (s & 7) {
    case 0: return two_point(k, 0, Tp, Tq, t, mu1, mu2);
    case 1: return two_point(k, 1, Tp, Tq, t, mu1, mu2);
    case 2: return two_point(k, 2, Tp, Tq, t, mu1, mu2);
    case 3: return two_point(k, 3, Tp, Tq, t, mu1, mu2);
    case 4: return two_point(k, 4, Tp, Tq, t, mu1, mu2);
    case 5: return two_point(k, 5, Tp, Tq, t, mu1, mu2);
    case 6: return two_point(k, 6, Tp, Tq, t, mu1, mu2);
    default: return two_point(k, 7, Tp, Tq, t, mu1, mu2);
    }
}

// Minimum over the valid candidates (two-point stencils 0..7 first, then
// one-point donors 0..7; the first minimum wins). Donors must be finite and,
// when strict_ref is finite, strictly below strict_ref. code receives the
// winner (0..15) or kUnreached, w1 the weight of the stencil's first donor.
template <typename R>
__device__ __forceinline__ R local_update(const NodeConst<R> &k, const R Tn[8], R strict_ref, int &code, R &w1)
{
    const R inf = inf_v<R>();
    R best = inf;
    code = kUnreached;
    w1 = R(1);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const R Tp = Tn[s], Tq = Tn[(s + 1) & 7];
        if (Tp < strict_ref && Tq < strict_ref) {
            R t, m1, m2;
            if (two_point(k, s, Tp, Tq, t, m1, m2) && t < best) {
                best = t;
                code = s;
                w1 = m1 / (m1 + m2);
            }
        }
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        if (Tn[s] < strict_ref) {
            const R t = Tn[s] + k.c1[s];
            if (t < best) {
                best = t;
                code = 8 + s;
                w1 = R(1);
            }
        }
    }
    return best;
}

// Candidates of one sweep direction (the line sweep steps along +x, +y, -x,
// -y for DIR = 0, 1, 2, 3). FULL: every candidate in the canonical order
// (two-point 0..7, then one-point 0..7; first minimum wins). Otherwise only
// the candidates whose donors all sit on the line just updated: donors
// 2 DIR, 2 DIR + 1, 2 DIR + 2 (mod 8) and the two stencils between them. Each
// stencil then belongs to exactly one direction, the one that sweeps its
// donors' line just before the node's, and each donor to one or two; the four
// directions together cover every candidate, so a field no direction can
// lower is a fixed point of the full update's minimum.
template <typename R, int DIR, bool FULL>
__device__ __forceinline__ R local_update_dir(const NodeConst<R> &k, const R Tn[8], int &code)
{
    const R inf = inf_v<R>();
    R best = inf;
    code = kUnreached;
    if (FULL) {
        // One-point candidates first. A valid two-point value exceeds both of
        // its donors, so a stencil whose donors are not both below the best
        // one-point value can neither beat nor tie it and is skipped; the
        // value and code returned are those of the canonical order (two-point
        // wins ties with one-point, lower index wins within a kind).
        R b1 = inf;
        int c1 = kUnreached;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const R t = Tn[s] + k.c1[s]; // +inf for an unreached donor, never below b1
            if (t < b1) {
                b1 = t;
                c1 = 8 + s;
            }
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const R Tp = Tn[s], Tq = Tn[(s + 1) & 7];
            if (Tp < b1 && Tq < b1) {
                R t, m1, m2;
                if (two_point(k, s, Tp, Tq, t, m1, m2) && t < best) {
                    best = t;
                    code = s;
                }
            }
        }
        if (!(best <= b1)) {
            best = b1;
            code = c1;
        }
    } else {
        // restricted candidates of direction DIR, with the same one-point-first
        // pruning and the same canonical order as the full update
        R b1 = inf;
        int c1 = kUnreached;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int s = (2 * DIR + q) & 7;
            const R t = Tn[s] + k.c1[s]; // +inf for an unreached donor
            if (t < b1) {
                b1 = t;
                c1 = 8 + s;
            }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int s = (2 * DIR + q) & 7;
            const R Tp = Tn[s], Tq = Tn[(s + 1) & 7];
            if (Tp < b1 && Tq < b1) {
                R t, m1, m2;
                if (two_point(k, s, Tp, Tq, t, m1, m2) && t < best) {
                    best = t;
                    code = s;
                }
            }
        }
        if (!(best <= b1)) {
            best = b1;
            code = c1;
        }
    }
    return best;
}

// Local derivatives of an active update (envelope form of the residual
// partials, Eqs. two_point_partials and one_point_partials): with donor
// weights (w1, 1 - w1) and v = w1 m_p + (1 - w1) m_q (v = m_k for a one-point
// update), dT/db = h v and dT/dG = h v v^T / (2 |v|_G). Returns the factors
// with respect to the stored m11, m12, m22, bx, by.
template <typename R>
__device__ __forceinline__ void param_derivs(int code, R w1, R m11, R m12, R m22, R h, R out[5])
{
    int kp, kq;
    R wp, wq;
    if (code < 8) {
        kp = code;
        kq = (code + 1) & 7;
        wp = w1;
        wq = R(1) - w1;
    } else {
        kp = kq = code - 8;
        wp = R(1);
        wq = R(0);
    }
    const R vx = -(wp * R(nb_dx(kp)) + wq * R(nb_dx(kq)));
    const R vy = -(wp * R(nb_dy(kp)) + wq * R(nb_dy(kq)));
    const R nv = dsqrt(m11 * vx * vx + R(2) * m12 * vx * vy + m22 * vy * vy);
    const R f = h / (R(2) * nv);
    out[0] = f * vx * vx;
    out[1] = R(2) * f * vx * vy;
    out[2] = f * vy * vy;
    out[3] = h * vx;
    out[4] = h * vy;
}

} // namespace eik
