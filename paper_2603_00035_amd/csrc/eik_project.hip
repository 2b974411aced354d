// eik_project.hip -- feasibility projections and their vector-Jacobian
// product on gfx950 (App. learning details, "Feasibility Projections").
//
// Forward, per node: eigenvalues by the trace-discriminant formula, clamped;
// when a clamp is active the metric is rebuilt as U diag U^T from the clamped
// eigenvalues and the principal angle theta = atan2(2 g12, g11 - g22)/2,
// otherwise it passes unchanged. The drift is clipped in Euclidean norm, then
// rescaled when |b|_{G^-1} exceeds rho_max. The backward pass differentiates
// the same branches analytically (clamps pass gradient on [lo, hi]).
#include <math.h>

#include "eik_device.h"
#include "eik_internal.h"

namespace eik {

template <typename R>
struct ProjBranch {
    R g11, g12, g22;  // input metric
    R dif, disc, lp, lm, lpc, lmc, th, cs, sn;
    bool clamped;
    R n11, n12, n22;  // projected metric
    R b1, b2;         // input drift
    R e, se;          // Euclidean norm and its clip factor
    R c1, c2;         // clipped drift
    R rho, sr;        // G^-1 norm of the clipped drift and its rescale factor
};

__device__ __forceinline__ float d_atan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double d_atan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ void d_sincos(float a, float *s, float *c) { sincosf(a, s, c); }
__device__ __forceinline__ void d_sincos(double a, double *s, double *c) { sincos(a, s, c); }

template <typename R>
__device__ __forceinline__ void proj_forward(R g11, R g12, R g22, R b1, R b2, R lo, R hi, R clip, R rmax,
                                             ProjBranch<R> &p)
{
    p.g11 = g11; p.g12 = g12; p.g22 = g22;
    const R tr = g11 + g22;
    p.dif = g11 - g22;
    p.disc = dsqrt(p.dif * p.dif + R(4) * g12 * g12);
    p.lp = R(0.5) * (tr + p.disc);
    p.lm = R(0.5) * (tr - p.disc);
    p.lpc = fmin(fmax(p.lp, lo), hi);
    p.lmc = fmin(fmax(p.lm, lo), hi);
    p.clamped = (p.lpc != p.lp) || (p.lmc != p.lm);
    if (p.clamped) {
        p.th = R(0.5) * d_atan2(R(2) * g12, p.dif);
        d_sincos(p.th, &p.sn, &p.cs);
        p.n11 = p.lpc * p.cs * p.cs + p.lmc * p.sn * p.sn;
        p.n12 = (p.lpc - p.lmc) * p.cs * p.sn;
        p.n22 = p.lpc * p.sn * p.sn + p.lmc * p.cs * p.cs;
    } else {
        p.n11 = g11; p.n12 = g12; p.n22 = g22;
    }
    p.b1 = b1; p.b2 = b2;
    p.e = dsqrt(b1 * b1 + b2 * b2);
    p.se = p.e > clip ? clip / p.e : R(1);
    p.c1 = b1 * p.se;
    p.c2 = b2 * p.se;
    const R det = p.n11 * p.n22 - p.n12 * p.n12;
    p.rho = dsqrt((p.c1 * p.c1 * p.n22 - R(2) * p.c1 * p.c2 * p.n12 + p.c2 * p.c2 * p.n11) / det);
    p.sr = p.rho > rmax ? rmax / p.rho : R(1);
}

template <typename R>
__global__ void k_project(int64_t n, const R *__restrict__ M, const R *__restrict__ om, R *__restrict__ Mo,
                          R *__restrict__ oo, R lo, R hi, R clip, R rmax)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        ProjBranch<R> p;
        proj_forward<R>(M[c], M[n + c], M[2 * n + c], om[c], om[n + c], lo, hi, clip, rmax, p);
        Mo[c] = p.n11;
        Mo[n + c] = p.n12;
        Mo[2 * n + c] = p.n22;
        oo[c] = p.c1 * p.sr;
        oo[n + c] = p.c2 * p.sr;
    }
}

template <typename R>
__global__ void k_project_backward(int64_t n, const R *__restrict__ M, const R *__restrict__ om,
                                   const R *__restrict__ gMo, const R *__restrict__ goo, R *__restrict__ gM,
                                   R *__restrict__ go, R lo, R hi, R clip, R rmax)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        ProjBranch<R> p;
        proj_forward<R>(M[c], M[n + c], M[2 * n + c], om[c], om[n + c], lo, hi, clip, rmax, p);
        R gn11 = gMo[c], gn12 = gMo[n + c], gn22 = gMo[2 * n + c];
        const R gb1 = goo[c], gb2 = goo[n + c];
        // drift rescale: out = c * rmax / rho(c, N) when rho > rmax
        R gc1 = gb1, gc2 = gb2;
        if (p.rho > rmax) {
            const R det = p.n11 * p.n22 - p.n12 * p.n12;
            const R u1 = (p.n22 * p.c1 - p.n12 * p.c2) / det; // u = N^-1 c
            const R u2 = (p.n11 * p.c2 - p.n12 * p.c1) / det;
            const R gdotc = gb1 * p.c1 + gb2 * p.c2;
            const R r3 = p.rho * p.rho * p.rho;
            gc1 = rmax * (gb1 / p.rho - gdotc * u1 / r3);
            gc2 = rmax * (gb2 / p.rho - gdotc * u2 / r3);
            const R K = rmax * gdotc / (R(2) * r3); // dL/dN = K u u^T
            gn11 += K * u1 * u1;
            gn12 += R(2) * K * u1 * u2;
            gn22 += K * u2 * u2;
        }
        // Euclidean clip: c = b * clip / |b| when |b| > clip
        R gb1i = gc1, gb2i = gc2;
        if (p.e > clip) {
            const R gdotb = gc1 * p.b1 + gc2 * p.b2;
            const R e3 = p.e * p.e * p.e;
            gb1i = clip * (gc1 / p.e - gdotb * p.b1 / e3);
            gb2i = clip * (gc2 / p.e - gdotb * p.b2 / e3);
        }
        go[c] = gb1i;
        go[n + c] = gb2i;
        // metric
        R g11 = gn11, g12 = gn12, g22 = gn22;
        if (p.clamped) {
            const R c2 = p.cs * p.cs, s2 = p.sn * p.sn, csn = p.cs * p.sn;
            const R glpc = gn11 * c2 + gn12 * csn + gn22 * s2;
            const R glmc = gn11 * s2 - gn12 * csn + gn22 * c2;
            const R sin2 = R(2) * csn, cos2 = c2 - s2;
            const R gth = (p.lpc - p.lmc) * (-gn11 * sin2 + gn12 * cos2 + gn22 * sin2);
            const R glp = (p.lp >= lo && p.lp <= hi) ? glpc : R(0);
            const R glm = (p.lm >= lo && p.lm <= hi) ? glmc : R(0);
            const R id = R(1) / p.disc;
            const R id2 = id * id;
            // d lp = (d tr + d disc)/2, d lm = (d tr - d disc)/2, disc^2 = dif^2 + 4 g12^2
            const R ddisc11 = p.dif * id, ddisc22 = -p.dif * id, ddisc12 = R(4) * p.g12 * id;
            g11 = R(0.5) * (glp * (R(1) + ddisc11) + glm * (R(1) - ddisc11)) - gth * p.g12 * id2;
            g22 = R(0.5) * (glp * (R(1) + ddisc22) + glm * (R(1) - ddisc22)) + gth * p.g12 * id2;
            g12 = R(0.5) * (glp - glm) * ddisc12 + gth * p.dif * id2;
        }
        gM[c] = g11;
        gM[n + c] = g12;
        gM[2 * n + c] = g22;
    }
}


template <typename R>
void launch_project(int64_t n, const void *M, const void *om, void *Mo, void *oo, double eig_min, double eig_max,
                    double eucl_clip, double rho_max, hipStream_t st)
{
    hipLaunchKernelGGL(k_project<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, (const R *)M, (const R *)om,
                       (R *)Mo, (R *)oo, R(eig_min), R(eig_max), R(eucl_clip), R(rho_max));
}

template <typename R>
void launch_project_backward(int64_t n, const void *M, const void *om, const void *gMo, const void *goo, void *gM,
                             void *go, double eig_min, double eig_max, double eucl_clip, double rho_max,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_project_backward<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, (const R *)M,
                       (const R *)om, (const R *)gMo, (const R *)goo, (R *)gM, (R *)go, R(eig_min), R(eig_max),
                       R(eucl_clip), R(rho_max));
}

template void launch_project<float>(int64_t, const void *, const void *, void *, void *, double, double, double,
                                    double, hipStream_t);
template void launch_project<double>(int64_t, const void *, const void *, void *, void *, double, double, double,
                                     double, hipStream_t);
template void launch_project_backward<float>(int64_t, const void *, const void *, const void *, const void *,
                                             void *, void *, double, double, double, double, hipStream_t);
template void launch_project_backward<double>(int64_t, const void *, const void *, const void *, const void *,
                                              void *, void *, double, double, double, double, hipStream_t);

} // namespace eik
