// unet.hip -- BF16 MFMA kernels of the learned warm start (gfx950).
//
// The convolutions are implicit GEMMs on v_mfma_f32_16x16x16bf16: the M
// dimension runs over pixels (NHWC, batch folded in), N over output channels,
// K over (tap, input channel). A 64-lane wave owns 16 pixels x 16*NT output
// channels; each lane feeds 4 consecutive channels of one pixel (8-byte load)
// and 4 consecutive input channels of one output channel's weights, and the
// accumulators stay in FP32. The weight gradient is the GEMM with K running
// over pixels: one wave per (pixel chunk, tap, 16x16 channel tile), partial
// sums added into FP32 gradients with atomics.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/eik_unet.h"

namespace eiku {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16;

__device__ __forceinline__ float bf2f(bf16 v) { return __uint_as_float((uint32_t)v << 16); }

// round to nearest even (NaN kept quiet)
__device__ __forceinline__ bf16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}

__device__ __forceinline__ s4 load4(const bf16 *p)
{
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    s4 r;
    r[0] = (short)(v.x & 0xffff);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xffff);
    r[3] = (short)(v.y >> 16);
    return r;
}

struct ConvArgs {
    const bf16 *x;
    const bf16 *w;
    const float *bias;
    bf16 *y;
    int x_cs, x_co, y_cs, y_co;
    int B, H, W, Cin, Cout, relu;
};

template <int MODE, int NT>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t npix = (int64_t)a.B * a.H * a.W;
    const int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    if (p0 >= npix) return; // no workgroup barrier below
    const int co0 = blockIdx.y * 16 * NT;
    const int r = lane & 15, kq = lane >> 4;
    int64_t pa = p0 + r;
    const bool va = pa < npix;
    if (!va) pa = npix - 1;
    const int xx = (int)(pa % a.W);
    const int64_t tt = pa / a.W;
    const int yy = (int)(tt % a.H);
    const int bb = (int)(tt / a.H);
    f4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
    const s4 zero = s4{0, 0, 0, 0};
    constexpr int NTAP = MODE == EIKU_CONV3 ? 9 : (MODE == EIKU_UP2 ? 1 : 4);
    for (int ti = 0; ti < NTAP; ++ti) {
        const int tap = MODE == EIKU_UP2 ? (int)blockIdx.z : ti;
        int64_t pin = pa;
        bool v = va;
        if (MODE == EIKU_CONV3) {
            const int sy = yy + tap / 3 - 1, sx = xx + tap % 3 - 1;
            v = v && sy >= 0 && sy < a.H && sx >= 0 && sx < a.W;
            pin = ((int64_t)bb * a.H + sy) * a.W + sx;
        } else if (MODE == EIKU_DOWN2) {
            const int sy = 2 * yy + (tap >> 1), sx = 2 * xx + (tap & 1);
            pin = ((int64_t)bb * 2 * a.H + sy) * (2 * a.W) + sx;
        }
        const bf16 *xr = a.x + (v ? pin : 0) * a.x_cs + a.x_co + 4 * kq;
        const bf16 *wr = a.w + ((int64_t)tap * a.Cout + co0 + r) * a.Cin + 4 * kq;
        for (int cb = 0; cb < a.Cin; cb += 16) {
            const s4 av = v ? load4(xr + cb) : zero;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const s4 bv = load4(wr + (int64_t)nt * 16 * a.Cin + cb);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[nt], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int col = co0 + nt * 16 + r;
        const float bias = a.bias ? a.bias[col] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t po = p0 + 4 * kq + i;
            if (po >= npix) continue;
            float val = acc[nt][i] + bias;
            if (a.relu) val = fmaxf(val, 0.f);
            int64_t pout = po;
            if (MODE == EIKU_UP2) {
                const int ox = (int)(po % a.W);
                const int64_t ot = po / a.W;
                const int oy = (int)(ot % a.H), ob = (int)(ot / a.H);
                const int tap = (int)blockIdx.z;
                pout = ((int64_t)ob * 2 * a.H + 2 * oy + (tap >> 1)) * (2 * a.W) + 2 * ox + (tap & 1);
            }
            a.y[pout * a.y_cs + a.y_co + col] = f2bf(val);
        }
    }
}

struct WgradArgs {
    const bf16 *x;
    const bf16 *dy;
    float *dw;
    int x_cs, x_co, dy_cs, dy_co;
    int B, H, W, Cin, Cout;
    int64_t chunk;
};

template <int MODE>
__global__ __launch_bounds__(64) void k_wgrad(WgradArgs a)
{
    const int lane = threadIdx.x;
    const int r = lane & 15, kq = lane >> 4;
    const int nco = a.Cout / 16, nci = a.Cin / 16;
    const int combo = blockIdx.y;
    const int tap = combo / (nco * nci);
    const int rem = combo - tap * nco * nci;
    const int co0 = (rem / nci) * 16, ci0 = (rem % nci) * 16;
    const int64_t npix = (int64_t)a.B * a.H * a.W;
    const int64_t pb = (int64_t)blockIdx.x * a.chunk;
    const int64_t pe = pb + a.chunk < npix ? pb + a.chunk : npix;
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    for (int64_t p = pb; p < pe; p += 16) {
        s4 av, bv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t pk = p + 4 * kq + j;
            const bool v = pk < pe;
            const int64_t pc = v ? pk : pb;
            const int xx = (int)(pc % a.W);
            const int64_t tt = pc / a.W;
            const int yy = (int)(tt % a.H), bb = (int)(tt / a.H);
            int64_t pdy = pc, pin = pc;
            bool vin = v;
            if (MODE == EIKU_CONV3) {
                const int sy = yy + tap / 3 - 1, sx = xx + tap % 3 - 1;
                vin = vin && sy >= 0 && sy < a.H && sx >= 0 && sx < a.W;
                pin = ((int64_t)bb * a.H + sy) * a.W + sx;
            } else { // EIKU_UP2: x on this grid, dy on the doubled grid
                pdy = ((int64_t)bb * 2 * a.H + 2 * yy + (tap >> 1)) * (2 * a.W) + 2 * xx + (tap & 1);
            }
            av[j] = v ? (short)a.dy[pdy * a.dy_cs + a.dy_co + co0 + r] : (short)0;
            bv[j] = vin ? (short)a.x[pin * a.x_cs + a.x_co + ci0 + r] : (short)0;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
        atomicAdd(&a.dw[((int64_t)tap * a.Cout + co0 + 4 * kq + i) * a.Cin + ci0 + r], acc[i]);
}

// ---------------------------------------------------------------------------
// Elementwise and small kernels.
// ---------------------------------------------------------------------------
// db[c] += sum over pixels of dy(p, c). A block of 256 threads takes a chunk
// of kBiasChunk pixels as R = 256 / C pixel lanes times C channels (reads of
// one pixel's channels are contiguous), adds the lanes in shared memory, and
// adds one value per channel to db.
constexpr int kBiasChunk = 128;
__global__ __launch_bounds__(256) void k_bias_grad(int64_t npix, const bf16 *__restrict__ dy, int cs, int co, int C,
                                                   float *__restrict__ db)
{
    __shared__ float sh[256];
    const int t = threadIdx.x, R = 256 / C;
    const int c = t % C, r = t / C;
    float s = 0.f;
    if (r < R) {
        const int64_t pb = (int64_t)blockIdx.x * kBiasChunk;
        const int64_t pe = pb + kBiasChunk < npix ? pb + kBiasChunk : npix;
        for (int64_t p = pb + r; p < pe; p += R) s += bf2f(dy[p * cs + co + c]);
    }
    sh[t] = s;
    __syncthreads();
    if (t < C) {
        float tot = 0.f;
        for (int k = 0; k < R; ++k) tot += sh[k * C + t];
        atomicAdd(&db[t], tot);
    }
}

__global__ void k_relu_mask(int64_t n, const bf16 *__restrict__ y, int ycs, int yco, bf16 *__restrict__ g, int gcs,
                            int gco, int C)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * C; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / C;
        const int c = (int)(e - p * C);
        if (!(bf2f(y[p * ycs + yco + c]) > 0.f)) g[p * gcs + gco + c] = 0;
    }
}

__global__ void k_add(int64_t n, bf16 *__restrict__ a, int acs, int aco, const bf16 *__restrict__ b, int bcs, int bco,
                      int C)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * C; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / C;
        const int c = (int)(e - p * C);
        bf16 &t = a[p * acs + aco + c];
        t = f2bf(bf2f(t) + bf2f(b[p * bcs + bco + c]));
    }
}

__global__ void k_maxpool_fwd(int B, int H, int W, const bf16 *__restrict__ x, int xcs, int xco, bf16 *__restrict__ y,
                              int ycs, int yco, int C)
{
    const int64_t n = (int64_t)B * H * W * C;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const int64_t p = e / C;
        const int xo = (int)(p % W);
        const int64_t t = p / W;
        const int yo = (int)(t % H), b = (int)(t / H);
        float m = -INFINITY;
        for (int q = 0; q < 4; ++q) {
            const int64_t pi = ((int64_t)b * 2 * H + 2 * yo + (q >> 1)) * (2 * W) + 2 * xo + (q & 1);
            m = fmaxf(m, bf2f(x[pi * xcs + xco + c]));
        }
        y[p * ycs + yco + c] = f2bf(m);
    }
}

__global__ void k_maxpool_bwd(int B, int H, int W, const bf16 *__restrict__ x, int xcs, int xco,
                              const bf16 *__restrict__ dy, int dycs, int dyco, bf16 *__restrict__ dx, int dxcs,
                              int dxco, int C)
{
    const int64_t n = (int64_t)B * H * W * C;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const int64_t p = e / C;
        const int xo = (int)(p % W);
        const int64_t t = p / W;
        const int yo = (int)(t % H), b = (int)(t / H);
        float m = -INFINITY;
        int arg = 0;
        for (int q = 0; q < 4; ++q) {
            const int64_t pi = ((int64_t)b * 2 * H + 2 * yo + (q >> 1)) * (2 * W) + 2 * xo + (q & 1);
            const float v = bf2f(x[pi * xcs + xco + c]);
            if (v > m) {
                m = v;
                arg = q;
            }
        }
        const bf16 g = dy[p * dycs + dyco + c];
        for (int q = 0; q < 4; ++q) {
            const int64_t pi = ((int64_t)b * 2 * H + 2 * yo + (q >> 1)) * (2 * W) + 2 * xo + (q & 1);
            dx[pi * dxcs + dxco + c] = q == arg ? g : (bf16)0;
        }
    }
}

__global__ void k_head_fwd(int64_t n, const bf16 *__restrict__ x, int cs, int co, int C, const float *__restrict__ w,
                           const float *__restrict__ b, float *__restrict__ out)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        float s = b[0];
        for (int c = 0; c < C; ++c) s += w[c] * bf2f(x[p * cs + co + c]);
        out[p] = s;
    }
}

__global__ void k_head_bwd(int64_t n, const bf16 *__restrict__ x, int cs, int co, int C, const float *__restrict__ w,
                           const float *__restrict__ g, bf16 *__restrict__ dx, int dxcs, int dxco,
                           float *__restrict__ dw, float *__restrict__ db)
{
    float sdw[16] = {0.f};
    float sdb = 0.f;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const float gp = g[p];
        sdb += gp;
        for (int c = 0; c < C && c < 16; ++c) {
            dx[p * dxcs + dxco + c] = f2bf(w[c] * gp);
            sdw[c] += gp * bf2f(x[p * cs + co + c]);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        sdb += __shfl_xor(sdb, off);
        for (int c = 0; c < 16; ++c) sdw[c] += __shfl_xor(sdw[c], off);
    }
    // the block's waves add their sums in shared memory; one atomic per value
    // and block (instead of per wave) keeps the contention on the 17 targets low
    __shared__ float sw[4][17];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        for (int c = 0; c < 16; ++c) sw[wv][c] = sdw[c];
        sw[wv][16] = sdb;
    }
    __syncthreads();
    if (threadIdx.x < 17) {
        const int c = threadIdx.x;
        const float v = sw[0][c] + sw[1][c] + sw[2][c] + sw[3][c];
        if (c == 16)
            atomicAdd(db, v);
        else if (c < C)
            atomicAdd(&dw[c], v);
    }
}

__global__ void k_features(int B, int H, int W, const float *__restrict__ M, const float *__restrict__ om,
                           const int32_t *__restrict__ src, int max_src, const float *__restrict__ h,
                           bf16 *__restrict__ x, float *__restrict__ dist)
{
    const int64_t n = (int64_t)B * H * W;
    const int64_t plane = (int64_t)H * W;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(p / plane);
        const int64_t q = p - (int64_t)b * plane;
        const int i = (int)(q % W), j = (int)(q / W);
        float d2 = INFINITY;
        for (int s = 0; s < max_src; ++s) {
            const int c = src[b * max_src + s];
            if (c < 0) continue;
            const float dx = (float)(i - c % W), dy = (float)(j - c / W);
            d2 = fminf(d2, dx * dx + dy * dy);
        }
        const float d = sqrtf(d2) * h[b];
        const float *Mb = M + (int64_t)b * 3 * plane;
        const float *ob = om + (int64_t)b * 2 * plane;
        bf16 *xp = x + p * 16;
        xp[0] = f2bf(Mb[q]);
        xp[1] = f2bf(Mb[plane + q]);
        xp[2] = f2bf(Mb[2 * plane + q]);
        xp[3] = f2bf(ob[q]);
        xp[4] = f2bf(ob[plane + q]);
        xp[5] = f2bf(d);
        for (int c = 6; c < 16; ++c) xp[c] = 0;
        if (dist) dist[p] = d;
    }
}

__global__ void k_mse(int64_t n, const float *__restrict__ pred, const float *__restrict__ tgt,
                      float *__restrict__ loss, float *__restrict__ grad)
{
    float s = 0.f;
    const float inv = 1.f / (float)n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float d = pred[e] - tgt[e];
        s += d * d;
        grad[e] = 2.f * d * inv;
    }
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, s * inv);
}

__global__ void k_adam(int64_t n, float *__restrict__ p, float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float gr = g[e];
        const float mm = b1 * m[e] + (1.f - b1) * gr;
        const float vv = b2 * v[e] + (1.f - b2) * gr * gr;
        m[e] = mm;
        v[e] = vv;
        p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
        g[e] = 0.f;
    }
}

__global__ void k_prep_weights(int mode, int taps, int Cout, int Cin, int cin_real, const float *__restrict__ w32,
                               bf16 *__restrict__ wf, bf16 *__restrict__ wb)
{
    const int64_t n = (int64_t)taps * Cout * Cin;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(e % Cin);
        const int64_t t1 = e / Cin;
        const int co = (int)(t1 % Cout);
        const int tap = (int)(t1 / Cout);
        const float v = ci < cin_real ? w32[((int64_t)tap * Cout + co) * cin_real + ci] : 0.f;
        const bf16 bv = f2bf(v);
        wf[e] = bv;
        if (wb) {
            const int tb = mode == EIKU_CONV3 ? 8 - tap : tap; // mirrored taps for the 3x3 data gradient
            wb[((int64_t)tb * Cin + ci) * Cout + co] = bv;
        }
    }
}

__global__ void k_to_bf16(int64_t n, const float *__restrict__ x, bf16 *__restrict__ y)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = f2bf(x[e]);
}

__global__ void k_to_f32(int64_t n, const bf16 *__restrict__ x, float *__restrict__ y)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = bf2f(x[e]);
}

static inline int gblocks(int64_t n, int bs) { return (int)std::min<int64_t>((n + bs - 1) / bs, 16384); }

} // namespace eiku

using namespace eiku;

extern "C" {

int eiku_conv_fwd(int32_t mode, int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t x_cs, int32_t x_co,
                  int32_t Cin, const uint16_t *w, const float *bias, int32_t relu, uint16_t *y, int32_t y_cs,
                  int32_t y_co, int32_t Cout, hipStream_t st)
{
    if (B < 1 || H < 1 || W < 1 || Cin < 16 || Cin % 16 || Cout < 16 || Cout % 16 || !x || !w || !y) return -1;
    if ((x_cs | x_co | y_co) % 4 || x_co + Cin > x_cs || y_co + Cout > y_cs) return -1;
    if (mode != EIKU_CONV3 && mode != EIKU_UP2 && mode != EIKU_DOWN2) return -1;
    ConvArgs a{x, w, bias, y, x_cs, x_co, y_cs, y_co, B, H, W, Cin, Cout, relu};
    const int64_t npix = (int64_t)B * H * W;
    const int nt = Cout % 64 == 0 ? 4 : (Cout % 32 == 0 ? 2 : 1);
    dim3 grid((unsigned)((npix + 63) / 64), (unsigned)(Cout / (16 * nt)), mode == EIKU_UP2 ? 4 : 1);
#define EIKU_LAUNCH(MODE)                                                                                 \
    do {                                                                                                  \
        if (nt == 4) hipLaunchKernelGGL((k_conv<MODE, 4>), grid, dim3(256), 0, st, a);                    \
        else if (nt == 2) hipLaunchKernelGGL((k_conv<MODE, 2>), grid, dim3(256), 0, st, a);               \
        else hipLaunchKernelGGL((k_conv<MODE, 1>), grid, dim3(256), 0, st, a);                            \
    } while (0)
    if (mode == EIKU_CONV3) EIKU_LAUNCH(EIKU_CONV3);
    else if (mode == EIKU_UP2) EIKU_LAUNCH(EIKU_UP2);
    else EIKU_LAUNCH(EIKU_DOWN2);
#undef EIKU_LAUNCH
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_conv_wgrad(int32_t mode, int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t x_cs, int32_t x_co,
                    int32_t Cin, const uint16_t *dy, int32_t dy_cs, int32_t dy_co, int32_t Cout, float *dw,
                    hipStream_t st)
{
    if (B < 1 || H < 1 || W < 1 || Cin < 16 || Cin % 16 || Cout < 16 || Cout % 16 || !x || !dy || !dw) return -1;
    if (x_co + Cin > x_cs || dy_co + Cout > dy_cs) return -1;
    if (mode != EIKU_CONV3 && mode != EIKU_UP2) return -1;
    const int64_t npix = (int64_t)B * H * W;
    int64_t chunk = npix / 128;
    chunk = chunk < 256 ? 256 : (chunk > 8192 ? 8192 : chunk);
    chunk = (chunk + 15) / 16 * 16;
    WgradArgs a{x, dy, dw, x_cs, x_co, dy_cs, dy_co, B, H, W, Cin, Cout, chunk};
    const int taps = mode == EIKU_CONV3 ? 9 : 4;
    dim3 grid((unsigned)((npix + chunk - 1) / chunk), (unsigned)(taps * (Cout / 16) * (Cin / 16)));
    if (mode == EIKU_CONV3) hipLaunchKernelGGL(k_wgrad<EIKU_CONV3>, grid, dim3(64), 0, st, a);
    else hipLaunchKernelGGL(k_wgrad<EIKU_UP2>, grid, dim3(64), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_bias_grad(int64_t npix, const uint16_t *dy, int32_t cs, int32_t co, int32_t C, float *db, hipStream_t st)
{
    if (npix < 1 || C < 1 || C > 256 || !dy || !db || co + C > cs) return -1;
    hipLaunchKernelGGL(k_bias_grad, dim3((unsigned)((npix + kBiasChunk - 1) / kBiasChunk)), dim3(256), 0, st, npix, dy,
                       cs, co, C, db);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_relu_mask(int64_t npix, const uint16_t *y, int32_t y_cs, int32_t y_co, uint16_t *g, int32_t g_cs,
                   int32_t g_co, int32_t C, hipStream_t st)
{
    if (npix < 1 || C < 1 || !y || !g || y_co + C > y_cs || g_co + C > g_cs) return -1;
    hipLaunchKernelGGL(k_relu_mask, dim3(gblocks(npix * C, 256)), dim3(256), 0, st, npix, y, y_cs, y_co, g, g_cs,
                       g_co, C);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_add(int64_t npix, uint16_t *a, int32_t a_cs, int32_t a_co, const uint16_t *b, int32_t b_cs, int32_t b_co,
             int32_t C, hipStream_t st)
{
    if (npix < 1 || C < 1 || !a || !b || a_co + C > a_cs || b_co + C > b_cs) return -1;
    hipLaunchKernelGGL(k_add, dim3(gblocks(npix * C, 256)), dim3(256), 0, st, npix, a, a_cs, a_co, b, b_cs, b_co, C);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_maxpool_fwd(int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t x_cs, int32_t x_co, uint16_t *y,
                     int32_t y_cs, int32_t y_co, int32_t C, hipStream_t st)
{
    if (B < 1 || H < 1 || W < 1 || C < 1 || !x || !y || x_co + C > x_cs || y_co + C > y_cs) return -1;
    hipLaunchKernelGGL(k_maxpool_fwd, dim3(gblocks((int64_t)B * H * W * C, 256)), dim3(256), 0, st, B, H, W, x, x_cs,
                       x_co, y, y_cs, y_co, C);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_maxpool_bwd(int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t x_cs, int32_t x_co,
                     const uint16_t *dy, int32_t dy_cs, int32_t dy_co, uint16_t *dx, int32_t dx_cs, int32_t dx_co,
                     int32_t C, hipStream_t st)
{
    if (B < 1 || H < 1 || W < 1 || C < 1 || !x || !dy || !dx || x_co + C > x_cs || dy_co + C > dy_cs ||
        dx_co + C > dx_cs)
        return -1;
    hipLaunchKernelGGL(k_maxpool_bwd, dim3(gblocks((int64_t)B * H * W * C, 256)), dim3(256), 0, st, B, H, W, x, x_cs,
                       x_co, dy, dy_cs, dy_co, dx, dx_cs, dx_co, C);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_head_fwd(int64_t npix, const uint16_t *x, int32_t cs, int32_t co, int32_t C, const float *w, const float *b,
                  float *out, hipStream_t st)
{
    if (npix < 1 || C < 1 || C > 16 || !x || !w || !b || !out || co + C > cs) return -1;
    hipLaunchKernelGGL(k_head_fwd, dim3(gblocks(npix, 256)), dim3(256), 0, st, npix, x, cs, co, C, w, b, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_head_bwd(int64_t npix, const uint16_t *x, int32_t cs, int32_t co, int32_t C, const float *w, const float *g,
                  uint16_t *dx, int32_t dx_cs, int32_t dx_co, float *dw, float *db, hipStream_t st)
{
    if (npix < 1 || C < 1 || C > 16 || !x || !w || !g || !dx || !dw || !db || co + C > cs || dx_co + C > dx_cs)
        return -1;
    hipLaunchKernelGGL(k_head_bwd, dim3(gblocks(npix, 256)), dim3(256), 0, st, npix, x, cs, co, C, w, g, dx, dx_cs,
                       dx_co, dw, db);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_features(int32_t B, int32_t H, int32_t W, const float *M, const float *omega, const int32_t *src,
                  int32_t max_src, const float *h, uint16_t *x, float *dist, hipStream_t st)
{
    if (B < 1 || H < 1 || W < 1 || max_src < 1 || !M || !omega || !src || !h || !x) return -1;
    hipLaunchKernelGGL(k_features, dim3(gblocks((int64_t)B * H * W, 256)), dim3(256), 0, st, B, H, W, M, omega, src,
                       max_src, h, x, dist);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_mse(int64_t n, const float *pred, const float *target, float *loss, float *grad, hipStream_t st)
{
    if (n < 1 || !pred || !target || !loss || !grad) return -1;
    hipLaunchKernelGGL(k_mse, dim3(gblocks(n, 256)), dim3(256), 0, st, n, pred, target, loss, grad);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_adam(int64_t n, float *param, float *grad, float *m, float *v, float lr, float beta1, float beta2, float eps,
              int32_t t, hipStream_t st)
{
    if (n < 1 || t < 1 || !param || !grad || !m || !v) return -1;
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(gblocks(n, 256)), dim3(256), 0, st, n, param, grad, m, v, lr, beta1, beta2, eps,
                       c1, c2);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_prep_weights(int32_t mode, int32_t taps, int32_t Cout, int32_t Cin, int32_t cin_real, const float *w32,
                      uint16_t *wfwd, uint16_t *wbwd, hipStream_t st)
{
    if (taps < 1 || Cout < 1 || Cin < cin_real || cin_real < 1 || !w32 || !wfwd) return -1;
    if (wbwd && ((mode == EIKU_CONV3 && taps != 9) || (mode == EIKU_UP2 && taps != 4))) return -1;
    hipLaunchKernelGGL(k_prep_weights, dim3(gblocks((int64_t)taps * Cout * Cin, 256)), dim3(256), 0, st, mode, taps,
                       Cout, Cin, cin_real, w32, wfwd, wbwd);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_to_bf16(int64_t n, const float *x, uint16_t *y, hipStream_t st)
{
    if (n < 1 || !x || !y) return -1;
    hipLaunchKernelGGL(k_to_bf16, dim3(gblocks(n, 256)), dim3(256), 0, st, n, x, y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_to_f32(int64_t n, const uint16_t *x, float *y, hipStream_t st)
{
    if (n < 1 || !x || !y) return -1;
    hipLaunchKernelGGL(k_to_f32, dim3(gblocks(n, 256)), dim3(256), 0, st, n, x, y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

} // extern "C"
