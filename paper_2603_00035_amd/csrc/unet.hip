// unet.hip -- BF16 MFMA kernels of the learned warm start (gfx950).
//
// The convolutions are implicit GEMMs over output channels x pixels (NHWC,
// batch folded in) with K over (tap, input channel), accumulated in FP32.
// k_conv_lds (3x3 convolution, 2x2 transposed convolution and its data
// gradient, the 2x2 stride-2 convolution): a workgroup owns one or two 8 x 32
// tiles of output pixels (of input pixels for the transposed convolution),
// taken in turn, and 16 NT output channels. Per slice of KC input channels it
// stages the tile's input patch and the slice of the weights in LDS, loads of
// the next slice (or tile) in flight while the current one is used; the 3x3
// convolution can read a concatenation from two buffers, one source per
// slice. Each wave runs 2 rows x 32 pixels through
// v_mfma_f32_16x16x32_bf16 (v_mfma_f32_16x16x16_bf16 for 16-channel slices),
// weights as the A operand and pixels as B, so a lane ends up with 4
// consecutive channels of one pixel and stores them as one 8-byte word.
// The weight gradients are GEMMs with K running over pixels: k_wgrad3_lds
// stages pixel tiles of dy and x in LDS transposed to channel-major rows;
// k_wgrad_up2 (transposed convolution) reads its operands from global memory.
// Partial sums go to the FP32 gradients with atomics.
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

// Input channels c < csplit come from x (channel x_co + c), the rest from x2
// (channel x2_co + c - csplit): a concatenation read from its two producers'
// own buffers (the kernels' CAT forms; one source: x2 = x and csplit = Cin).
// tpw: pixel tiles per workgroup, taken one after another with the next
// tile's loads in flight while the current one is computed.
struct ConvArgs {
    const bf16 *x;
    const bf16 *w;
    const float *bias;
    bf16 *y;
    int x_cs, x_co, y_cs, y_co;
    int B, H, W, Cin, Cout, relu;
    const bf16 *x2;
    int x2_cs, x2_co, csplit;
    int tpw;
};

// Address of the 8 channels c .. c+7 of pixel pix of a two-source input
// (csplit is a multiple of 16, so the 8 channels come from one source).
__device__ __forceinline__ const bf16 *src8(const bf16 *x, int x_cs, int x_co, const bf16 *x2, int x2_cs, int x2_co,
                                            int csplit, int64_t pix, int c)
{
    return c < csplit ? x + pix * x_cs + x_co + c : x2 + pix * x2_cs + x2_co + (c - csplit);
}

// ---------------------------------------------------------------------------
// LDS-staged convolution (EIKU_CONV3, EIKU_UP2).
// ---------------------------------------------------------------------------
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kTileY = 8, kTileX = 32; // pixels per workgroup: 4 waves x 2 rows x 32 columns

// Patch geometry per mode: EIKU_CONV3 reads the output tile plus a one-pixel
// halo, EIKU_UP2 the input tile itself (its pixel grid is the input's), and
// EIKU_DOWN2 the 2x finer input region under the output tile.
template <int MODE, int KC, int NT> struct LdsConv {
    static constexpr int HALO = MODE == EIKU_CONV3 ? 1 : 0;
    static constexpr int SCALE = MODE == EIKU_DOWN2 ? 2 : 1;
    static constexpr int PY = SCALE * kTileY + 2 * HALO, PX = SCALE * kTileX + 2 * HALO;
    static constexpr int NPATCH = PY * PX;
    // staged row pitch in bf16: 16 lanes reading 16 consecutive rows then hit
    // 16 disjoint groups of 4 banks (pitch 40 or 24 elements = 20 or 12 banks)
    static constexpr int PITCH = KC + 8;
    // taps staged per step (EIKU_UP2: the step's own tap)
    static constexpr int TAPS = MODE == EIKU_CONV3 ? 9 : (MODE == EIKU_DOWN2 ? 4 : 1);
    static constexpr int COT = 16 * NT;
    static constexpr int U16 = KC / 8; // 16-byte units per staged row
};

template <int KC> struct Frag;
template <> struct Frag<16> {
    typedef s4 type;
    static __device__ __forceinline__ type load(const uint16_t *p)
    {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
        return __builtin_bit_cast(type, v);
    }
    static __device__ __forceinline__ f4 mma(type a, type b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
};
template <> struct Frag<32> {
    typedef bf8 type;
    static __device__ __forceinline__ type load(const uint16_t *p)
    {
        const uint4 v = *reinterpret_cast<const uint4 *>(p);
        return __builtin_bit_cast(type, v);
    }
    static __device__ __forceinline__ f4 mma(type a, type b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

__device__ __forceinline__ uint32_t pack2(float lo, float hi) { return (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16); }

// The staging of one step: the patch's slice of KC input channels (skipped
// when the slice is already resident) and the weights of the step's taps for
// the workgroup's output channels, loaded into registers first so that every
// load of the step is in flight at once, then written to LDS. CAT: the input
// is a two-source concatenation split at a multiple of KC, so each slice
// comes from one source, chosen once per slice.
template <int MODE, int KC, int NT, bool CAT> struct Staging {
    using G = LdsConv<MODE, KC, NT>;
    static constexpr int NP = (G::NPATCH * G::U16 + 255) / 256;
    static constexpr int NW = (G::TAPS * G::COT * G::U16 + 255) / 256;
    uint4 p[NP], w[NW];

    __device__ __forceinline__ void load(const ConvArgs &a, int t, int b, int x0, int y0, int co0, int c0, int wtap,
                                         bool patch, bool wts)
    {
        if (patch) {
            const bool hi = CAT && c0 >= a.csplit; // uniform over the workgroup
            const bf16 *xs = hi ? a.x2 : a.x;
            const int xcs = hi ? a.x2_cs : a.x_cs, xco = hi ? a.x2_co + (c0 - a.csplit) : a.x_co + c0;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int u = t + 256 * i;
                p[i] = uint4{0u, 0u, 0u, 0u};
                if (u < G::NPATCH * G::U16) {
                    const int pp = u / G::U16, q = u - pp * G::U16;
                    const int py = pp / G::PX, px = pp - py * G::PX;
                    const int gy = G::SCALE * y0 + py - G::HALO, gx = G::SCALE * x0 + px - G::HALO;
                    const int hin = G::SCALE * a.H, win = G::SCALE * a.W;
                    if (gy >= 0 && gy < hin && gx >= 0 && gx < win)
                        p[i] = *reinterpret_cast<const uint4 *>(xs + (((int64_t)b * hin + gy) * win + gx) * xcs + xco +
                                                                8 * q);
                }
            }
        }
        if (!wts) return;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            const int u = t + 256 * i;
            if (u < G::TAPS * G::COT * G::U16) {
                const int q = u % G::U16, r = u / G::U16;
                const int col = r % G::COT, tp = r / G::COT;
                const int tap = MODE == EIKU_UP2 ? wtap : tp;
                w[i] = *reinterpret_cast<const uint4 *>(a.w + ((int64_t)tap * a.Cout + co0 + col) * a.Cin + c0 + 8 * q);
            }
        }
    }

    __device__ __forceinline__ void store(uint16_t *s_patch, uint16_t *s_w, int t, bool patch, bool wts) const
    {
        if (patch) {
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int u = t + 256 * i;
                if (u < G::NPATCH * G::U16) {
                    const int pp = u / G::U16, q = u - pp * G::U16;
                    *reinterpret_cast<uint4 *>(s_patch + pp * G::PITCH + 8 * q) = p[i];
                }
            }
        }
        if (!wts) return;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            const int u = t + 256 * i;
            if (u < G::TAPS * G::COT * G::U16) {
                const int q = u % G::U16, r = u / G::U16;
                *reinterpret_cast<uint4 *>(s_w + r * G::PITCH + 8 * q) = w[i];
            }
        }
    }
};

// grid: x = ceil(B * tiles_y * tiles_x / tpw), y = Cout / (16 NT). A
// workgroup takes tpw consecutive pixel tiles; per tile the steps run over the
// slices of KC input channels, for EIKU_UP2 over (tap, slice) pairs, each
// tap's outputs (one of the four interleaved sub-grids) stored after its last
// slice, so the four sub-grids of a tile are written by one workgroup close in
// time. The next step's loads (the next tile's patch at a tile boundary) are
// in flight while a step is computed; weights that every tile shares (one
// step per tile) are staged once.
template <int MODE, int KC, int NT, bool CAT>
__global__ __launch_bounds__(256) void k_conv_lds(ConvArgs a)
{
    using G = LdsConv<MODE, KC, NT>;
    using F = Frag<KC>;
    __shared__ __attribute__((aligned(16))) uint16_t s_patch[G::NPATCH * G::PITCH];
    __shared__ __attribute__((aligned(16))) uint16_t s_w[G::TAPS * G::COT * G::PITCH];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int tiles_x = (a.W + kTileX - 1) / kTileX, tiles_y = (a.H + kTileY - 1) / kTileY;
    const int64_t ntiles = (int64_t)a.B * tiles_y * tiles_x;
    const int64_t t0 = (int64_t)blockIdx.x * a.tpw;
    const int ntile = (int)(t0 + a.tpw < ntiles ? a.tpw : ntiles - t0);
    const int co0 = blockIdx.y * G::COT;
    const int n = lane & 15, kq = lane >> 4;
    const int nch = a.Cin / KC;
    const int per_tile = (MODE == EIKU_UP2 ? 4 : 1) * nch;
    const int nsteps = ntile * per_tile;
    auto origin = [&](int s, int &b, int &x0, int &y0) { // tile of step s
        const int64_t tile = t0 + s / per_tile;
        const int bx = (int)(tile % tiles_x);
        const int64_t rest = tile / tiles_x;
        y0 = (int)(rest % tiles_y) * kTileY;
        b = (int)(rest / tiles_y);
        x0 = bx * kTileX;
    };
    f4 acc[4][NT];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[f][nt] = f4{0.f, 0.f, 0.f, 0.f};
    Staging<MODE, KC, NT, CAT> stg;
    int b, x0, y0;
    origin(0, b, x0, y0);
    stg.load(a, t, b, x0, y0, co0, 0, 0, true, true);
    for (int s = 0; s < nsteps; ++s) {
        const int sl = s % per_tile; // step within the tile
        const int ci = sl % nch, utap = sl / nch;
        origin(s, b, x0, y0);
        // one slice: the patch stays resident for every tap of the tile
        const bool patch = nch > 1 || sl == 0;
        const bool wts = per_tile > 1 || s == 0;
        __syncthreads(); // the previous step's readers are done
        stg.store(s_patch, s_w, t, patch, wts);
        __syncthreads();
        if (s + 1 < nsteps) {
            const int sn = (s + 1) % per_tile;
            int bn, xn, yn;
            origin(s + 1, bn, xn, yn);
            stg.load(a, t, bn, xn, yn, co0, (sn % nch) * KC, sn / nch, nch > 1 || sn == 0, per_tile > 1);
        }
#pragma unroll 1
        for (int tp = 0; tp < G::TAPS; ++tp) {
            const int dy = MODE == EIKU_CONV3 ? tp / 3 : (MODE == EIKU_DOWN2 ? tp >> 1 : 0);
            const int dx = MODE == EIKU_CONV3 ? tp % 3 : (MODE == EIKU_DOWN2 ? tp & 1 : 0);
            typename F::type wa[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) wa[nt] = F::load(s_w + (tp * G::COT + nt * 16 + n) * G::PITCH + kq * (KC / 4));
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int r = 2 * wave + (f >> 1), cx = 16 * (f & 1) + n;
                const int prow = G::SCALE * r + dy, pcol = G::SCALE * cx + dx;
                const typename F::type xb = F::load(s_patch + (prow * G::PX + pcol) * G::PITCH + kq * (KC / 4));
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[f][nt] = F::mma(wa[nt], xb, acc[f][nt]);
            }
        }
        if (ci != nch - 1) continue;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int gy = y0 + 2 * wave + (f >> 1), gx = x0 + 16 * (f & 1) + n;
            if (gy < a.H && gx < a.W) {
                const int64_t pout =
                    MODE == EIKU_UP2 ? ((int64_t)b * 2 * a.H + 2 * gy + (utap >> 1)) * (2 * a.W) + 2 * gx + (utap & 1)
                                     : ((int64_t)b * a.H + gy) * a.W + gx;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int col = co0 + nt * 16 + 4 * kq;
                    float v[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        v[i] = acc[f][nt][i] + (a.bias ? a.bias[col + i] : 0.f);
                        if (a.relu) v[i] = fmaxf(v[i], 0.f);
                    }
                    *reinterpret_cast<uint2 *>(a.y + pout * a.y_cs + a.y_co + col) =
                        uint2{pack2(v[0], v[1]), pack2(v[2], v[3])};
                }
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[f][nt] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
}

// x2 and csplit as in ConvArgs (read by the 3x3 weight gradient only).
struct WgradArgs {
    const bf16 *x;
    const bf16 *dy;
    float *dw;
    int x_cs, x_co, dy_cs, dy_co;
    int B, H, W, Cin, Cout;
    int64_t chunk;
    const bf16 *x2;
    int x2_cs, x2_co, csplit;
};

// Weight gradient of the transposed convolution, dW[tap][co][ci] = sum over
// input pixels p of dy(2p + d_tap, co) x(p, ci): one wave per (pixel chunk,
// tap, 16x16 channel tile), partial sums added with atomics.
__global__ __launch_bounds__(64) void k_wgrad_up2(WgradArgs a)
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
            const int64_t pdy = ((int64_t)bb * 2 * a.H + 2 * yy + (tap >> 1)) * (2 * a.W) + 2 * xx + (tap & 1);
            av[j] = v ? (short)a.dy[pdy * a.dy_cs + a.dy_co + co0 + r] : (short)0;
            bv[j] = v ? (short)a.x[pc * a.x_cs + a.x_co + ci0 + r] : (short)0;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
        atomicAdd(&a.dw[((int64_t)tap * a.Cout + co0 + 4 * kq + i) * a.Cin + ci0 + r], acc[i]);
}

// ---------------------------------------------------------------------------
// LDS-staged weight gradient of the 3x3 convolution:
//   dW[tap][co][ci] = sum_p dy(p, co) x(p + d_tap, ci)
// a GEMM per tap with K over pixels. A workgroup owns a block of 16 CT output
// x 16 IT input channels and a run of 8 x 32 pixel tiles; per tile it stages
// dy (256 pixels) and the x patch (10 x 34 pixels) in LDS transposed to
// channel-major rows, so a lane's MFMA operand (8 consecutive pixels of one
// channel) is one 16-byte read; the tap's column shift of the x operand is
// taken from two aligned reads in registers. Wave w takes the tile's rows
// 2w, 2w+1 (one 32-pixel K step each) for all taps and channel tiles; the
// partial sums go to dw with one atomic per element and wave at the end.
// ---------------------------------------------------------------------------
constexpr int kWdPitch = 264; // dy row per channel: 256 pixels + 8 (an odd number of 16-byte bank groups)
constexpr int kWxCols = 40;   // x patch row: 34 columns + 6
constexpr int kWxPlane = 408; // x patch per channel: 10 rows x 40 + 8 (an odd number of 16-byte bank groups)

template <int CT, int IT, bool CAT>
__global__ __launch_bounds__(256) void k_wgrad3_lds(WgradArgs a, int tiles_per_wg)
{
    __shared__ __attribute__((aligned(16))) uint16_t s_dy[CT * 16 * kWdPitch];
    __shared__ __attribute__((aligned(16))) uint16_t s_x[IT * 16 * kWxPlane];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int n = lane & 15, kq = lane >> 4;
    const int cblocks = a.Cout / (16 * CT);
    const int co0 = (int)(blockIdx.y % cblocks) * 16 * CT, ci0 = (int)(blockIdx.y / cblocks) * 16 * IT;
    const int tiles_x = (a.W + kTileX - 1) / kTileX, tiles_y = (a.H + kTileY - 1) / kTileY;
    const int64_t ntiles = (int64_t)a.B * tiles_y * tiles_x;
    const int64_t t0 = (int64_t)blockIdx.x * tiles_per_wg;
    const int64_t t1 = t0 + tiles_per_wg < ntiles ? t0 + tiles_per_wg : ntiles;
    f4 acc[9][CT][IT];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int i = 0; i < IT; ++i) acc[k][c][i] = f4{0.f, 0.f, 0.f, 0.f};
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int bx = (int)(tile % tiles_x);
        const int64_t rest = tile / tiles_x;
        const int by = (int)(rest % tiles_y), b = (int)(rest / tiles_y);
        const int x0 = bx * kTileX, y0 = by * kTileY;
        __syncthreads(); // the previous tile's readers are done
        // dy: pairs of horizontally adjacent pixels x 8-channel groups; each
        // channel's two values go to LDS as one 32-bit word
        for (int u = t; u < 128 * 2 * CT; u += 256) {
            const int pr = u / (2 * CT), q = u - pr * (2 * CT);
            const int px = 2 * pr, r = px / kTileX, c = px - r * kTileX;
            const int gy = y0 + r, gx = x0 + c;
            uint4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
            if (gy < a.H) {
                const bf16 *row = a.dy + ((int64_t)b * a.H + gy) * a.W * a.dy_cs + a.dy_co + co0 + 8 * q;
                if (gx < a.W) v0 = *reinterpret_cast<const uint4 *>(row + (int64_t)gx * a.dy_cs);
                if (gx + 1 < a.W) v1 = *reinterpret_cast<const uint4 *>(row + (int64_t)(gx + 1) * a.dy_cs);
            }
            const uint32_t e0[4] = {v0.x, v0.y, v0.z, v0.w}, e1[4] = {v1.x, v1.y, v1.z, v1.w};
            uint32_t *dst = reinterpret_cast<uint32_t *>(s_dy + (8 * q) * kWdPitch + px);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                dst[(2 * j) * (kWdPitch / 2)] = (e0[j] & 0xffffu) | (e1[j] << 16);
                dst[(2 * j + 1) * (kWdPitch / 2)] = (e0[j] >> 16) | (e1[j] & 0xffff0000u);
            }
        }
        // x patch rows y0-1 .. y0+8, columns x0-1 .. x0+32, zero outside the image
        for (int u = t; u < 170 * 2 * IT; u += 256) {
            const int pr = u / (2 * IT), q = u - pr * (2 * IT);
            const int py = pr / 17, pc = 2 * (pr - py * 17);
            const int gy = y0 + py - 1, gx = x0 + pc - 1;
            uint4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
            if (gy >= 0 && gy < a.H) {
                if (CAT) { // a channel block may straddle the split: the source per 8 channels
                    const int64_t pix = ((int64_t)b * a.H + gy) * a.W + gx;
                    const int c = ci0 + 8 * q;
                    if (gx >= 0 && gx < a.W)
                        v0 = *reinterpret_cast<const uint4 *>(src8(a.x, a.x_cs, a.x_co, a.x2, a.x2_cs, a.x2_co,
                                                                   a.csplit, pix, c));
                    if (gx + 1 >= 0 && gx + 1 < a.W)
                        v1 = *reinterpret_cast<const uint4 *>(src8(a.x, a.x_cs, a.x_co, a.x2, a.x2_cs, a.x2_co,
                                                                   a.csplit, pix + 1, c));
                } else {
                    const bf16 *row = a.x + ((int64_t)b * a.H + gy) * a.W * a.x_cs + a.x_co + ci0 + 8 * q;
                    if (gx >= 0 && gx < a.W) v0 = *reinterpret_cast<const uint4 *>(row + (int64_t)gx * a.x_cs);
                    if (gx + 1 >= 0 && gx + 1 < a.W)
                        v1 = *reinterpret_cast<const uint4 *>(row + (int64_t)(gx + 1) * a.x_cs);
                }
            }
            const uint32_t e0[4] = {v0.x, v0.y, v0.z, v0.w}, e1[4] = {v1.x, v1.y, v1.z, v1.w};
            uint32_t *dst = reinterpret_cast<uint32_t *>(s_x + (8 * q) * kWxPlane + py * kWxCols + pc);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                dst[(2 * j) * (kWxPlane / 2)] = (e0[j] & 0xffffu) | (e1[j] << 16);
                dst[(2 * j + 1) * (kWxPlane / 2)] = (e0[j] >> 16) | (e1[j] & 0xffff0000u);
            }
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int r = 2 * wave + rr;
            bf8 dv[CT];
#pragma unroll
            for (int c = 0; c < CT; ++c)
                dv[c] = Frag<32>::load(s_dy + (c * 16 + n) * kWdPitch + r * kTileX + 8 * kq);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int ty = tap / 3, tx = tap % 3;
#pragma unroll
                for (int i = 0; i < IT; ++i) {
                    const uint16_t *src = s_x + (i * 16 + n) * kWxPlane + (r + ty) * kWxCols + 8 * kq;
                    const uint4 lo = *reinterpret_cast<const uint4 *>(src);
                    uint4 w;
                    if (tx == 0) {
                        w = lo;
                    } else {
                        const uint4 hi = *reinterpret_cast<const uint4 *>(src + 8);
                        if (tx == 2)
                            w = uint4{lo.y, lo.z, lo.w, hi.x};
                        else
                            w = uint4{(lo.x >> 16) | (lo.y << 16), (lo.y >> 16) | (lo.z << 16),
                                      (lo.z >> 16) | (lo.w << 16), (lo.w >> 16) | (hi.x << 16)};
                    }
                    const bf8 xv = __builtin_bit_cast(bf8, w);
#pragma unroll
                    for (int c = 0; c < CT; ++c) acc[tap][c][i] = Frag<32>::mma(dv[c], xv, acc[tap][c][i]);
                }
            }
        }
    }
    if (t0 >= t1) return;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int i = 0; i < IT; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    atomicAdd(&a.dw[((int64_t)tap * a.Cout + co0 + c * 16 + 4 * kq + e) * a.Cin + ci0 + i * 16 + n],
                              acc[tap][c][i][e]);
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

// The same pooling 8 channels (one 16-byte word) per thread, for layouts whose
// channel strides and offsets are multiples of 8.
__global__ void k_maxpool_fwd8(int B, int H, int W, const bf16 *__restrict__ x, int xcs, int xco,
                               bf16 *__restrict__ y, int ycs, int yco, int C)
{
    const int G = C / 8;
    const int64_t n = (int64_t)B * H * W * G;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)(e % G);
        const int64_t p = e / G;
        const int xo = (int)(p % W);
        const int64_t t = p / W;
        const int yo = (int)(t % H), b = (int)(t / H);
        float m[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) m[j] = -INFINITY;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t pi = ((int64_t)b * 2 * H + 2 * yo + (q >> 1)) * (2 * W) + 2 * xo + (q & 1);
            const uint4 v = *reinterpret_cast<const uint4 *>(x + pi * xcs + xco + 8 * g);
            const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                m[2 * j] = fmaxf(m[2 * j], bf2f((bf16)(w4[j] & 0xffffu)));
                m[2 * j + 1] = fmaxf(m[2 * j + 1], bf2f((bf16)(w4[j] >> 16)));
            }
        }
        *reinterpret_cast<uint4 *>(y + p * ycs + yco + 8 * g) =
            uint4{pack2(m[0], m[1]), pack2(m[2], m[3]), pack2(m[4], m[5]), pack2(m[6], m[7])};
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

// 16 channels per pixel read as two 16-byte words (the same sum in the same order).
__global__ void k_head_fwd16(int64_t n, const bf16 *__restrict__ x, int cs, int co, const float *__restrict__ w,
                             const float *__restrict__ b, float *__restrict__ out)
{
    float wr[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) wr[c] = w[c];
    const float b0 = b[0];
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint4 v0 = *reinterpret_cast<const uint4 *>(x + p * cs + co);
        const uint4 v1 = *reinterpret_cast<const uint4 *>(x + p * cs + co + 8);
        const uint32_t u[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        float s = b0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            s += wr[2 * j] * bf2f((bf16)(u[j] & 0xffffu));
            s += wr[2 * j + 1] * bf2f((bf16)(u[j] >> 16));
        }
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
        uint4 *xp = reinterpret_cast<uint4 *>(x + p * 16);
        xp[0] = uint4{pack2(Mb[q], Mb[plane + q]), pack2(Mb[2 * plane + q], ob[q]), pack2(ob[plane + q], d), 0u};
        xp[1] = uint4{0u, 0u, 0u, 0u};
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

namespace {

// Pixel tiles per workgroup: one per kTpwTiles tiles of the launch, at most
// kTpwMax, so that large launches keep at least kTpwTiles workgroups. On the
// 256^2 network over 250 grids (64 000 tiles per level-0 launch) the forward
// took 4.16 ms with one tile per workgroup, 4.08 with two, 4.09 with four and
// 4.14 with eight.
constexpr int64_t kTpwTiles = 16384;
constexpr int kTpwMax = 2;

// Launch k_conv_lds for arguments already checked. cat: a two-source 3x3
// convolution, its slices of KC channels kept on one side of the split.
int conv_launch(int mode, const ConvArgs &args, hipStream_t st, bool cat = false)
{
    const int nt = args.Cout % 64 == 0 ? 4 : (args.Cout % 32 == 0 ? 2 : 1);
    const int64_t tiles = (int64_t)args.B * ((args.H + kTileY - 1) / kTileY) * ((args.W + kTileX - 1) / kTileX);
    ConvArgs a = args;
    a.tpw = (int)std::max<int64_t>(1, std::min<int64_t>(kTpwMax, tiles / kTpwTiles));
    const int64_t groups = (tiles + a.tpw - 1) / a.tpw;
    if (groups > 0x7fffffff) return -1;
    const dim3 g((unsigned)groups, (unsigned)(a.Cout / (16 * nt)));
    const bool k32 = a.Cin % 32 == 0 && a.csplit % 32 == 0;
#define EIKU_LDS(MODE, KC, CAT)                                                                               \
    do {                                                                                                      \
        if (nt == 4) hipLaunchKernelGGL((k_conv_lds<MODE, KC, 4, CAT>), g, dim3(256), 0, st, a);              \
        else if (nt == 2) hipLaunchKernelGGL((k_conv_lds<MODE, KC, 2, CAT>), g, dim3(256), 0, st, a);         \
        else hipLaunchKernelGGL((k_conv_lds<MODE, KC, 1, CAT>), g, dim3(256), 0, st, a);                      \
    } while (0)
    if (mode == EIKU_CONV3 && cat) {
        if (k32) EIKU_LDS(EIKU_CONV3, 32, true);
        else EIKU_LDS(EIKU_CONV3, 16, true);
    } else if (mode == EIKU_CONV3) {
        if (k32) EIKU_LDS(EIKU_CONV3, 32, false);
        else EIKU_LDS(EIKU_CONV3, 16, false);
    } else if (mode == EIKU_UP2) {
        if (k32) EIKU_LDS(EIKU_UP2, 32, false);
        else EIKU_LDS(EIKU_UP2, 16, false);
    } else {
        EIKU_LDS(EIKU_DOWN2, 16, false); // 16-channel slices keep the 2x patch at 48 KiB of LDS
    }
#undef EIKU_LDS
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Launch k_wgrad3_lds for arguments already checked.
template <bool CAT>
int wgrad3_launch(const WgradArgs &a, hipStream_t st)
{
    const int ct = a.Cout % 32 == 0 ? 2 : 1, it = a.Cin % 32 == 0 ? 2 : 1;
    const int blocks = (a.Cout / (16 * ct)) * (a.Cin / (16 * it));
    const int64_t ntiles = (int64_t)a.B * ((a.H + kTileY - 1) / kTileY) * ((a.W + kTileX - 1) / kTileX);
    // about 2048 workgroups over the channel blocks and pixel runs
    int64_t per = (ntiles * blocks + 2047) / 2048;
    per = per < 1 ? 1 : per;
    const int64_t runs = (ntiles + per - 1) / per;
    if (runs > 0x7fffffff) return -1;
    const dim3 g((unsigned)runs, (unsigned)blocks);
    if (ct == 2 && it == 2) hipLaunchKernelGGL((k_wgrad3_lds<2, 2, CAT>), g, dim3(256), 0, st, a, (int)per);
    else if (ct == 2) hipLaunchKernelGGL((k_wgrad3_lds<2, 1, CAT>), g, dim3(256), 0, st, a, (int)per);
    else if (it == 2) hipLaunchKernelGGL((k_wgrad3_lds<1, 2, CAT>), g, dim3(256), 0, st, a, (int)per);
    else hipLaunchKernelGGL((k_wgrad3_lds<1, 1, CAT>), g, dim3(256), 0, st, a, (int)per);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The two sources of a concatenated input: channel strides and offsets in
// multiples of 8, each slice inside its pixel, 16-byte aligned buffers, and
// Ca, Cb multiples of 16.
bool cat_ok(const uint16_t *xa, int xa_cs, int xa_co, int Ca, const uint16_t *xb, int xb_cs, int xb_co, int Cb)
{
    if (!xa || !xb || Ca < 16 || Cb < 16 || (Ca | Cb) % 16) return false;
    if ((xa_cs | xa_co | xb_cs | xb_co) % 8 || xa_co < 0 || xb_co < 0 || xa_co + Ca > xa_cs || xb_co + Cb > xb_cs)
        return false;
    return ((uintptr_t)xa | (uintptr_t)xb) % 16 == 0;
}

} // namespace

extern "C" {

int eiku_conv_fwd(int32_t mode, int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t x_cs, int32_t x_co,
                  int32_t Cin, const uint16_t *w, const float *bias, int32_t relu, uint16_t *y, int32_t y_cs,
                  int32_t y_co, int32_t Cout, hipStream_t st)
{
    if (B < 1 || H < 1 || W < 1 || Cin < 16 || Cin % 16 || Cout < 16 || Cout % 16 || !x || !w || !y) return -1;
    if ((x_cs | x_co) % 8 || (y_cs | y_co) % 4 || x_co + Cin > x_cs || y_co + Cout > y_cs) return -1;
    if (((uintptr_t)x | (uintptr_t)w) % 16 || (uintptr_t)y % 8) return -1;
    if (mode != EIKU_CONV3 && mode != EIKU_UP2 && mode != EIKU_DOWN2) return -1;
    const ConvArgs a{x, w, bias, y, x_cs, x_co, y_cs, y_co, B, H, W, Cin, Cout, relu, x, x_cs, x_co, Cin};
    return conv_launch(mode, a, st);
}

int eiku_conv_fwd_cat(int32_t B, int32_t H, int32_t W, const uint16_t *xa, int32_t xa_cs, int32_t xa_co, int32_t Ca,
                      const uint16_t *xb, int32_t xb_cs, int32_t xb_co, int32_t Cb, const uint16_t *w,
                      const float *bias, int32_t relu, uint16_t *y, int32_t y_cs, int32_t y_co, int32_t Cout,
                      hipStream_t st)
{
    if (B < 1 || H < 1 || W < 1 || Cout < 16 || Cout % 16 || !w || !y) return -1;
    if (!cat_ok(xa, xa_cs, xa_co, Ca, xb, xb_cs, xb_co, Cb)) return -1;
    if ((y_cs | y_co) % 4 || y_co < 0 || y_co + Cout > y_cs || (uintptr_t)w % 16 || (uintptr_t)y % 8) return -1;
    const ConvArgs a{xa, w, bias, y, xa_cs, xa_co, y_cs, y_co, B, H, W, Ca + Cb, Cout, relu, xb, xb_cs, xb_co, Ca};
    return conv_launch(EIKU_CONV3, a, st, true);
}

int eiku_conv_wgrad(int32_t mode, int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t x_cs, int32_t x_co,
                    int32_t Cin, const uint16_t *dy, int32_t dy_cs, int32_t dy_co, int32_t Cout, float *dw,
                    hipStream_t st)
{
    if (B < 1 || H < 1 || W < 1 || Cin < 16 || Cin % 16 || Cout < 16 || Cout % 16 || !x || !dy || !dw) return -1;
    if (x_co + Cin > x_cs || dy_co + Cout > dy_cs) return -1;
    if (mode != EIKU_CONV3 && mode != EIKU_UP2) return -1;
    const int64_t npix = (int64_t)B * H * W;
    if (mode == EIKU_CONV3) {
        if ((x_cs | x_co | dy_cs | dy_co) % 8 || ((uintptr_t)x | (uintptr_t)dy) % 16) return -1;
        const WgradArgs a{x, dy, dw, x_cs, x_co, dy_cs, dy_co, B, H, W, Cin, Cout, 0, x, x_cs, x_co, Cin};
        return wgrad3_launch<false>(a, st);
    }
    int64_t chunk = npix / 128;
    chunk = chunk < 256 ? 256 : (chunk > 8192 ? 8192 : chunk);
    chunk = (chunk + 15) / 16 * 16;
    WgradArgs a{x, dy, dw, x_cs, x_co, dy_cs, dy_co, B, H, W, Cin, Cout, chunk, x, x_cs, x_co, Cin};
    dim3 grid((unsigned)((npix + chunk - 1) / chunk), (unsigned)(4 * (Cout / 16) * (Cin / 16)));
    hipLaunchKernelGGL(k_wgrad_up2, grid, dim3(64), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int eiku_conv_wgrad_cat(int32_t B, int32_t H, int32_t W, const uint16_t *xa, int32_t xa_cs, int32_t xa_co,
                        int32_t Ca, const uint16_t *xb, int32_t xb_cs, int32_t xb_co, int32_t Cb, const uint16_t *dy,
                        int32_t dy_cs, int32_t dy_co, int32_t Cout, float *dw, hipStream_t st)
{
    if (B < 1 || H < 1 || W < 1 || Cout < 16 || Cout % 16 || !dy || !dw) return -1;
    if (!cat_ok(xa, xa_cs, xa_co, Ca, xb, xb_cs, xb_co, Cb)) return -1;
    if ((dy_cs | dy_co) % 8 || dy_co < 0 || dy_co + Cout > dy_cs || (uintptr_t)dy % 16) return -1;
    const WgradArgs a{xa, dy, dw, xa_cs, xa_co, dy_cs, dy_co, B, H, W, Ca + Cb, Cout, 0, xb, xb_cs, xb_co, Ca};
    return wgrad3_launch<true>(a, st);
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
    if (C % 8 == 0 && (x_cs | x_co | y_cs | y_co) % 8 == 0 && ((uintptr_t)x | (uintptr_t)y) % 16 == 0)
        hipLaunchKernelGGL(k_maxpool_fwd8, dim3(gblocks((int64_t)B * H * W * (C / 8), 256)), dim3(256), 0, st, B, H, W,
                           x, x_cs, x_co, y, y_cs, y_co, C);
    else
        hipLaunchKernelGGL(k_maxpool_fwd, dim3(gblocks((int64_t)B * H * W * C, 256)), dim3(256), 0, st, B, H, W, x,
                           x_cs, x_co, y, y_cs, y_co, C);
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
    if (C == 16 && (cs | co) % 8 == 0 && (uintptr_t)x % 16 == 0)
        hipLaunchKernelGGL(k_head_fwd16, dim3(gblocks(npix, 256)), dim3(256), 0, st, npix, x, cs, co, w, b, out);
    else
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
    if (B < 1 || H < 1 || W < 1 || max_src < 1 || !M || !omega || !src || !h || !x || (uintptr_t)x % 16) return -1;
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
