// hb_nn.hip -- a small BF16 convolutional U-Net on the MFMA matrix cores
// (gfx950), trained on the GPU by the kernels of this file, used to
// warm-start the nodal projection solve.
//
// Network: 4 levels with 16, 32, 64, 64 channels; two 3x3 convolutions with
// ReLU per level on the way down (2x2 average pooling between levels) and on
// the way up (nearest-neighbour upsampling, concatenation with the skip
// connection), then a 3x3 head without activation.  Activations are NHWC
// BF16 with channel counts padded to multiples of 16; weights are FP32
// master copies with BF16 copies for the products; every product
// accumulates in FP32.
//
// Convolution = implicit GEMM on v_mfma_f32_16x16x16_bf16: output channels
// x pixels, reduced over (tap, input channel).  The backward pass to the
// input is the same kernel with the spatially flipped, transposed weights;
// the weight gradient is a GEMM reduced over pixels.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hb_internal.h"

namespace hb {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even FP32 -> BF16 and back
__device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int kStrip = 64;   // pixels of one row per convolution block (4 waves x 16)

// ---------------------------------------------------------------------------
// 3x3 convolution, zero padding: y[b,p,co] = sum_{tap,ci} w[co,tap,ci] x[b,p+off(tap),ci] (+ bias, ReLU)
// x: [n][H][W][Cin] bf16; w: [Cout][9][Cin] bf16; outputs bf16 and/or fp32.
// Block: image blockIdx.z, row blockIdx.y, 64-pixel strip blockIdx.x; wave w
// owns pixels 16w..16w+15 of the strip and all MT = Cout/16 output tiles.
// MFMA operand layout (16x16x16): lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16], and D[4(l/16)+j][l%16], j = 0..3.
// ---------------------------------------------------------------------------
// CIN > 0 fixes the input channel count at compile time, so the tap and
// channel loops unroll and the weight loads (from L2) can be issued well
// ahead of the MFMAs that use them; CIN = 0 takes it from cin_rt.  Same
// products in the same order either way.
template <int MT, int CIN = 0>
__global__ void __launch_bounds__(256)
k_conv3(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w, const float* __restrict__ bias, int H, int W,
        int cin_rt, int relu, uint16_t* __restrict__ y, float* __restrict__ yf)
{
    const int Cin = CIN > 0 ? CIN : cin_rt;
    extern __shared__ __align__(16) uint16_t sx[];   // [3][kStrip + 2][Cin]
    const int b = blockIdx.z, yr = blockIdx.y, x0 = blockIdx.x * kStrip;
    const int cols = kStrip + 2;
    const int total4 = 3 * cols * Cin / 4;
    for (int t = threadIdx.x; t < total4; t += blockDim.x) {
        const int e = t * 4;
        const int ci = e % Cin, col = (e / Cin) % cols, r = e / (Cin * cols);
        const int yy = yr - 1 + r, xx = x0 - 1 + col;
        uint2 v = make_uint2(0u, 0u);
        if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = *(const uint2*)(x + (((long)b * H + yy) * W + xx) * Cin + ci);
        *(uint2*)(sx + e) = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int pn = lane & 15, kg = lane >> 4;
    const int px = wv * 16 + pn;
    f32x4 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
        const uint16_t* brow = sx + (dy * cols + px + dx) * Cin + 4 * kg;
        const uint16_t* wt = w + (long)tap * Cin + 4 * kg;
#pragma unroll
        for (int c0 = 0; c0 < Cin; c0 += 16) {
            const bf16x4 B = *(const bf16x4*)(brow + c0);
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const bf16x4 A = *(const bf16x4*)(wt + (long)(m * 16 + pn) * 9 * Cin + c0);
                acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[m], 0, 0, 0);
            }
        }
    }
    const int xx = x0 + px;
    if (xx >= W) return;
    const long base = (((long)b * H + yr) * W + xx) * (MT * 16);
    // a lane's four channels 4 kg .. 4 kg + 3 of tile m are contiguous (NHWC):
    // one 8-byte (bf16) or 16-byte (fp32) store each
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int co = m * 16 + 4 * kg;
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = acc[m][j] + (bias ? bias[co + j] : 0.0f);
            if (relu) v[j] = fmaxf(v[j], 0.0f);
        }
        if (y)
            *(uint2*)(y + base + co) = make_uint2((uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                                                  (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16));
        if (yf) *(float4*)(yf + base + co) = make_float4(v[0], v[1], v[2], v[3]);
    }
}

// ---------------------------------------------------------------------------
// weight gradient dw[co,tap,ci] += sum_p dz[p,co] x[p+off(tap),ci]: each wave
// owns one 16x16 tile (co tile, (tap,ci) tile) and a chunk of pixels (the K
// dimension, 16 per MFMA), then adds its tile to dw atomically.
// ---------------------------------------------------------------------------
constexpr int kPixChunk = 2048;

__global__ void __launch_bounds__(256)
k_conv3_dw(const uint16_t* __restrict__ dz, const uint16_t* __restrict__ x, int n, int H, int W, int Cin, int Cout,
           float* __restrict__ dw)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ntn = 9 * Cin / 16, ntm = Cout / 16;
    const int tile = blockIdx.x * 4 + wv;
    if (tile >= ntm * ntn) return;
    const int mt = tile / ntn, nt = tile % ntn;
    const int pn = lane & 15, kg = lane >> 4;
    const int co = mt * 16 + pn;                  // A row of this lane
    const int kn = nt * 16 + pn;                  // B column of this lane: (tap, ci)
    const int tap = kn / Cin, ci = kn % Cin;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const long npix = (long)n * H * W;
    const long p0 = (long)blockIdx.y * kPixChunk;
    f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (long k0 = p0; k0 < p0 + kPixChunk && k0 < npix; k0 += 16) {
        bf16x4 A, B;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long p = k0 + 4 * kg + j;
            short av = 0, bv = 0;
            if (p < npix) {
                av = (short)dz[p * Cout + co];
                const int xx = (int)(p % W), yy = (int)((p / W) % H);
                const long bb = p / ((long)W * H);
                const int sy = yy + dy, sxx = xx + dx;
                if (sy >= 0 && sy < H && sxx >= 0 && sxx < W) bv = (short)x[((bb * H + sy) * W + sxx) * Cin + ci];
            }
            A[j] = av;
            B[j] = bv;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc, 0, 0, 0);
    }
    // D[4kg+j][pn]: row = co tile row, column = (tap, ci) within the tile
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = mt * 16 + 4 * kg + j;
        atomicAdd(dw + (long)r * 9 * Cin + nt * 16 + pn, acc[j]);
    }
}

// ---------------------------------------------------------------------------
// elementwise and layout kernels
// ---------------------------------------------------------------------------

#define NN_LOOP(i, n) for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)

// fp32 [P][cin] -> bf16 [P][cpad] (extra channels zero)
__global__ void k_pack_in(const float* __restrict__ x, long P, int cin, int cpad, uint16_t* __restrict__ y)
{
    NN_LOOP(i, P * cpad)
    {
        const long p = i / cpad;
        const int c = (int)(i % cpad);
        y[i] = c < cin ? f2bf(x[p * cin + c]) : (uint16_t)0;
    }
}

// fp32 [P][cpad] -> fp32 [P][cout] (first channels)
__global__ void k_unpack_out(const float* __restrict__ y, long P, int cpad, int cout, float* __restrict__ o)
{
    NN_LOOP(i, P * cout) o[i] = y[(i / cout) * cpad + i % cout];
}

// 2x2 average pooling, four channels per thread (C is a multiple of 16 and
// every activation has fewer than 2^31 values)
__global__ void k_pool2(const uint16_t* __restrict__ x, int n, int H, int W, int C, uint16_t* __restrict__ y)
{
    const int h = H / 2, w = W / 2, C4 = C / 4;
    const int total = n * h * w * C4;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int c = 4 * (i % C4), q = i / C4;
        const int X = q % w, Y = (q / w) % h, b = q / (w * h);
        const long s = ((long)(b * H + 2 * Y) * W + 2 * X) * C + c;
        const uint2 p00 = *(const uint2*)(x + s), p01 = *(const uint2*)(x + s + C);
        const uint2 p10 = *(const uint2*)(x + s + (long)W * C), p11 = *(const uint2*)(x + s + (long)W * C + C);
        const uint32_t a00[2] = {p00.x, p00.y}, a01[2] = {p01.x, p01.y}, a10[2] = {p10.x, p10.y}, a11[2] = {p11.x, p11.y};
        uint32_t o[2];
#pragma unroll
        for (int hw = 0; hw < 2; ++hw) {
            uint32_t r = 0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int sh = 16 * k;
                const float v = bf2f((uint16_t)(a00[hw] >> sh)) + bf2f((uint16_t)(a01[hw] >> sh)) +
                                bf2f((uint16_t)(a10[hw] >> sh)) + bf2f((uint16_t)(a11[hw] >> sh));
                r |= (uint32_t)f2bf(0.25f * v) << sh;
            }
            o[hw] = r;
        }
        *(uint2*)(y + (long)q * C + c) = make_uint2(o[0], o[1]);
    }
}

// dx (fp32, full resolution) += dy / 4 spread over the 2x2 children
__global__ void k_pool2_bwd(const float* __restrict__ dy, int n, int H, int W, int C, float* __restrict__ dx)
{
    NN_LOOP(i, (long)n * H * W * C)
    {
        const int c = (int)(i % C);
        const long q = i / C;
        const int xx = (int)(q % W), yy = (int)((q / W) % H);
        const long b = q / ((long)W * H);
        dx[i] += 0.25f * dy[((b * (H / 2) + yy / 2) * (W / 2) + xx / 2) * C + c];
    }
}

// y[b, y, x, 0:Ca] = up(a)[..], y[.., Ca:Ca+Cb] = s  (a at half resolution)
// four channels per thread (Ca and Cb are multiples of 16, so a group never
// straddles the two sources)
__global__ void k_up_concat(const uint16_t* __restrict__ a, int Ca, const uint16_t* __restrict__ s, int Cb, int n, int H,
                            int W, uint16_t* __restrict__ y)
{
    const int C = Ca + Cb, C4 = C / 4;
    const int total = n * H * W * C4;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int c = 4 * (i % C4), q = i / C4;
        const int xx = q % W, yy = (q / W) % H, b = q / (W * H);
        const uint16_t* src = c < Ca ? a + ((long)(b * (H / 2) + yy / 2) * (W / 2) + xx / 2) * Ca + c
                                     : s + (long)q * Cb + (c - Ca);
        *(uint2*)(y + (long)q * C + c) = *(const uint2*)src;
    }
}

// split the gradient of an up-concat: da (half resolution) = sum of the 2x2
// children's first Ca channels; ds += the remaining channels
__global__ void k_up_concat_bwd_a(const float* __restrict__ dy, int Ca, int Cb, int n, int H, int W, float* __restrict__ da)
{
    const int C = Ca + Cb, h = H / 2, w = W / 2;
    NN_LOOP(i, (long)n * h * w * Ca)
    {
        const int c = (int)(i % Ca);
        const long q = i / Ca;
        const int X = (int)(q % w), Y = (int)((q / w) % h);
        const long b = q / ((long)w * h);
        const long s = ((b * H + 2 * Y) * W + 2 * X) * C + c;
        da[i] = dy[s] + dy[s + C] + dy[s + (long)W * C] + dy[s + (long)W * C + C];
    }
}

__global__ void k_up_concat_bwd_s(const float* __restrict__ dy, int Ca, int Cb, long P, float* __restrict__ ds)
{
    NN_LOOP(i, P * Cb) ds[i] += dy[(i / Cb) * (Ca + Cb) + Ca + i % Cb];
}

// dz = dy * relu'(y) (y > 0), bf16 for the products; fp32 copy for the bias
__global__ void k_relu_bwd(const float* __restrict__ dy, const uint16_t* __restrict__ y, long N, int relu,
                           uint16_t* __restrict__ dzb, float* __restrict__ dzf)
{
    NN_LOOP(i, N)
    {
        const float v = (!relu || bf2f(y[i]) > 0.0f) ? dy[i] : 0.0f;
        dzb[i] = f2bf(v);
        dzf[i] = v;
    }
}

// db[c] += sum over pixels of dz[p, c]: block per channel, fixed order
__global__ void k_bias_grad(const float* __restrict__ dz, long P, int C, float* __restrict__ db)
{
    __shared__ float sh[256];
    const int c = blockIdx.x;
    float s = 0.0f;
    for (long p = threadIdx.x; p < P; p += blockDim.x) s += dz[p * C + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] += sh[0];
}

// loss = mean over (p, c < cout) of (y - t)^2; dy = 2 (y - t) / count
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t, long P, int cpad, int cout,
                      float* __restrict__ dy, float* __restrict__ part)
{
    __shared__ float sh[256];
    float s = 0.0f;
    const float inv = 1.0f / (float)(P * cout);
    NN_LOOP(i, P * cpad)
    {
        const long p = i / cpad;
        const int c = (int)(i % cpad);
        float g = 0.0f;
        if (c < cout) {
            const float d = y[i] - t[p * cout + c];
            s += d * d;
            g = 2.0f * d * inv;
        }
        dy[i] = g;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] * inv;
}

// Adam step on the FP32 master weights
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long N, float lr, float b1, float b2, float c1, float c2, float eps)
{
    NN_LOOP(i, N)
    {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// BF16 copies of one layer's weights: w16[co][tap][ci] and the flipped
// transpose wt16[ci][tap][co] = w[co][8 - tap][ci] for the input gradient
__global__ void k_weights_bf16(const float* __restrict__ w, int Cout, int Cin, uint16_t* __restrict__ w16,
                               uint16_t* __restrict__ wt16)
{
    NN_LOOP(i, (long)Cout * 9 * Cin)
    {
        const int ci = (int)(i % Cin), tap = (int)((i / Cin) % 9), co = (int)(i / (9L * Cin));
        const uint16_t h = f2bf(w[i]);
        w16[i] = h;
        wt16[((long)ci * 9 + (8 - tap)) * Cout + co] = h;
    }
}

static unsigned nn_blocks(long n)
{
    const long b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

// ---------------------------------------------------------------------------
// the network
// ---------------------------------------------------------------------------

struct ConvL {
    int cin, cout, relu;
    long woff, boff;           // offsets in the flat parameter vector
    uint16_t *w16 = nullptr, *wt16 = nullptr;
};

struct Act {                   // one activation with its gradient
    int H = 0, W = 0, C = 0;
    uint16_t* a = nullptr;     // bf16 values
    float* g = nullptr;        // fp32 gradient
};

struct NNet {
    int in_ch, out_ch;
    hipStream_t s = nullptr;
    std::vector<ConvL> L;
    long np = 0;
    float *w = nullptr, *gw = nullptr, *m = nullptr, *v = nullptr;   // flat FP32 parameters, gradient, Adam moments
    long step = 0;
    // activation buffers for the current (n, H, W)
    int n = 0, H = 0, W = 0;
    std::vector<Act> A;
    uint16_t* dzb = nullptr;
    float *dzf = nullptr, *yout = nullptr, *hg = nullptr, *part = nullptr, *hpart = nullptr;
    long scratch = 0;
    std::string err;
};

// layer list: (cin, cout, relu); channels 16, 32, 64, 64
static const int kLay[15][3] = {
    {16, 16, 1}, {16, 16, 1},      // level 0 down
    {16, 32, 1}, {32, 32, 1},      // level 1 down
    {32, 64, 1}, {64, 64, 1},      // level 2 down
    {64, 64, 1}, {64, 64, 1},      // level 3 (bottom)
    {128, 64, 1}, {64, 64, 1},     // level 2 up (64 up + 64 skip)
    {96, 32, 1}, {32, 32, 1},      // level 1 up (64 up + 32 skip)
    {48, 16, 1}, {16, 16, 1},      // level 0 up (32 up + 16 skip)
    {16, 16, 0}};                  // head

// activation slots: 0 input; per layer its output; pools and concats
enum {
    A_IN = 0, A_E0A, A_E0, A_P0, A_E1A, A_E1, A_P1, A_E2A, A_E2, A_P2, A_E3A, A_E3,
    A_C2, A_D2A, A_D2, A_C1, A_D1A, A_D1, A_C0, A_D0A, A_D0, A_NACT
};

static void nn_free_acts(NNet* t)
{
    for (Act& a : t->A) {
        (void)hipFree(a.a);
        (void)hipFree(a.g);
    }
    t->A.clear();
    (void)hipFree(t->dzb);
    (void)hipFree(t->dzf);
    (void)hipFree(t->yout);
    (void)hipFree(t->hg);
    (void)hipFree(t->part);
    if (t->hpart) (void)hipHostFree(t->hpart);
    t->dzb = nullptr;
    t->dzf = t->yout = t->hg = t->part = t->hpart = nullptr;
    t->n = t->H = t->W = 0;
}

static int nn_shape(NNet* t, int n, int H, int W)
{
    if (t->n == n && t->H == H && t->W == W) return HB_OK;
    nn_free_acts(t);
    const int dims[A_NACT][2] = {{0, 16}, {0, 16}, {0, 16}, {1, 16}, {1, 32}, {1, 32}, {2, 32}, {2, 64}, {2, 64},
                                 {3, 64}, {3, 64}, {3, 64}, {2, 128}, {2, 64}, {2, 64}, {1, 96}, {1, 32}, {1, 32},
                                 {0, 48}, {0, 16}, {0, 16}};
    t->A.resize(A_NACT);
    long big = 0;
    for (int i = 0; i < A_NACT; ++i) {
        Act& a = t->A[i];
        a.H = H >> dims[i][0];
        a.W = W >> dims[i][0];
        a.C = dims[i][1];
        const long e = (long)n * a.H * a.W * a.C;
        if (e >= (1L << 31)) {   // the layout kernels index activations with 32 bits
            nn_free_acts(t);
            return HB_ERR_ARG;
        }
        big = e > big ? e : big;
        if (hipMalloc((void**)&a.a, 2 * e) != hipSuccess || hipMalloc((void**)&a.g, 4 * e) != hipSuccess) {
            nn_free_acts(t);
            return HB_ERR_OOM;
        }
    }
    const long P = (long)n * H * W;
    if (hipMalloc((void**)&t->dzb, 2 * big) != hipSuccess || hipMalloc((void**)&t->dzf, 4 * big) != hipSuccess ||
        hipMalloc((void**)&t->yout, 4 * P * 16) != hipSuccess || hipMalloc((void**)&t->hg, 4 * P * 16) != hipSuccess ||
        hipMalloc((void**)&t->part, 4 * 16384) != hipSuccess ||
        hipHostMalloc((void**)&t->hpart, 4 * 16384) != hipSuccess) {
        nn_free_acts(t);
        return HB_ERR_OOM;
    }
    t->n = n;
    t->H = H;
    t->W = W;
    return HB_OK;
}

static void conv_fwd(NNet* t, int li, const Act& in, Act& out, float* yf)
{
    const ConvL& l = t->L[li];
    const dim3 grid((in.W + kStrip - 1) / kStrip, in.H, t->n);
    const size_t lds = 2 * 3 * (kStrip + 2) * (size_t)l.cin;
    const float* b = t->w + l.boff;
    uint16_t* y = yf ? nullptr : out.a;
#define HB_CONV(M, C) k_conv3<M, C><<<grid, 256, lds, t->s>>>(in.a, l.w16, b, in.H, in.W, l.cin, l.relu, y, yf)
    // the network's (output tiles, input channels) pairs with the channel
    // count fixed at compile time; anything else with it at run time
    const int mt = l.cout / 16;
    if (mt == 1 && l.cin == 16) HB_CONV(1, 16);
    else if (mt == 1 && l.cin == 48) HB_CONV(1, 48);
    else if (mt == 2 && l.cin == 16) HB_CONV(2, 16);
    else if (mt == 2 && l.cin == 32) HB_CONV(2, 32);
    else if (mt == 2 && l.cin == 96) HB_CONV(2, 96);
    else if (mt == 4 && l.cin == 32) HB_CONV(4, 32);
    else if (mt == 4 && l.cin == 64) HB_CONV(4, 64);
    else if (mt == 4 && l.cin == 128) HB_CONV(4, 128);
    else if (mt == 1) HB_CONV(1, 0);
    else if (mt == 2) HB_CONV(2, 0);
    else HB_CONV(4, 0);
#undef HB_CONV
}

// backward of layer li: out.g (fp32) -> parameter gradients, and in.g +=
// (or =) the input gradient when want_dx
static void conv_bwd(NNet* t, int li, Act& in, const Act& out, bool want_dx, float* gin_override)
{
    const ConvL& l = t->L[li];
    const long P = (long)t->n * in.H * in.W;
    const long N = P * l.cout;
    k_relu_bwd<<<nn_blocks(N), 256, 0, t->s>>>(out.g, out.a, N, l.relu, t->dzb, t->dzf);
    k_bias_grad<<<l.cout, 256, 0, t->s>>>(t->dzf, P, l.cout, t->gw + l.boff);
    const int tiles = (l.cout / 16) * (9 * l.cin / 16);
    const dim3 g2((tiles + 3) / 4, (unsigned)((P + kPixChunk - 1) / kPixChunk));
    k_conv3_dw<<<g2, 256, 0, t->s>>>(t->dzb, in.a, t->n, in.H, in.W, l.cin, l.cout, t->gw + l.woff);
    if (!want_dx) return;
    // input gradient: the convolution of dz with the flipped, transposed weights
    const dim3 grid((in.W + kStrip - 1) / kStrip, in.H, t->n);
    const size_t lds = 2 * 3 * (kStrip + 2) * (size_t)l.cout;
    float* gx = gin_override ? gin_override : in.g;
    switch (l.cin / 16) {
    case 1: k_conv3<1><<<grid, 256, lds, t->s>>>(t->dzb, l.wt16, nullptr, in.H, in.W, l.cout, 0, nullptr, gx); break;
    case 2: k_conv3<2><<<grid, 256, lds, t->s>>>(t->dzb, l.wt16, nullptr, in.H, in.W, l.cout, 0, nullptr, gx); break;
    case 3: k_conv3<3><<<grid, 256, lds, t->s>>>(t->dzb, l.wt16, nullptr, in.H, in.W, l.cout, 0, nullptr, gx); break;
    case 4: k_conv3<4><<<grid, 256, lds, t->s>>>(t->dzb, l.wt16, nullptr, in.H, in.W, l.cout, 0, nullptr, gx); break;
    case 6: k_conv3<6><<<grid, 256, lds, t->s>>>(t->dzb, l.wt16, nullptr, in.H, in.W, l.cout, 0, nullptr, gx); break;
    default: k_conv3<8><<<grid, 256, lds, t->s>>>(t->dzb, l.wt16, nullptr, in.H, in.W, l.cout, 0, nullptr, gx); break;
    }
}

static void refresh_bf16(NNet* t)
{
    for (ConvL& l : t->L)
        k_weights_bf16<<<nn_blocks((long)l.cout * 9 * l.cin), 256, 0, t->s>>>(t->w + l.woff, l.cout, l.cin, l.w16, l.wt16);
}

// forward pass from the packed input t->A[A_IN]; head output (fp32, 16
// channels) into t->yout
static void forward(NNet* t)
{
    std::vector<Act>& A = t->A;
    const int n = t->n;
    auto pool = [&](const Act& a, Act& b) {
        k_pool2<<<nn_blocks((long)n * b.H * b.W * b.C / 4), 256, 0, t->s>>>(a.a, n, a.H, a.W, a.C, b.a);
    };
    auto upcat = [&](const Act& lo, const Act& skip, Act& out) {
        k_up_concat<<<nn_blocks((long)n * out.H * out.W * out.C / 4), 256, 0, t->s>>>(lo.a, lo.C, skip.a, skip.C, n,
                                                                                       out.H, out.W, out.a);
    };
    conv_fwd(t, 0, A[A_IN], A[A_E0A], nullptr);
    conv_fwd(t, 1, A[A_E0A], A[A_E0], nullptr);
    pool(A[A_E0], A[A_P0]);
    conv_fwd(t, 2, A[A_P0], A[A_E1A], nullptr);
    conv_fwd(t, 3, A[A_E1A], A[A_E1], nullptr);
    pool(A[A_E1], A[A_P1]);
    conv_fwd(t, 4, A[A_P1], A[A_E2A], nullptr);
    conv_fwd(t, 5, A[A_E2A], A[A_E2], nullptr);
    pool(A[A_E2], A[A_P2]);
    conv_fwd(t, 6, A[A_P2], A[A_E3A], nullptr);
    conv_fwd(t, 7, A[A_E3A], A[A_E3], nullptr);
    upcat(A[A_E3], A[A_E2], A[A_C2]);
    conv_fwd(t, 8, A[A_C2], A[A_D2A], nullptr);
    conv_fwd(t, 9, A[A_D2A], A[A_D2], nullptr);
    upcat(A[A_D2], A[A_E1], A[A_C1]);
    conv_fwd(t, 10, A[A_C1], A[A_D1A], nullptr);
    conv_fwd(t, 11, A[A_D1A], A[A_D1], nullptr);
    upcat(A[A_D1], A[A_E0], A[A_C0]);
    conv_fwd(t, 12, A[A_C0], A[A_D0A], nullptr);
    conv_fwd(t, 13, A[A_D0A], A[A_D0], nullptr);
    conv_fwd(t, 14, A[A_D0], A[A_D0], t->yout);   // head: fp32 output only
}

// backward pass from dL/dy of the head output (fp32, [P][16]): fills t->gw
static void backward(NNet* t, float* head_g)
{
    std::vector<Act>& A = t->A;
    const int n = t->n;
    (void)hipMemsetAsync(t->gw, 0, sizeof(float) * t->np, t->s);
    for (Act& a : A) (void)hipMemsetAsync(a.g, 0, sizeof(float) * (long)n * a.H * a.W * a.C, t->s);
    // head: its "output activation" for the ReLU mask is unused (relu = 0)
    Act head;
    head.H = t->H;
    head.W = t->W;
    head.C = 16;
    head.a = A[A_D0].a;
    head.g = head_g;
    conv_bwd(t, 14, A[A_D0], head, true, nullptr);
    conv_bwd(t, 13, A[A_D0A], A[A_D0], true, nullptr);
    conv_bwd(t, 12, A[A_C0], A[A_D0A], true, nullptr);
    auto upcat_bwd = [&](Act& lo, Act& skip, const Act& cat) {
        k_up_concat_bwd_a<<<nn_blocks((long)n * lo.H * lo.W * lo.C), 256, 0, t->s>>>(cat.g, lo.C, skip.C, n, cat.H, cat.W,
                                                                                     lo.g);
        const long P = (long)n * cat.H * cat.W;
        k_up_concat_bwd_s<<<nn_blocks(P * skip.C), 256, 0, t->s>>>(cat.g, lo.C, skip.C, P, skip.g);
    };
    auto pool_bwd = [&](const Act& pooled, Act& full) {
        k_pool2_bwd<<<nn_blocks((long)n * full.H * full.W * full.C), 256, 0, t->s>>>(pooled.g, n, full.H, full.W, full.C,
                                                                                      full.g);
    };
    upcat_bwd(A[A_D1], A[A_E0], A[A_C0]);
    conv_bwd(t, 11, A[A_D1A], A[A_D1], true, nullptr);
    conv_bwd(t, 10, A[A_C1], A[A_D1A], true, nullptr);
    upcat_bwd(A[A_D2], A[A_E1], A[A_C1]);
    conv_bwd(t, 9, A[A_D2A], A[A_D2], true, nullptr);
    conv_bwd(t, 8, A[A_C2], A[A_D2A], true, nullptr);
    upcat_bwd(A[A_E3], A[A_E2], A[A_C2]);
    conv_bwd(t, 7, A[A_E3A], A[A_E3], true, nullptr);
    conv_bwd(t, 6, A[A_P2], A[A_E3A], true, nullptr);
    pool_bwd(A[A_P2], A[A_E2]);
    conv_bwd(t, 5, A[A_E2A], A[A_E2], true, nullptr);
    conv_bwd(t, 4, A[A_P1], A[A_E2A], true, nullptr);
    pool_bwd(A[A_P1], A[A_E1]);
    conv_bwd(t, 3, A[A_E1A], A[A_E1], true, nullptr);
    conv_bwd(t, 2, A[A_P0], A[A_E1A], true, nullptr);
    pool_bwd(A[A_P0], A[A_E0]);
    conv_bwd(t, 1, A[A_E0A], A[A_E0], true, nullptr);
    conv_bwd(t, 0, A[A_IN], A[A_E0A], false, nullptr);
}

// He-normal initial weights from SplitMix64 + Box-Muller, zero biases
static void init_params(NNet* t, uint64_t seed, std::vector<float>& h)
{
    h.assign(t->np, 0.0f);
    uint64_t s = seed;
    auto next = [&]() {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto unif = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
    for (const ConvL& l : t->L) {
        const double sd = std::sqrt(2.0 / (9.0 * l.cin));
        for (long i = 0; i < (long)l.cout * 9 * l.cin; i += 2) {
            const double r = std::sqrt(-2.0 * std::log(unif())), th = 6.283185307179586 * unif();
            h[l.woff + i] = (float)(sd * r * std::cos(th));
            if (i + 1 < (long)l.cout * 9 * l.cin) h[l.woff + i + 1] = (float)(sd * r * std::sin(th));
        }
    }
}

static int nn_make(int in_ch, int out_ch, uint64_t seed, hipStream_t s, NNet** out)
{
    NNet* t = new (std::nothrow) NNet();
    if (!t) return HB_ERR_OOM;
    t->in_ch = in_ch;
    t->out_ch = out_ch;
    t->s = s;
    long off = 0;
    for (int i = 0; i < 15; ++i) {
        ConvL l;
        l.cin = kLay[i][0];
        l.cout = kLay[i][1];
        l.relu = kLay[i][2];
        l.woff = off;
        off += (long)l.cout * 9 * l.cin;
        l.boff = off;
        off += l.cout;
        t->L.push_back(l);
    }
    t->np = off;
    bool ok = hipMalloc((void**)&t->w, 4 * off) == hipSuccess && hipMalloc((void**)&t->gw, 4 * off) == hipSuccess &&
              hipMalloc((void**)&t->m, 4 * off) == hipSuccess && hipMalloc((void**)&t->v, 4 * off) == hipSuccess;
    for (ConvL& l : t->L) {
        const long e = (long)l.cout * 9 * l.cin;
        ok = ok && hipMalloc((void**)&l.w16, 2 * e) == hipSuccess && hipMalloc((void**)&l.wt16, 2 * e) == hipSuccess;
    }
    if (!ok) {
        *out = t;
        return HB_ERR_OOM;
    }
    std::vector<float> h;
    init_params(t, seed, h);
    (void)hipMemcpy(t->w, h.data(), 4 * off, hipMemcpyHostToDevice);
    (void)hipMemset(t->m, 0, 4 * off);
    (void)hipMemset(t->v, 0, 4 * off);
    refresh_bf16(t);
    (void)hipStreamSynchronize(t->s);
    *out = t;
    return HB_OK;
}

static void nn_free(NNet* t)
{
    if (!t) return;
    if (t->s) (void)hipStreamSynchronize(t->s);
    nn_free_acts(t);
    for (ConvL& l : t->L) {
        (void)hipFree(l.w16);
        (void)hipFree(l.wt16);
    }
    (void)hipFree(t->w);
    (void)hipFree(t->gw);
    (void)hipFree(t->m);
    (void)hipFree(t->v);
    if (t->s) (void)hipStreamDestroy(t->s);
    delete t;
}

// input x (device fp32 [n][H][W][in_ch]) packed into the network's input
static int nn_load_input(NNet* t, const float* x, int n, int H, int W)
{
    if (n < 1 || H < 8 || W < 8 || H % 8 || W % 8) return HB_ERR_ARG;
    int rc = nn_shape(t, n, H, W);
    if (rc != HB_OK) return rc;
    const long P = (long)n * H * W;
    k_pack_in<<<nn_blocks(P * 16), 256, 0, t->s>>>(x, P, t->in_ch, 16, t->A[A_IN].a);
    return HB_OK;
}

// loss of the head output against the target, and its gradient into headg
static double nn_loss(NNet* t, const float* target, float* headg)
{
    const long P = (long)t->n * t->H * t->W;
    const unsigned nb = nn_blocks(P * 16);
    k_mse<<<nb, 256, 0, t->s>>>(t->yout, target, P, 16, t->out_ch, headg, t->part);
    (void)hipMemcpyAsync(t->hpart, t->part, 4 * nb, hipMemcpyDeviceToHost, t->s);
    (void)hipStreamSynchronize(t->s);
    double s = 0.0;
    for (unsigned i = 0; i < nb; ++i) s += t->hpart[i];
    return s;
}

int nn_infer(NNet* t, const float* x, int n, int H, int W, float* y)
{
    int rc = nn_load_input(t, x, n, H, W);
    if (rc != HB_OK) return rc;
    forward(t);
    const long P = (long)n * H * W;
    k_unpack_out<<<nn_blocks(P * t->out_ch), 256, 0, t->s>>>(t->yout, P, 16, t->out_ch, y);
    return hipStreamSynchronize(t->s) == hipSuccess ? HB_OK : HB_ERR_DEVICE;
}

}  // namespace hb

using namespace hb;

struct hb_nn : public hb::NNet {};

namespace hb {
NNet* nn_of(hb_nn* nn) { return nn; }
int nn_channels_in(const NNet* t) { return t->in_ch; }
int nn_channels_out(const NNet* t) { return t->out_ch; }
}  // namespace hb

extern "C" {

int hb_nn_create(int in_ch, int out_ch, uint64_t seed, hb_nn** out)
{
    if (!out) return HB_ERR_ARG;
    *out = nullptr;
    if (in_ch < 1 || in_ch > 16 || out_ch < 1 || out_ch > 16) return HB_ERR_ARG;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return HB_ERR_DEVICE;
    NNet* t = nullptr;
    const int rc = nn_make(in_ch, out_ch, seed, s, &t);
    if (rc != HB_OK) {
        nn_free(t);
        return rc;
    }
    *out = static_cast<hb_nn*>(t);
    return HB_OK;
}

void hb_nn_destroy(hb_nn* nn) { nn_free(nn); }

int64_t hb_nn_param_count(const hb_nn* nn) { return nn ? nn->np : 0; }

int hb_nn_get_params(hb_nn* nn, float* host)
{
    if (!nn || !host) return HB_ERR_ARG;
    return hipMemcpy(host, nn->w, 4 * nn->np, hipMemcpyDeviceToHost) == hipSuccess ? HB_OK : HB_ERR_DEVICE;
}

int hb_nn_set_params(hb_nn* nn, const float* host)
{
    if (!nn || !host) return HB_ERR_ARG;
    if (hipMemcpy(nn->w, host, 4 * nn->np, hipMemcpyHostToDevice) != hipSuccess) return HB_ERR_DEVICE;
    refresh_bf16(nn);
    return hipStreamSynchronize(nn->s) == hipSuccess ? HB_OK : HB_ERR_DEVICE;
}

int hb_nn_forward(hb_nn* nn, const float* x, int n, int H, int W, float* y)
{
    if (!nn || !x || !y) return HB_ERR_ARG;
    return nn_infer(nn, x, n, H, W, y);
}

int hb_nn_grad(hb_nn* nn, const float* x, const float* target, int n, int H, int W, double* loss, float* grad_host)
{
    if (!nn || !x || !target) return HB_ERR_ARG;
    int rc = nn_load_input(nn, x, n, H, W);
    if (rc != HB_OK) return rc;
    forward(nn);
    const double L = nn_loss(nn, target, nn->hg);
    backward(nn, nn->hg);
    if (hipStreamSynchronize(nn->s) != hipSuccess) return HB_ERR_DEVICE;
    if (loss) *loss = L;
    if (grad_host && hipMemcpy(grad_host, nn->gw, 4 * nn->np, hipMemcpyDeviceToHost) != hipSuccess) return HB_ERR_DEVICE;
    return HB_OK;
}

int hb_nn_train_step(hb_nn* nn, const float* x, const float* target, int n, int H, int W, float lr, double* loss)
{
    int rc = hb_nn_grad(nn, x, target, n, H, W, loss, nullptr);
    if (rc != HB_OK) return rc;
    ++nn->step;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)nn->step), c2 = 1.0f - std::pow(b2, (float)nn->step);
    k_adam<<<nn_blocks(nn->np), 256, 0, nn->s>>>(nn->w, nn->gw, nn->m, nn->v, nn->np, lr, b1, b2, c1, c2, 1e-8f);
    refresh_bf16(nn);
    return hipStreamSynchronize(nn->s) == hipSuccess ? HB_OK : HB_ERR_DEVICE;
}

}  // extern "C"
