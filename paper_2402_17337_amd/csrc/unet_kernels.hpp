// unet_kernels.hpp -- gfx950 kernels of the learned warm start: a 4-level
// convolutional U-Net (3x3 convolutions, 2x2 average pooling, nearest
// up-sampling, concatenated skips) trained and evaluated on the GPU.
//
// Activations and gradients are BF16 in NHWC layout (pixel-major, the channels
// of a pixel contiguous, channel counts multiples of 8); convolutions multiply
// BF16 operands and accumulate in FP32 on the 16x16x32 BF16 matrix cores;
// weights live in FP32 (master copy and Adam moments) and are rounded to BF16
// for the convolutions.  Kernel weight layout: [cout_pad][9][cin], where tap
// t = 3 (dy + 1) + (dx + 1) multiplies the input pixel (y + dy, x + dx), i.e.
// the master tensor w[co][ci][dy + 1][dx + 1] of a cross-correlation with zero
// padding 1.  Image widths are multiples of 8 at every level, so the 8
// consecutive pixels of one lane's K slice lie in one image row.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ibm {
namespace unet {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kWave = 64;
constexpr int kConvWaves = 4;                        // waves per block of the convolution
constexpr int kConvNB = 2;                           // 16-pixel blocks per wave
constexpr int kConvPix = kConvWaves * kConvNB * 16;  // pixels per block
constexpr int kGradPix = 1024;                       // pixels per weight/bias-gradient partial
constexpr int kEw = 256;                             // threads per block of the elementwise kernels

struct Shape {
    int n, h, w;  // batch, height, width
};

__device__ inline bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int q = 0; q < 8; ++q) z[q] = (bf16)0.0f;
    return z;
}

// D += A B for a 16 x 32 A and a 32 x 16 B spread over the wave: lane l holds
// A row (l % 16) and B column (l % 16), K elements 8 (l / 16) .. 8 (l / 16) + 7;
// D column (l % 16), rows 4 (l / 16) .. 4 (l / 16) + 3.
__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 3x3 convolution with zero padding 1 as an implicit GEMM:
//   y[p, co] = act(bias[co] + sum_{t, ci} wt[co][t][ci] x[p + off(t), ci])
// M = output channels (16 per block row), N = pixels (kConvNB x 16 per wave),
// K = 9 cin in slices of 32 (zero beyond 9 cin).  x: bf16 NHWC, cin channels
// (a multiple of 8); wt: bf16 [>= 16 gridDim.y][9][cin]; bias: f32 or null;
// y: NHWC with cout channels (bf16, or f32 with OUTF32); rows co >= cout are
// computed and dropped.  Grid: (ceil(npix / kConvPix), cout_pad / 16).
template <bool RELU, bool OUTF32>
__global__ __launch_bounds__(kConvWaves * kWave) void k_conv3x3(Shape s, const bf16* __restrict__ x, int cin,
                                                                const bf16* __restrict__ wt,
                                                                const float* __restrict__ bias,
                                                                void* __restrict__ y, int cout) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int g = lane >> 4, col = lane & 15;
    const int co0 = blockIdx.y * 16;
    const int npix = s.n * s.h * s.w;
    const int K = 9 * cin;
    const int nslice = (K + 31) / 32;
    int pn[kConvNB], py[kConvNB], px[kConvNB];
    bool pv[kConvNB];
#pragma unroll
    for (int b = 0; b < kConvNB; ++b) {
        const int p = (blockIdx.x * kConvWaves + wave) * (kConvNB * 16) + b * 16 + col;
        pv[b] = p < npix;
        const int pp = pv[b] ? p : 0;
        px[b] = pp % s.w;
        py[b] = (pp / s.w) % s.h;
        pn[b] = pp / (s.w * s.h);
    }
    f32x4 acc[kConvNB];
#pragma unroll
    for (int b = 0; b < kConvNB; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16* wrow = wt + (size_t)(co0 + col) * K;
    for (int sl = 0; sl < nslice; ++sl) {
        const int k0 = sl * 32 + 8 * g;  // 8 consecutive K indices of one tap (cin % 8 == 0)
        const bool kin = k0 < K;
        const bf16x8 a = kin ? *(const bf16x8*)(wrow + k0) : zero8();
        const int t = kin ? k0 / cin : 0;
        const int ci0 = k0 - t * cin;
        const int dy = t / 3 - 1, dx = t % 3 - 1;
#pragma unroll
        for (int b = 0; b < kConvNB; ++b) {
            const int yy = py[b] + dy, xx = px[b] + dx;
            const bool in = kin && pv[b] && yy >= 0 && yy < s.h && xx >= 0 && xx < s.w;
            const bf16x8 v =
                in ? *(const bf16x8*)(x + ((size_t)(pn[b] * s.h + yy) * s.w + xx) * cin + ci0) : zero8();
            acc[b] = mfma(a, v, acc[b]);
        }
    }
#pragma unroll
    for (int b = 0; b < kConvNB; ++b) {
        if (!pv[b]) continue;
        const size_t p = (size_t)(pn[b] * s.h + py[b]) * s.w + px[b];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int co = co0 + 4 * g + q;
            if (co >= cout) continue;
            float v = acc[b][q] + (bias ? bias[co] : 0.0f);
            if (RELU) v = v > 0.0f ? v : 0.0f;
            if (OUTF32) ((float*)y)[p * cout + co] = v;
            else ((bf16*)y)[p * cout + co] = (bf16)v;
        }
    }
}

// The same convolution with the block's input tile staged in LDS: a block
// computes a (8 PB) x 8 tile of output pixels (4 waves, each PB blocks of 16
// pixels: two rows of 8) for NCO blocks of 16 output channels; the input
// pixels of the tile and its one-pixel halo, with all cin channels, are
// loaded once (zero outside the image) and each K slice's input fragment,
// read from LDS, feeds NCO products.  Grid: (n ceil(h / (8 PB)) ceil(w / 8),
// cout_pad / (16 NCO)); (8 PB + 2) 10 (cin / 8 + 1) <= kTileVec.
constexpr int kTile = 8;
constexpr int kTileVec = 2500;  // 16-byte LDS vectors: 40 000 bytes
template <bool RELU, bool OUTF32, int NCO, int PB>
__global__ __launch_bounds__(4 * kWave) void k_conv3x3_tile(Shape s, const bf16* __restrict__ x, int cin,
                                                           const bf16* __restrict__ wt,
                                                           const float* __restrict__ bias,
                                                           void* __restrict__ y, int cout) {
    constexpr int TH = 8 * PB, TW = kTile;
    __shared__ bf16x8 tile[kTileVec];  // pixel-major, one 16-byte pad per pixel
    const int cs = cin / 8 + 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int g = lane >> 4, col = lane & 15;
    const int tpr = (s.w + TW - 1) / TW, tpc = (s.h + TH - 1) / TH;
    const int tb = blockIdx.x;
    const int bn = tb / (tpr * tpc), rem = tb - bn * tpr * tpc;
    const int y0 = (rem / tpr) * TH, x0 = (rem % tpr) * TW;
    const int nv = cin / 8;
    for (int q = threadIdx.x; q < (TH + 2) * (TW + 2) * nv; q += 4 * kWave) {
        const int pix = q / nv, v = q - pix * nv;
        const int yy = y0 - 1 + pix / (TW + 2), xx = x0 - 1 + pix % (TW + 2);
        bf16x8 val = zero8();
        if (yy >= 0 && yy < s.h && xx >= 0 && xx < s.w)
            val = *(const bf16x8*)(x + ((size_t)(bn * s.h + yy) * s.w + xx) * cin + 8 * v);
        tile[pix * cs + v] = val;
    }
    __syncthreads();
    const int lx = col & 7;
    int ly[PB];
#pragma unroll
    for (int b = 0; b < PB; ++b) ly[b] = 2 * (wave * PB + b) + (col >> 3);
    const int co0 = blockIdx.y * 16 * NCO;
    const int K = 9 * cin;
    const int nslice = (K + 31) / 32;
    f32x4 acc[NCO][PB];
#pragma unroll
    for (int j = 0; j < NCO; ++j)
#pragma unroll
        for (int b = 0; b < PB; ++b) acc[j][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int sl = 0; sl < nslice; ++sl) {
        const int k0 = sl * 32 + 8 * g;
        const bool kin = k0 < K;
        const int t = kin ? k0 / cin : 0;
        const int ci0 = k0 - t * cin;
        const int dy = t / 3 - 1, dx = t % 3 - 1;
        bf16x8 a[NCO];
#pragma unroll
        for (int j = 0; j < NCO; ++j)
            a[j] = kin ? *(const bf16x8*)(wt + (size_t)(co0 + 16 * j + col) * K + k0) : zero8();
#pragma unroll
        for (int b = 0; b < PB; ++b) {
            const bf16x8 v = kin ? tile[((ly[b] + 1 + dy) * (TW + 2) + lx + 1 + dx) * cs + ci0 / 8] : zero8();
#pragma unroll
            for (int j = 0; j < NCO; ++j) acc[j][b] = mfma(a[j], v, acc[j][b]);
        }
    }
#pragma unroll
    for (int b = 0; b < PB; ++b) {
        const int oy = y0 + ly[b], ox = x0 + lx;
        if (oy >= s.h || ox >= s.w) continue;
        const size_t p = (size_t)(bn * s.h + oy) * s.w + ox;
#pragma unroll
        for (int j = 0; j < NCO; ++j) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int co = co0 + 16 * j + 4 * g + q;
                if (co >= cout) continue;
                float v = acc[j][b][q] + (bias ? bias[co] : 0.0f);
                if (RELU) v = v > 0.0f ? v : 0.0f;
                if (OUTF32) ((float*)y)[p * cout + co] = v;
                else ((bf16*)y)[p * cout + co] = (bf16)v;
            }
        }
    }
}

// Weight-gradient partials of a 3x3 convolution, one per kGradPix pixels:
//   part[chunk][co][t cin + ci] = sum_{p in chunk} gz[p, co] x[p + off(t), ci]
// M = co (16 per block), N = (t, ci) (16 per block), K = pixels (32 per
// product).  gz: bf16 NHWC with gs channels of which cout are live; x: bf16
// NHWC with cin channels.  Rows co in [cout, cout_pad) come out zero.  Grid:
// (chunks, cout_pad / 16, ceil(9 cin / 16)); one wave per block.
__global__ __launch_bounds__(kWave) void k_wgrad(Shape s, const bf16* __restrict__ x, int cin,
                                                 const bf16* __restrict__ gz, int gs, int cout, int cout_pad,
                                                 float* __restrict__ part) {
    const int lane = threadIdx.x;
    const int g = lane >> 4, col = lane & 15;
    const int co = blockIdx.y * 16 + col;  // A row of this lane
    const int N = 9 * cin;
    const int nn = blockIdx.z * 16 + col;  // B column of this lane
    const bool nok = nn < N;
    const int t = nok ? nn / cin : 0;
    const int ci = nn - t * cin;
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    const bool cok = co < cout;
    const int npix = s.n * s.h * s.w;
    const int p_begin = blockIdx.x * kGradPix;
    const int p_end = min(npix, p_begin + kGradPix);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int pb = p_begin; pb < p_end; pb += 32) {
        const int p0 = pb + 8 * g;  // this lane's 8 pixels, one image row
        bf16x8 a = zero8(), b = zero8();
        if (p0 < p_end) {
            const int x0 = p0 % s.w, yq = (p0 / s.w) % s.h, nq = p0 / (s.w * s.h);
            const int yy = yq + dy;
            const bool row_in = nok && yy >= 0 && yy < s.h;
            const size_t rbase = (size_t)(nq * s.h + (row_in ? yy : 0)) * s.w;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (cok) a[q] = gz[(size_t)(p0 + q) * gs + co];
                const int xx = x0 + q + dx;
                if (row_in && xx >= 0 && xx < s.w) b[q] = x[(rbase + xx) * cin + ci];
            }
        }
        acc = mfma(a, b, acc);
    }
    float* dst = part + (size_t)blockIdx.x * cout_pad * N;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = blockIdx.y * 16 + 4 * g + q;
        if (nok) dst[(size_t)r * N + nn] = acc[q];
    }
}

// Weight gradient in the master layout (co, ci, 3, 3) from the partials, summed
// in chunk order: gw[co][ci][t] = sum_c part[c][co][t cin + ci], ci < cin_real.
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nchunk, int cout, int cout_pad, int cin,
                               int cin_real, float* __restrict__ gw) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cout * cin_real * 9) return;
    const int t = e % 9, ci = (e / 9) % cin_real, co = e / (9 * cin_real);
    const size_t stride = (size_t)cout_pad * 9 * cin;
    const size_t idx = (size_t)co * 9 * cin + (size_t)t * cin + ci;
    float acc = 0.0f;
    for (int c = 0; c < nchunk; ++c) acc += part[c * stride + idx];
    gw[e] = acc;
}

// Bias-gradient partials: part[chunk][co] = sum_{p in chunk} gz[p, co].  The
// kEw threads of a block split as co = tid % cp (cp: cout rounded up to a power
// of two, <= kEw) and kEw / cp pixel lanes, each summing every (kEw / cp)-th
// pixel of the chunk; the lanes' sums are then added in a fixed tree order.
__global__ __launch_bounds__(kEw) void k_bgrad(int npix, const bf16* __restrict__ gz, int gs, int cout, int cp,
                                               float* __restrict__ part) {
    __shared__ float red[kEw];
    const int co = threadIdx.x % cp, lanes = kEw / cp, l = threadIdx.x / cp;
    const int p0 = blockIdx.x * kGradPix, p1 = min(npix, p0 + kGradPix);
    float acc = 0.0f;
    if (co < cout)
        for (int p = p0 + l; p < p1; p += lanes) acc += (float)gz[(size_t)p * gs + co];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = lanes / 2; o > 0; o >>= 1) {
        if (l < o) red[threadIdx.x] += red[threadIdx.x + o * cp];
        __syncthreads();
    }
    if (l == 0 && co < cout) part[(size_t)blockIdx.x * cout + co] = red[threadIdx.x];
}

__global__ void k_bgrad_reduce(const float* __restrict__ part, int nchunk, int cout, float* __restrict__ gb) {
    const int co = blockIdx.x * blockDim.x + threadIdx.x;
    if (co >= cout) return;
    float acc = 0.0f;
    for (int c = 0; c < nchunk; ++c) acc += part[(size_t)c * cout + co];
    gb[co] = acc;
}

// The elementwise kernels below move 8 channels (16 bytes) per thread; every
// channel count is a multiple of 8.
__device__ inline bf16x8 ld8(const bf16* p) { return *(const bf16x8*)p; }
__device__ inline void st8(bf16* p, bf16x8 v) { *(bf16x8*)p = v; }

// Gradient through the ReLU: gz = g where the layer's output y is positive
// (n elements, a multiple of 8).
__global__ void k_relu_back(size_t n, const bf16* __restrict__ g, const bf16* __restrict__ y,
                            bf16* __restrict__ gz) {
    const size_t i = 8 * ((size_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const bf16x8 gv = ld8(g + i), yv = ld8(y + i);
    bf16x8 o;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (float)yv[q] > 0.0f ? gv[q] : (bf16)0.0f;
    st8(gz + i, o);
}

// 2x2 average pooling (so: the output shape), 8 channels per thread.
__global__ void k_pool(Shape so, int c, const bf16* __restrict__ x, bf16* __restrict__ y) {
    const int cv = c / 8;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)so.n * so.h * so.w * cv) return;
    const int ch = 8 * (int)(i % cv);
    const size_t p = i / cv;
    const int xo = (int)(p % so.w), yo = (int)((p / so.w) % so.h), bn = (int)(p / ((size_t)so.w * so.h));
    const int wi = 2 * so.w, hi = 2 * so.h;
    const size_t b0 = ((size_t)(bn * hi + 2 * yo) * wi + 2 * xo) * c + ch;
    const size_t rs = (size_t)wi * c;
    const bf16x8 a = ld8(x + b0), b = ld8(x + b0 + c), d = ld8(x + b0 + rs), e = ld8(x + b0 + rs + c);
    bf16x8 o;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (bf16)(0.25f * (((float)a[q] + (float)b[q]) + ((float)d[q] + (float)e[q])));
    st8(y + p * c + ch, o);
}

// Gradient of the pooling added to gx (si: the input shape): gx[p] += g[p / 2] / 4.
__global__ void k_pool_back_add(Shape si, int c, const bf16* __restrict__ g, bf16* __restrict__ gx) {
    const int cv = c / 8;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)si.n * si.h * si.w * cv) return;
    const int ch = 8 * (int)(i % cv);
    const size_t p = i / cv;
    const int xi = (int)(p % si.w), yi = (int)((p / si.w) % si.h), bn = (int)(p / ((size_t)si.w * si.h));
    const int wo = si.w / 2, ho = si.h / 2;
    const bf16x8 gv = ld8(g + ((size_t)(bn * ho + yi / 2) * wo + xi / 2) * c + ch);
    bf16x8 xv = ld8(gx + p * c + ch);
#pragma unroll
    for (int q = 0; q < 8; ++q) xv[q] = (bf16)((float)xv[q] + 0.25f * (float)gv[q]);
    st8(gx + p * c + ch, xv);
}

// y = concat(nearest 2x up-sampling of a (ca channels), b (cb channels)) on the
// output shape so, 8 channels per thread.
__global__ void k_up_concat(Shape so, const bf16* __restrict__ a, int ca, const bf16* __restrict__ b, int cb,
                            bf16* __restrict__ y) {
    const int c = ca + cb, cv = c / 8;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)so.n * so.h * so.w * cv) return;
    const int ch = 8 * (int)(i % cv);
    const size_t p = i / cv;
    bf16x8 v;
    if (ch < ca) {
        const int xo = (int)(p % so.w), yo = (int)((p / so.w) % so.h), bn = (int)(p / ((size_t)so.w * so.h));
        v = ld8(a + ((size_t)(bn * (so.h / 2) + yo / 2) * (so.w / 2) + xo / 2) * ca + ch);
    } else {
        v = ld8(b + p * cb + (ch - ca));
    }
    st8(y + p * c + ch, v);
}

// Gradient of k_up_concat: ga[q] = sum of g over the 2x2 block of q (first ca
// channels), gb = the last cb channels of g.  One thread per 8 channels of
// the larger of the two outputs.
__global__ void k_up_concat_back(Shape so, const bf16* __restrict__ g, int ca, int cb, bf16* __restrict__ ga,
                                 bf16* __restrict__ gb) {
    const int c = ca + cb;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int cbv = cb / 8, cav = ca / 8;
    if (i < (size_t)so.n * so.h * so.w * cbv) {
        const size_t p = i / cbv;
        const int ch = 8 * (int)(i % cbv);
        st8(gb + p * cb + ch, ld8(g + p * c + ca + ch));
    }
    const Shape sa = {so.n, so.h / 2, so.w / 2};
    if (i < (size_t)sa.n * sa.h * sa.w * cav) {
        const int ch = 8 * (int)(i % cav);
        const size_t p = i / cav;
        const int xa = (int)(p % sa.w), ya = (int)((p / sa.w) % sa.h), bn = (int)(p / ((size_t)sa.w * sa.h));
        const size_t q0 = ((size_t)(bn * so.h + 2 * ya) * so.w + 2 * xa) * c + ch;
        const size_t rs = (size_t)so.w * c;
        const bf16x8 a = ld8(g + q0), b = ld8(g + q0 + c), d = ld8(g + q0 + rs), e = ld8(g + q0 + rs + c);
        bf16x8 o;
#pragma unroll
        for (int q = 0; q < 8; ++q) o[q] = (bf16)(((float)a[q] + (float)b[q]) + ((float)d[q] + (float)e[q]));
        st8(ga + p * ca + ch, o);
    }
}

// NCHW float (c channels) -> NHWC bf16 with cp >= c channels (the rest zero).
__global__ void k_pack_nchw(Shape s, int c, int cp, const float* __restrict__ x, bf16* __restrict__ y) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t hw = (size_t)s.h * s.w;
    if (i >= (size_t)s.n * hw * cp) return;
    const int ch = (int)(i % cp);
    const size_t p = i / cp;
    y[i] = ch < c ? (bf16)x[((p / hw) * c + ch) * hw + p % hw] : (bf16)0.0f;
}

// NHWC float (c channels) -> NCHW float.
__global__ void k_unpack_nhwc(Shape s, int c, const float* __restrict__ x, float* __restrict__ y) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t hw = (size_t)s.h * s.w;
    if (i >= (size_t)s.n * hw * c) return;
    const size_t r = i % hw, ch = (i / hw) % c, bn = i / (hw * c);
    y[i] = x[(bn * hw + r) * c + ch];
}

// Mean squared error of out against t over npix values, each image b of hw
// values weighted by w[b] (w null: 1): g = 2 w (out - t) / npix as bf16 in
// channel 0 of an 8-channel NHWC gradient (channels 1..7 zero), and per-block
// partial sums of w (out - t)^2.
__global__ __launch_bounds__(kEw) void k_mse(int npix, int hw, const float* __restrict__ out,
                                             const float* __restrict__ t, const float* __restrict__ w,
                                             bf16* __restrict__ g, float* __restrict__ part) {
    __shared__ float red[kEw];
    const int i = blockIdx.x * kEw + threadIdx.x;
    float d = 0.0f, wi = 0.0f;
    if (i < npix) {
        d = out[i] - t[i];
        wi = w ? w[i / hw] : 1.0f;
        bf16x8 v = zero8();
        v[0] = (bf16)(2.0f * wi * d / (float)npix);
        *(bf16x8*)(g + (size_t)i * 8) = v;
    }
    red[threadIdx.x] = wi * d * d;
    __syncthreads();
    for (int o = kEw / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] = sum of the n partials / npix (one block).
__global__ __launch_bounds__(kEw) void k_loss_reduce(const float* __restrict__ part, int n, int npix,
                                                     float* __restrict__ out) {
    __shared__ float red[kEw];
    float acc = 0.0f;
    for (int i = threadIdx.x; i < n; i += kEw) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kEw / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] / (float)npix;
}

// One Adam update (Kingma & Ba 2015, Algorithm 1) of the FP32 master
// parameters; c1 = 1 - beta1^step, c2 = 1 - beta2^step.
__global__ void k_adam(size_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float c1, float c2, float eps) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Master weights w (co_n, ci_n, 3, 3) -> bf16 [co_pad][9][ci_pad] (forward) or,
// for the input gradient, the flipped transpose [ci_pad][9][co_pad] with tap
// 8 - t (a 3x3 correlation with it maps output gradients to input gradients).
__global__ void k_pack_weights(const float* __restrict__ w, int co_n, int ci_n, int co_pad, int ci_pad,
                               int transposed, bf16* __restrict__ out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)co_pad * 9 * ci_pad) return;
    if (!transposed) {
        const int ci = (int)(i % ci_pad), t = (int)((i / ci_pad) % 9), co = (int)(i / ((size_t)9 * ci_pad));
        out[i] = (co < co_n && ci < ci_n) ? (bf16)w[((size_t)co * ci_n + ci) * 9 + t] : (bf16)0.0f;
    } else {
        const int co = (int)(i % co_pad), t = (int)((i / co_pad) % 9), ci = (int)(i / ((size_t)9 * co_pad));
        out[i] = (co < co_n && ci < ci_n) ? (bf16)w[((size_t)co * ci_n + ci) * 9 + (8 - t)] : (bf16)0.0f;
    }
}

}  // namespace unet
}  // namespace ibm
