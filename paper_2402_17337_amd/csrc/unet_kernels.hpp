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

// Bias-gradient partials: part[chunk][co] = sum_{p in chunk} gz[p, co].
__global__ void k_bgrad(int npix, const bf16* __restrict__ gz, int gs, int cout, float* __restrict__ part) {
    const int co = threadIdx.x;
    if (co >= cout) return;
    const int p0 = blockIdx.x * kGradPix, p1 = min(npix, p0 + kGradPix);
    float acc = 0.0f;
    for (int p = p0; p < p1; ++p) acc += (float)gz[(size_t)p * gs + co];
    part[(size_t)blockIdx.x * cout + co] = acc;
}

__global__ void k_bgrad_reduce(const float* __restrict__ part, int nchunk, int cout, float* __restrict__ gb) {
    const int co = blockIdx.x * blockDim.x + threadIdx.x;
    if (co >= cout) return;
    float acc = 0.0f;
    for (int c = 0; c < nchunk; ++c) acc += part[(size_t)c * cout + co];
    gb[co] = acc;
}

// Gradient through the ReLU: gz = g where the layer's output y is positive.
__global__ void k_relu_back(size_t n, const bf16* __restrict__ g, const bf16* __restrict__ y,
                            bf16* __restrict__ gz) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    gz[i] = (float)y[i] > 0.0f ? g[i] : (bf16)0.0f;
}

// 2x2 average pooling (so: the output shape).
__global__ void k_pool(Shape so, int c, const bf16* __restrict__ x, bf16* __restrict__ y) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)so.n * so.h * so.w * c) return;
    const int ch = (int)(i % c);
    const size_t p = i / c;
    const int xo = (int)(p % so.w), yo = (int)((p / so.w) % so.h), bn = (int)(p / ((size_t)so.w * so.h));
    const int wi = 2 * so.w, hi = 2 * so.h;
    const size_t b0 = ((size_t)(bn * hi + 2 * yo) * wi + 2 * xo) * c + ch;
    const size_t rs = (size_t)wi * c;
    const float sum = ((float)x[b0] + (float)x[b0 + c]) + ((float)x[b0 + rs] + (float)x[b0 + rs + c]);
    y[i] = (bf16)(0.25f * sum);
}

// Gradient of the pooling added to gx (si: the input shape): gx[p] += g[p / 2] / 4.
__global__ void k_pool_back_add(Shape si, int c, const bf16* __restrict__ g, bf16* __restrict__ gx) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)si.n * si.h * si.w * c) return;
    const int ch = (int)(i % c);
    const size_t p = i / c;
    const int xi = (int)(p % si.w), yi = (int)((p / si.w) % si.h), bn = (int)(p / ((size_t)si.w * si.h));
    const int wo = si.w / 2, ho = si.h / 2;
    const float v = 0.25f * (float)g[((size_t)(bn * ho + yi / 2) * wo + xi / 2) * c + ch];
    gx[i] = (bf16)((float)gx[i] + v);
}

// y = concat(nearest 2x up-sampling of a (ca channels), b (cb channels)) on the
// output shape so.
__global__ void k_up_concat(Shape so, const bf16* __restrict__ a, int ca, const bf16* __restrict__ b, int cb,
                            bf16* __restrict__ y) {
    const int c = ca + cb;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)so.n * so.h * so.w * c) return;
    const int ch = (int)(i % c);
    const size_t p = i / c;
    if (ch < ca) {
        const int xo = (int)(p % so.w), yo = (int)((p / so.w) % so.h), bn = (int)(p / ((size_t)so.w * so.h));
        y[i] = a[((size_t)(bn * (so.h / 2) + yo / 2) * (so.w / 2) + xo / 2) * ca + ch];
    } else {
        y[i] = b[p * cb + (ch - ca)];
    }
}

// Gradient of k_up_concat: ga[q] = sum of g over the 2x2 block of q (first ca
// channels), gb = the last cb channels of g.
__global__ void k_up_concat_back(Shape so, const bf16* __restrict__ g, int ca, int cb, bf16* __restrict__ ga,
                                 bf16* __restrict__ gb) {
    const int c = ca + cb;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nb = (size_t)so.n * so.h * so.w * cb;
    if (i < nb) {
        const size_t p = i / cb;
        gb[i] = g[p * c + ca + (int)(i % cb)];
    }
    const Shape sa = {so.n, so.h / 2, so.w / 2};
    if (i < (size_t)sa.n * sa.h * sa.w * ca) {
        const int ch = (int)(i % ca);
        const size_t p = i / ca;
        const int xa = (int)(p % sa.w), ya = (int)((p / sa.w) % sa.h), bn = (int)(p / ((size_t)sa.w * sa.h));
        const size_t q0 = ((size_t)(bn * so.h + 2 * ya) * so.w + 2 * xa) * c + ch;
        const size_t rs = (size_t)so.w * c;
        ga[i] = (bf16)(((float)g[q0] + (float)g[q0 + c]) + ((float)g[q0 + rs] + (float)g[q0 + rs + c]));
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
