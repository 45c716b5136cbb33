// unet_lib.hip -- host side of the learned warm start (include/ibm_unet.h):
// workspace layout, forward and backward schedules of the U-Net and the
// single-layer entry point.  Every arithmetic step runs in the kernels of
// unet_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "ibm_unet.h"
#include "unet_internal.hpp"
#include "unet_kernels.hpp"

using namespace ibm::unet;

namespace {

constexpr int kLevels = 4;
constexpr int kWidths[kLevels] = {16, 32, 64, 128};

inline int pad8(int c) { return (c + 7) / 8 * 8; }
inline int pad16(int c) { return (c + 15) / 16 * 16; }
inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }
inline int pow2_at_least(int c) {
    int p = 1;
    while (p < c) p <<= 1;
    return p;
}

struct LayerSpec {
    const char* name;
    int cin, cout, relu, level;
};

// Evaluation order; also the order of the parameter vector.
const LayerSpec kSpecs[IBM_UNET_LAYERS] = {
    {"enc0a", IBM_UNET_IN_CHANNELS, 16, 1, 0}, {"enc0b", 16, 16, 1, 0},
    {"enc1a", 16, 32, 1, 1}, {"enc1b", 32, 32, 1, 1},
    {"enc2a", 32, 64, 1, 2}, {"enc2b", 64, 64, 1, 2},
    {"mid_a", 64, 128, 1, 3}, {"mid_b", 128, 128, 1, 3},
    {"dec2a", 192, 64, 1, 2}, {"dec2b", 64, 64, 1, 2},
    {"dec1a", 96, 32, 1, 1}, {"dec1b", 32, 32, 1, 1},
    {"dec0a", 48, 16, 1, 0}, {"dec0b", 16, 16, 1, 0},
    {"out", 16, 1, 0, 0},
};

size_t param_count() {
    size_t n = 0;
    for (const LayerSpec& L : kSpecs) n += (size_t)L.cout * L.cin * 9 + L.cout;
    return n;
}

// Sub-allocation of one device workspace: offsets first (sizing pass), then
// pointers (binding pass).
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        T* p = base ? (T*)(base + off) : nullptr;
        off += align256(count * sizeof(T));
        return p;
    }
};

struct Layer {
    LayerSpec s;
    int cin8, cin16, cout8, cout16;
    size_t w_off, b_off;  // into the parameter vector
    bf16* wf;             // [cout16][9][cin8]
    bf16* wt;             // [cin16][9][cout8]
};

}  // namespace

struct ibm_unet {
    int max_batch, h, w;
    hipStream_t stream;
    size_t nparam;
    float *params, *grads, *m, *v;
    Layer L[IBM_UNET_LAYERS];
    // activations, bf16 NHWC (see plan())
    bf16 *x0, *a0, *s0, *p0, *a1, *s1, *p1, *a2, *s2, *p2, *am, *mm;
    bf16 *c2, *b2, *d2, *c1, *b1, *d1, *c0, *b0, *d0;
    float* y;
    // gradients
    bf16* gy;
    bf16 *gA[kLevels], *gB[kLevels], *gz[kLevels];
    bf16 *gs0, *gs1, *gs2;
    float *part, *bpart, *lpart, *loss_dev;
    size_t part_elems, bpart_elems;
    int adam_k;
    std::string err;
};

namespace {

Shape level_shape(int n, int h, int w, int l) { return Shape{n, h >> l, w >> l}; }
size_t npix(const Shape& s) { return (size_t)s.n * s.h * s.w; }
int nchunk(const Shape& s) { return (int)((npix(s) + kGradPix - 1) / kGradPix); }

bool shape_ok(int b, int h, int w) {
    if (b < 1 || h < 8 || w < 64 || h % 8 || w % 64) return false;
    return (double)b * h * w * 192 < 2e9;  // element indices of the widest level fit in int ranges used
}

// Lays out (or sizes, with a null base) the whole workspace.
void plan(ibm_unet* u, Arena& A) {
    const int B = u->max_batch;
    size_t P[kLevels];
    for (int l = 0; l < kLevels; ++l) P[l] = npix(level_shape(B, u->h, u->w, l));
    u->nparam = param_count();
    u->params = A.take<float>(u->nparam);
    u->grads = A.take<float>(u->nparam);
    u->m = A.take<float>(u->nparam);
    u->v = A.take<float>(u->nparam);
    size_t off = 0, part = 0, bpart = 0;
    for (int i = 0; i < IBM_UNET_LAYERS; ++i) {
        Layer& L = u->L[i];
        L.s = kSpecs[i];
        L.cin8 = pad8(L.s.cin);
        L.cin16 = pad16(L.s.cin);
        L.cout8 = pad8(L.s.cout);
        L.cout16 = pad16(L.s.cout);
        L.w_off = off;
        off += (size_t)L.s.cout * L.s.cin * 9;
        L.b_off = off;
        off += L.s.cout;
        L.wf = A.take<bf16>((size_t)L.cout16 * 9 * L.cin8);
        L.wt = A.take<bf16>((size_t)L.cin16 * 9 * L.cout8);
        const Shape s = level_shape(B, u->h, u->w, L.s.level);
        part = std::max(part, (size_t)nchunk(s) * L.cout16 * 9 * L.cin8);
        bpart = std::max(bpart, (size_t)nchunk(s) * L.s.cout);
    }
    u->x0 = A.take<bf16>(P[0] * 8);
    u->a0 = A.take<bf16>(P[0] * 16);
    u->s0 = A.take<bf16>(P[0] * 16);
    u->p0 = A.take<bf16>(P[1] * 16);
    u->a1 = A.take<bf16>(P[1] * 32);
    u->s1 = A.take<bf16>(P[1] * 32);
    u->p1 = A.take<bf16>(P[2] * 32);
    u->a2 = A.take<bf16>(P[2] * 64);
    u->s2 = A.take<bf16>(P[2] * 64);
    u->p2 = A.take<bf16>(P[3] * 64);
    u->am = A.take<bf16>(P[3] * 128);
    u->mm = A.take<bf16>(P[3] * 128);
    u->c2 = A.take<bf16>(P[2] * 192);
    u->b2 = A.take<bf16>(P[2] * 64);
    u->d2 = A.take<bf16>(P[2] * 64);
    u->c1 = A.take<bf16>(P[1] * 96);
    u->b1 = A.take<bf16>(P[1] * 32);
    u->d1 = A.take<bf16>(P[1] * 32);
    u->c0 = A.take<bf16>(P[0] * 48);
    u->b0 = A.take<bf16>(P[0] * 16);
    u->d0 = A.take<bf16>(P[0] * 16);
    u->y = A.take<float>(P[0]);
    u->gy = A.take<bf16>(P[0] * 8);
    const int gmax[kLevels] = {48, 96, 192, 128};  // widest gradient per level
    for (int l = 0; l < kLevels; ++l) {
        u->gA[l] = A.take<bf16>(P[l] * gmax[l]);
        u->gB[l] = A.take<bf16>(P[l] * gmax[l]);
        u->gz[l] = A.take<bf16>(P[l] * kWidths[l]);
    }
    u->gs0 = A.take<bf16>(P[0] * 16);
    u->gs1 = A.take<bf16>(P[1] * 32);
    u->gs2 = A.take<bf16>(P[2] * 64);
    u->part_elems = part;
    u->bpart_elems = bpart;
    u->part = A.take<float>(part);
    u->bpart = A.take<float>(bpart);
    u->lpart = A.take<float>((P[0] + kEw - 1) / kEw);
    u->loss_dev = A.take<float>(1);
}

inline unsigned blocks(size_t n, int t = kEw) { return (unsigned)((n + t - 1) / t); }

#define UNET_TRY(expr)                                                    \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) {                                           \
            u->err = std::string(#expr) + ": " + hipGetErrorString(e_);   \
            return IBM_ERR_HIP;                                           \
        }                                                                 \
    } while (0)

#define UNET_LAUNCHED()                                                   \
    do {                                                                  \
        hipError_t e_ = hipGetLastError();                                \
        if (e_ != hipSuccess) {                                           \
            u->err = std::string("kernel launch: ") + hipGetErrorString(e_); \
            return IBM_ERR_HIP;                                           \
        }                                                                 \
    } while (0)

// y = act(conv(x) + b): the LDS-tiled kernel for cin <= kTileCin, sharing
// each input fragment across up to 4 blocks of 16 output channels; rows16 is
// the padded number of weight rows (a multiple of 16).
template <bool RELU, bool OUTF32>
void launch_conv(Shape s, const bf16* x, int cin, const bf16* wt, const float* bias, void* y, int cout, int rows16,
                 hipStream_t st) {
    const int nblk = rows16 / 16;
    // pixel blocks per wave: as many as the LDS tile holds, up to 4 (a
    // narrow layer otherwise gives each block too little work)
    const int cs = cin / 8 + 1;
    const int pb = (34 * 10 * cs <= kTileVec) ? 4 : (18 * 10 * cs <= kTileVec) ? 2 : (10 * 10 * cs <= kTileVec) ? 1 : 0;
    if (pb == 0) {
        k_conv3x3<RELU, OUTF32><<<dim3(blocks(npix(s), kConvPix), nblk), kConvWaves * kWave, 0, st>>>(
            s, x, cin, wt, bias, y, cout);
        return;
    }
    const int th = 8 * pb;
    const unsigned tiles = (unsigned)(s.n * ((s.h + th - 1) / th) * ((s.w + kTile - 1) / kTile));
    const int nco = nblk % 4 == 0 ? 4 : nblk % 2 == 0 ? 2 : 1;
    const dim3 grid(tiles, nblk / nco), bl(4 * kWave);
#define CONV_TILE(NCO, PB) k_conv3x3_tile<RELU, OUTF32, NCO, PB><<<grid, bl, 0, st>>>(s, x, cin, wt, bias, y, cout)
    if (nco == 4) {
        if (pb == 4) CONV_TILE(4, 4); else if (pb == 2) CONV_TILE(4, 2); else CONV_TILE(4, 1);
    } else if (nco == 2) {
        if (pb == 4) CONV_TILE(2, 4); else if (pb == 2) CONV_TILE(2, 2); else CONV_TILE(2, 1);
    } else {
        if (pb == 4) CONV_TILE(1, 4); else if (pb == 2) CONV_TILE(1, 2); else CONV_TILE(1, 1);
    }
#undef CONV_TILE
}

// y = act(conv(x) + b) of layer L on shape s (bf16 out, or f32 for the last).
void conv_forward(ibm_unet* u, const Layer& L, Shape s, const bf16* x, void* y) {
    const float* bias = u->params + L.b_off;
    if (!L.s.relu)
        launch_conv<false, true>(s, x, L.cin8, L.wf, bias, y, L.s.cout, L.cout16, u->stream);
    else
        launch_conv<true, false>(s, x, L.cin8, L.wf, bias, y, L.s.cout, L.cout16, u->stream);
}

// Backward of layer L: g = gradient at its output (cout8 channels), y = its
// output (for the ReLU), x = its input.  Writes the parameter gradients and,
// when gx is not null, the input gradient (cin8 channels).
void conv_backward(ibm_unet* u, const Layer& L, Shape s, const bf16* x, const bf16* y, const bf16* g, bf16* gz,
                   bf16* gx) {
    const size_t P = npix(s);
    const bf16* gzv = g;
    if (L.s.relu) {
        k_relu_back<<<blocks(P * L.cout8 / 8), kEw, 0, u->stream>>>(P * L.cout8, g, y, gz);
        gzv = gz;
    }
    const int nc = nchunk(s);
    k_wgrad<<<dim3(nc, L.cout16 / 16, (9 * L.cin8 + 15) / 16), kWave, 0, u->stream>>>(
        s, x, L.cin8, gzv, L.cout8, L.s.cout, L.cout16, u->part);
    const int nw = L.s.cout * L.s.cin * 9;
    k_wgrad_reduce<<<blocks(nw), kEw, 0, u->stream>>>(u->part, nc, L.s.cout, L.cout16, L.cin8, L.s.cin,
                                                      u->grads + L.w_off);
    k_bgrad<<<nc, kEw, 0, u->stream>>>((int)P, gzv, L.cout8, L.s.cout, pow2_at_least(L.s.cout), u->bpart);
    k_bgrad_reduce<<<1, 128, 0, u->stream>>>(u->bpart, nc, L.s.cout, u->grads + L.b_off);
    if (gx) launch_conv<false, false>(s, gzv, L.cout8, L.wt, nullptr, gx, L.cin8, L.cin16, u->stream);
}

void pack_weights(ibm_unet* u) {
    for (Layer& L : u->L) {
        const float* w = u->params + L.w_off;
        k_pack_weights<<<blocks((size_t)L.cout16 * 9 * L.cin8), kEw, 0, u->stream>>>(w, L.s.cout, L.s.cin, L.cout16,
                                                                                     L.cin8, 0, L.wf);
        k_pack_weights<<<blocks((size_t)L.cin16 * 9 * L.cout8), kEw, 0, u->stream>>>(w, L.s.cout, L.s.cin, L.cout8,
                                                                                     L.cin16, 1, L.wt);
    }
}

int32_t forward(ibm_unet* u, const float* x, int B) {
    Shape S[kLevels];
    for (int l = 0; l < kLevels; ++l) S[l] = level_shape(B, u->h, u->w, l);
    const Layer* L = u->L;
    k_pack_nchw<<<blocks(npix(S[0]) * 8), kEw, 0, u->stream>>>(S[0], IBM_UNET_IN_CHANNELS, 8, x, u->x0);
    conv_forward(u, L[0], S[0], u->x0, u->a0);
    conv_forward(u, L[1], S[0], u->a0, u->s0);
    k_pool<<<blocks(npix(S[1]) * 2), kEw, 0, u->stream>>>(S[1], 16, u->s0, u->p0);
    conv_forward(u, L[2], S[1], u->p0, u->a1);
    conv_forward(u, L[3], S[1], u->a1, u->s1);
    k_pool<<<blocks(npix(S[2]) * 4), kEw, 0, u->stream>>>(S[2], 32, u->s1, u->p1);
    conv_forward(u, L[4], S[2], u->p1, u->a2);
    conv_forward(u, L[5], S[2], u->a2, u->s2);
    k_pool<<<blocks(npix(S[3]) * 8), kEw, 0, u->stream>>>(S[3], 64, u->s2, u->p2);
    conv_forward(u, L[6], S[3], u->p2, u->am);
    conv_forward(u, L[7], S[3], u->am, u->mm);
    k_up_concat<<<blocks(npix(S[2]) * 24), kEw, 0, u->stream>>>(S[2], u->mm, 128, u->s2, 64, u->c2);
    conv_forward(u, L[8], S[2], u->c2, u->b2);
    conv_forward(u, L[9], S[2], u->b2, u->d2);
    k_up_concat<<<blocks(npix(S[1]) * 12), kEw, 0, u->stream>>>(S[1], u->d2, 64, u->s1, 32, u->c1);
    conv_forward(u, L[10], S[1], u->c1, u->b1);
    conv_forward(u, L[11], S[1], u->b1, u->d1);
    k_up_concat<<<blocks(npix(S[0]) * 6), kEw, 0, u->stream>>>(S[0], u->d1, 32, u->s0, 16, u->c0);
    conv_forward(u, L[12], S[0], u->c0, u->b0);
    conv_forward(u, L[13], S[0], u->b0, u->d0);
    conv_forward(u, L[14], S[0], u->d0, u->y);
    UNET_LAUNCHED();
    return IBM_OK;
}

int32_t backward(ibm_unet* u, int B) {
    Shape S[kLevels];
    for (int l = 0; l < kLevels; ++l) S[l] = level_shape(B, u->h, u->w, l);
    const Layer* L = u->L;
    bf16 **gA = u->gA, **gB = u->gB, **gz = u->gz;
    // level 0, decoder
    conv_backward(u, L[14], S[0], u->d0, nullptr, u->gy, nullptr, gA[0]);  // g d0 (16)
    conv_backward(u, L[13], S[0], u->b0, u->d0, gA[0], gz[0], gB[0]);     // g b0 (16)
    conv_backward(u, L[12], S[0], u->c0, u->b0, gB[0], gz[0], gA[0]);     // g c0 (48)
    k_up_concat_back<<<blocks(npix(S[0]) * 2), kEw, 0, u->stream>>>(S[0], gA[0], 32, 16, gA[1], u->gs0);
    // level 1, decoder
    conv_backward(u, L[11], S[1], u->b1, u->d1, gA[1], gz[1], gB[1]);     // g b1 (32)
    conv_backward(u, L[10], S[1], u->c1, u->b1, gB[1], gz[1], gA[1]);     // g c1 (96)
    k_up_concat_back<<<blocks(npix(S[1]) * 4), kEw, 0, u->stream>>>(S[1], gA[1], 64, 32, gA[2], u->gs1);
    // level 2, decoder
    conv_backward(u, L[9], S[2], u->b2, u->d2, gA[2], gz[2], gB[2]);      // g b2 (64)
    conv_backward(u, L[8], S[2], u->c2, u->b2, gB[2], gz[2], gA[2]);      // g c2 (192)
    k_up_concat_back<<<blocks(npix(S[2]) * 8), kEw, 0, u->stream>>>(S[2], gA[2], 128, 64, gA[3], u->gs2);
    // level 3
    conv_backward(u, L[7], S[3], u->am, u->mm, gA[3], gz[3], gB[3]);      // g am (128)
    conv_backward(u, L[6], S[3], u->p2, u->am, gB[3], gz[3], gA[3]);      // g p2 (64)
    k_pool_back_add<<<blocks(npix(S[2]) * 8), kEw, 0, u->stream>>>(S[2], 64, gA[3], u->gs2);
    // level 2, encoder
    conv_backward(u, L[5], S[2], u->a2, u->s2, u->gs2, gz[2], gB[2]);     // g a2 (64)
    conv_backward(u, L[4], S[2], u->p1, u->a2, gB[2], gz[2], gA[2]);      // g p1 (32)
    k_pool_back_add<<<blocks(npix(S[1]) * 4), kEw, 0, u->stream>>>(S[1], 32, gA[2], u->gs1);
    // level 1, encoder
    conv_backward(u, L[3], S[1], u->a1, u->s1, u->gs1, gz[1], gB[1]);     // g a1 (32)
    conv_backward(u, L[2], S[1], u->p0, u->a1, gB[1], gz[1], gA[1]);      // g p0 (16)
    k_pool_back_add<<<blocks(npix(S[0]) * 2), kEw, 0, u->stream>>>(S[0], 16, gA[1], u->gs0);
    // level 0, encoder
    conv_backward(u, L[1], S[0], u->a0, u->s0, u->gs0, gz[0], gB[0]);     // g a0 (16)
    conv_backward(u, L[0], S[0], u->x0, u->a0, gB[0], gz[0], nullptr);
    UNET_LAUNCHED();
    return IBM_OK;
}

int32_t check_net(const ibm_unet* u) { return u ? IBM_OK : IBM_ERR_INVALID; }

}  // namespace

namespace ibm {
namespace unet {

hipStream_t net_stream(const ibm_unet* u) { return u->stream; }
void net_shape(const ibm_unet* u, int* max_batch, int* h, int* w) {
    *max_batch = u->max_batch;
    *h = u->h;
    *w = u->w;
}

}  // namespace unet
}  // namespace ibm

extern "C" {

size_t ibm_unet_param_count(void) { return param_count(); }

size_t ibm_unet_workspace_bytes(int32_t max_batch, int32_t height, int32_t width) {
    if (!shape_ok(max_batch, height, width)) return 0;
    ibm_unet u{};
    u.max_batch = max_batch;
    u.h = height;
    u.w = width;
    Arena A;
    plan(&u, A);
    return A.off;
}

int32_t ibm_unet_create(int32_t max_batch, int32_t height, int32_t width, void* workspace, size_t workspace_bytes,
                        void* hip_stream, ibm_unet** out) {
    if (!out) return IBM_ERR_INVALID;
    *out = nullptr;
    const size_t need = ibm_unet_workspace_bytes(max_batch, height, width);
    if (need == 0 || !workspace || workspace_bytes < need || ((uintptr_t)workspace & 255)) return IBM_ERR_INVALID;
    ibm_unet* u = new ibm_unet();
    u->max_batch = max_batch;
    u->h = height;
    u->w = width;
    u->stream = (hipStream_t)hip_stream;
    Arena A;
    A.base = (char*)workspace;
    plan(u, A);
    // zero parameters, moments and (once) every buffer, so padded channels
    // and unused rows read as zero
    hipError_t e = hipMemsetAsync(workspace, 0, need, u->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(u->stream);
    if (e != hipSuccess) {
        delete u;
        return IBM_ERR_HIP;
    }
    *out = u;
    return IBM_OK;
}

int32_t ibm_unet_set_params(ibm_unet* u, const float* host, size_t n) {
    if (check_net(u) || !host || n != u->nparam) return IBM_ERR_INVALID;
    UNET_TRY(hipMemcpyAsync(u->params, host, n * sizeof(float), hipMemcpyHostToDevice, u->stream));
    UNET_TRY(hipMemsetAsync(u->m, 0, n * sizeof(float), u->stream));
    UNET_TRY(hipMemsetAsync(u->v, 0, n * sizeof(float), u->stream));
    u->adam_k = 0;
    pack_weights(u);
    UNET_LAUNCHED();
    UNET_TRY(hipStreamSynchronize(u->stream));
    return IBM_OK;
}

int32_t ibm_unet_get_params(ibm_unet* u, float* host, size_t n) {
    if (check_net(u) || !host || n != u->nparam) return IBM_ERR_INVALID;
    UNET_TRY(hipMemcpyAsync(host, u->params, n * sizeof(float), hipMemcpyDeviceToHost, u->stream));
    UNET_TRY(hipStreamSynchronize(u->stream));
    return IBM_OK;
}

int32_t ibm_unet_get_grads(ibm_unet* u, float* host, size_t n) {
    if (check_net(u) || !host || n != u->nparam) return IBM_ERR_INVALID;
    UNET_TRY(hipMemcpyAsync(host, u->grads, n * sizeof(float), hipMemcpyDeviceToHost, u->stream));
    UNET_TRY(hipStreamSynchronize(u->stream));
    return IBM_OK;
}

int32_t ibm_unet_forward(ibm_unet* u, const float* x, float* y, int32_t batch) {
    if (check_net(u) || !x || !y || batch < 1 || batch > u->max_batch) return IBM_ERR_INVALID;
    const int32_t rc = forward(u, x, batch);
    if (rc) return rc;
    const size_t P = (size_t)batch * u->h * u->w;
    UNET_TRY(hipMemcpyAsync(y, u->y, P * sizeof(float), hipMemcpyDeviceToDevice, u->stream));
    return IBM_OK;
}

int32_t ibm_unet_loss_grad(ibm_unet* u, const float* x, const float* target, const float* weight, int32_t batch,
                           float* loss) {
    if (check_net(u) || !x || !target || batch < 1 || batch > u->max_batch) return IBM_ERR_INVALID;
    int32_t rc = forward(u, x, batch);
    if (rc) return rc;
    const int P = batch * u->h * u->w;
    const int nb = (int)blocks(P);
    k_mse<<<nb, kEw, 0, u->stream>>>(P, u->h * u->w, u->y, target, weight, u->gy, u->lpart);
    k_loss_reduce<<<1, kEw, 0, u->stream>>>(u->lpart, nb, P, u->loss_dev);
    UNET_LAUNCHED();
    rc = backward(u, batch);
    if (rc) return rc;
    if (loss) {
        UNET_TRY(hipMemcpyAsync(loss, u->loss_dev, sizeof(float), hipMemcpyDeviceToHost, u->stream));
        UNET_TRY(hipStreamSynchronize(u->stream));
    }
    return IBM_OK;
}

int32_t ibm_unet_adam_step(ibm_unet* u, float lr, float beta1, float beta2, float eps) {
    if (check_net(u) || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return IBM_ERR_INVALID;
    u->adam_k += 1;
    const float c1 = (float)(1.0 - std::pow((double)beta1, u->adam_k));
    const float c2 = (float)(1.0 - std::pow((double)beta2, u->adam_k));
    k_adam<<<blocks(u->nparam), kEw, 0, u->stream>>>(u->nparam, u->params, u->grads, u->m, u->v, lr, beta1, beta2,
                                                     c1, c2, eps);
    pack_weights(u);
    UNET_LAUNCHED();
    return IBM_OK;
}

int32_t ibm_unet_train_step(ibm_unet* u, const float* x, const float* target, const float* weight, int32_t batch,
                            float lr, float* loss) {
    const int32_t rc = ibm_unet_loss_grad(u, x, target, weight, batch, loss);
    if (rc) return rc;
    return ibm_unet_adam_step(u, lr, 0.9f, 0.999f, 1e-8f);
}

void ibm_unet_destroy(ibm_unet* u) {
    if (!u) return;
    (void)hipStreamSynchronize(u->stream);
    delete u;
}

const char* ibm_unet_last_error(const ibm_unet* u) { return u ? u->err.c_str() : "null network"; }

// ---------------------------------------------------------------------------
// single layer
// ---------------------------------------------------------------------------
namespace {

struct ConvPlan {
    bf16 *xb, *gb, *wf, *wt;
    float *tmp, *part, *bpart;
};

void conv_plan(int n, int h, int w, int cin, int cout, Arena& A, ConvPlan& c) {
    const size_t P = (size_t)n * h * w;
    const Shape s{n, h, w};
    c.xb = A.take<bf16>(P * pad8(cin));
    c.gb = A.take<bf16>(P * pad8(cout));
    c.wf = A.take<bf16>((size_t)pad16(cout) * 9 * pad8(cin));
    c.wt = A.take<bf16>((size_t)pad16(cin) * 9 * pad8(cout));
    c.tmp = A.take<float>(P * std::max(cin, cout));
    c.part = A.take<float>((size_t)nchunk(s) * pad16(cout) * 9 * pad8(cin));
    c.bpart = A.take<float>((size_t)nchunk(s) * cout);
}

bool conv_shape_ok(int n, int h, int w, int cin, int cout) {
    return n >= 1 && h >= 1 && w >= 8 && w % 8 == 0 && cin >= 1 && cin <= 256 && cout >= 1 && cout <= 256 &&
           (double)n * h * w * 256 < 2e9;
}

}  // namespace

size_t ibm_unet_conv_workspace_bytes(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout) {
    if (!conv_shape_ok(n, h, w, cin, cout)) return 0;
    Arena A;
    ConvPlan c;
    conv_plan(n, h, w, cin, cout, A, c);
    return A.off;
}

int32_t ibm_unet_conv3x3(int32_t op, int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout, const float* x,
                         const float* wt, const float* b, const float* gy, float* out, void* workspace,
                         size_t workspace_bytes, void* hip_stream) {
    const size_t need = ibm_unet_conv_workspace_bytes(n, h, w, cin, cout);
    if (need == 0 || !workspace || workspace_bytes < need || ((uintptr_t)workspace & 255) || !out || !wt)
        return IBM_ERR_INVALID;
    if ((op == IBM_UNET_CONV_FORWARD && !x) || (op == IBM_UNET_CONV_DGRAD && !gy) ||
        (op == IBM_UNET_CONV_WGRAD && (!x || !gy)) || op < 0 || op > 2)
        return IBM_ERR_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    Arena A;
    A.base = (char*)workspace;
    ConvPlan c;
    conv_plan(n, h, w, cin, cout, A, c);
    const Shape s{n, h, w};
    const size_t P = npix(s);
    const int ci8 = pad8(cin), co8 = pad8(cout), ci16 = pad16(cin), co16 = pad16(cout);
    if (x) k_pack_nchw<<<blocks(P * ci8), kEw, 0, st>>>(s, cin, ci8, x, c.xb);
    if (gy) k_pack_nchw<<<blocks(P * co8), kEw, 0, st>>>(s, cout, co8, gy, c.gb);
    if (op == IBM_UNET_CONV_FORWARD) {
        k_pack_weights<<<blocks((size_t)co16 * 9 * ci8), kEw, 0, st>>>(wt, cout, cin, co16, ci8, 0, c.wf);
        launch_conv<false, true>(s, c.xb, ci8, c.wf, b, c.tmp, cout, co16, st);
        k_unpack_nhwc<<<blocks(P * cout), kEw, 0, st>>>(s, cout, c.tmp, out);
    } else if (op == IBM_UNET_CONV_DGRAD) {
        k_pack_weights<<<blocks((size_t)ci16 * 9 * co8), kEw, 0, st>>>(wt, cout, cin, co8, ci16, 1, c.wt);
        launch_conv<false, true>(s, c.gb, co8, c.wt, nullptr, c.tmp, cin, ci16, st);
        k_unpack_nhwc<<<blocks(P * cin), kEw, 0, st>>>(s, cin, c.tmp, out);
    } else {
        const int nc = nchunk(s);
        k_wgrad<<<dim3(nc, co16 / 16, (9 * ci8 + 15) / 16), kWave, 0, st>>>(s, c.xb, ci8, c.gb, co8, cout, co16,
                                                                           c.part);
        k_wgrad_reduce<<<blocks((size_t)cout * cin * 9), kEw, 0, st>>>(c.part, nc, cout, co16, ci8, cin, out);
        k_bgrad<<<nc, kEw, 0, st>>>((int)P, c.gb, co8, cout, pow2_at_least(cout), c.bpart);
        k_bgrad_reduce<<<blocks(cout), kEw, 0, st>>>(c.bpart, nc, cout, out + (size_t)cout * cin * 9);
    }
    return hipGetLastError() == hipSuccess ? IBM_OK : IBM_ERR_HIP;
}

}  // extern "C"
