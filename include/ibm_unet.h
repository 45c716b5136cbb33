/*
 * ibm_unet.h -- C ABI of the learned warm start of the pressure-correction
 * solve: a small convolutional U-Net, trained and evaluated on the MI355X
 * (gfx950) by hand-written BF16 matrix-core kernels.
 *
 * The paper starts each pressure Poisson solve of its fractional-step method
 * (Sec. 2.2-2.3) from the previous solution; this network is an extension of
 * that method, not part of the paper.  It maps three feature maps to one
 * output map of the same size:
 *
 *   network    4 levels, widths 16/32/64/128, 3x3 convolutions with zero
 *              padding 1, bias and ReLU after every convolution but the last;
 *              level l -> l+1 by 2x2 averaging, l+1 -> l by repeating each
 *              value over a 2x2 block and concatenating the level-l features
 *              after the up-sampled ones; two convolutions per level on each
 *              side, one output convolution to 1 channel.  Layers, in the
 *              order of the parameter vector: enc0a (3->16), enc0b, enc1a
 *              (16->32), enc1b, enc2a (32->64), enc2b, mid_a (64->128), mid_b,
 *              dec2a (192->64), dec2b, dec1a (96->32), dec1b, dec0a (48->16),
 *              dec0b, out (16->1);
 *   parameters float32, per layer the weights (cout, cin, 3, 3), then the
 *              biases (cout); weight [co][ci][a][b] multiplies the input pixel
 *              (y + a - 1, x + b - 1);
 *   arithmetic activations and gradients in bfloat16, products on the BF16
 *              matrix cores with float32 accumulation, float32 master weights
 *              rounded to bfloat16 for every convolution, biases added in
 *              float32, loss and Adam in float32;
 *   training   mean squared error over all output values, Adam (Kingma & Ba
 *              2015) on the float32 master weights.
 *
 * Image tensors at the boundary are float32 NCHW (batch, channels, height,
 * width), row-major, device memory.  height must be a multiple of 8 and width
 * a multiple of 64 (every level's width a multiple of 8).  Return codes are
 * those of ibm.h.  A network is bound to the HIP stream given at creation;
 * every call is stream-ordered on it and borrows device pointers for the
 * duration of the call only.  A network is not thread-safe.
 */
#ifndef IBM_UNET_H
#define IBM_UNET_H

#include <stddef.h>
#include <stdint.h>

#include "ibm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define IBM_UNET_IN_CHANNELS 3
#define IBM_UNET_LAYERS 15

typedef struct ibm_unet ibm_unet;

/* Number of float32 parameters (weights and biases of all layers). */
size_t ibm_unet_param_count(void);

/* Device workspace for batches of up to max_batch images of height x width,
 * in bytes; 0 if the shape is invalid.  Pure function. */
size_t ibm_unet_workspace_bytes(int32_t max_batch, int32_t height, int32_t width);

/* Create a network with all parameters zero (load them with
 * ibm_unet_set_params).  workspace: device memory of at least
 * ibm_unet_workspace_bytes bytes, 256-byte aligned, owned by the caller and
 * kept alive until ibm_unet_destroy.  hip_stream: hipStream_t, borrowed (NULL
 * = null stream).  IBM_ERR_INVALID for a bad shape or a small or misaligned
 * workspace. */
int32_t ibm_unet_create(int32_t max_batch, int32_t height, int32_t width, void* workspace,
                        size_t workspace_bytes, void* hip_stream, ibm_unet** out);

/* Host copies in and out of the parameter vector (n = ibm_unet_param_count()).
 * set_params also resets the Adam moments and step count.  Synchronous. */
int32_t ibm_unet_set_params(ibm_unet* net, const float* host, size_t n);
int32_t ibm_unet_get_params(ibm_unet* net, float* host, size_t n);
/* Gradient of the last ibm_unet_loss_grad call, same layout.  Synchronous. */
int32_t ibm_unet_get_grads(ibm_unet* net, float* host, size_t n);

/* Inference: x (batch, 3, height, width) -> y (batch, 1, height, width),
 * float32 device arrays, 1 <= batch <= max_batch.  Enqueued only. */
int32_t ibm_unet_forward(ibm_unet* net, const float* x_dev, float* y_dev, int32_t batch);

/* Forward, mean squared error against target (batch, 1, height, width) and
 * backward: the parameter gradient is kept in the network.  weight_dev
 * (device, batch floats, nullable = all 1) weights each image's squared
 * errors: loss = sum_b weight[b] sum_p (y - target)^2 / (batch height width).
 * loss (host, nullable): the loss, which synchronizes the stream; NULL
 * enqueues only. */
int32_t ibm_unet_loss_grad(ibm_unet* net, const float* x_dev, const float* target_dev, const float* weight_dev,
                           int32_t batch, float* loss);

/* One Adam update with the kept gradient: m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2, w -= lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps)
 * at update k = 1, 2, ...  Enqueued only. */
int32_t ibm_unet_adam_step(ibm_unet* net, float lr, float beta1, float beta2, float eps);

/* ibm_unet_loss_grad then ibm_unet_adam_step(lr, 0.9, 0.999, 1e-8). */
int32_t ibm_unet_train_step(ibm_unet* net, const float* x_dev, const float* target_dev, const float* weight_dev,
                            int32_t batch, float lr, float* loss);

void ibm_unet_destroy(ibm_unet* net);
const char* ibm_unet_last_error(const ibm_unet* net);

/* One convolution layer of the network on its own, for numerical checks:
 * the operands are rounded to bfloat16 exactly as in the network, results
 * come out in float32 without the final bfloat16 rounding.
 *   x[n][cin][h][w], w[cout][cin][3][3], b[cout] (nullable), gy[n][cout][h][w]:
 *   device float32; out: device float32;
 *   op IBM_UNET_CONV_FORWARD:  out[n][cout][h][w] = conv(x, w) + b (no ReLU);
 *   op IBM_UNET_CONV_DGRAD:    out[n][cin][h][w]  = gradient of sum(gy conv(x, w))
 *                                                    with respect to x;
 *   op IBM_UNET_CONV_WGRAD:    out[cout*cin*9 + cout] = its gradient with respect
 *                                                    to w, then to b.
 * 1 <= cin, cout <= 256; h >= 1; w a multiple of 8.  workspace:
 * device, ibm_unet_conv_workspace_bytes bytes, 256-byte aligned.  Enqueued on
 * hip_stream. */
#define IBM_UNET_CONV_FORWARD 0
#define IBM_UNET_CONV_DGRAD 1
#define IBM_UNET_CONV_WGRAD 2
size_t ibm_unet_conv_workspace_bytes(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout);
int32_t ibm_unet_conv3x3(int32_t op, int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout,
                         const float* x, const float* wt, const float* b, const float* gy, float* out,
                         void* workspace, size_t workspace_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* IBM_UNET_H */
