"""Oracle of the learned warm start: a 4-level convolutional U-Net that maps
(Poisson right-hand side, previous pressure correction, body mask) to an
initial pressure correction, in plain PyTorch CPU operations in float64.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the GPU path never imports it.

The network (channel widths 16/32/64/128, 3x3 kernels, bias and ReLU after
every convolution but the last) is the warm-start network this code extends
the method with; it is not part of the paper, whose
pressure solve starts from the previous step.  Layout of every tensor:
(batch, channels, height, width).  Down-sampling is a 2x2 average, up-sampling
repeats each value over a 2x2 block, skips are concatenated after the
up-sampled channels.  Library primitives (conv2d, avg_pool2d, interpolate,
autograd) are the steps; nothing is fused or reordered.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

WIDTHS = (16, 32, 64, 128)
IN_CHANNELS = 3

# (name, in channels, out channels, ReLU after) in evaluation order
def layer_specs(widths=WIDTHS, cin=IN_CHANNELS):
    w0, w1, w2, w3 = widths
    return [
        ("enc0a", cin, w0, True), ("enc0b", w0, w0, True),
        ("enc1a", w0, w1, True), ("enc1b", w1, w1, True),
        ("enc2a", w1, w2, True), ("enc2b", w2, w2, True),
        ("mid_a", w2, w3, True), ("mid_b", w3, w3, True),
        ("dec2a", w3 + w2, w2, True), ("dec2b", w2, w2, True),
        ("dec1a", w2 + w1, w1, True), ("dec1b", w1, w1, True),
        ("dec0a", w1 + w0, w0, True), ("dec0b", w0, w0, True),
        ("out", w0, 1, False),
    ]


def init_params(seed=0, widths=WIDTHS, cin=IN_CHANNELS):
    """He-uniform weights (bound sqrt(6 / fan_in)) and zero biases from a
    seeded numpy generator; weights (out, in, 3, 3), float64."""
    rng = np.random.default_rng(seed)
    params = {}
    for name, ci, co, _ in layer_specs(widths, cin):
        bound = math.sqrt(6.0 / (ci * 9))
        params[name + ".w"] = rng.uniform(-bound, bound, size=(co, ci, 3, 3))
        params[name + ".b"] = np.zeros(co)
    return params


def _conv(x, p, name, relu):
    y = F.conv2d(x, p[name + ".w"], p[name + ".b"], padding=1)
    return F.relu(y) if relu else y


def forward(params, x):
    """x: (B, 3, H, W) float64 tensor with H, W divisible by 8 -> (B, 1, H, W);
    the channel widths follow from the parameters."""
    p = {k: (v if torch.is_tensor(v) else torch.as_tensor(v)) for k, v in params.items()}
    s0 = _conv(_conv(x, p, "enc0a", True), p, "enc0b", True)
    s1 = _conv(_conv(F.avg_pool2d(s0, 2), p, "enc1a", True), p, "enc1b", True)
    s2 = _conv(_conv(F.avg_pool2d(s1, 2), p, "enc2a", True), p, "enc2b", True)
    m = _conv(_conv(F.avg_pool2d(s2, 2), p, "mid_a", True), p, "mid_b", True)
    d2 = torch.cat([F.interpolate(m, scale_factor=2, mode="nearest"), s2], dim=1)
    d2 = _conv(_conv(d2, p, "dec2a", True), p, "dec2b", True)
    d1 = torch.cat([F.interpolate(d2, scale_factor=2, mode="nearest"), s1], dim=1)
    d1 = _conv(_conv(d1, p, "dec1a", True), p, "dec1b", True)
    d0 = torch.cat([F.interpolate(d1, scale_factor=2, mode="nearest"), s0], dim=1)
    d0 = _conv(_conv(d0, p, "dec0a", True), p, "dec0b", True)
    return _conv(d0, p, "out", False)


def loss_and_grads(params, x, target, weight=None):
    """Mean squared error over all outputs and its gradient with respect to
    every parameter (autograd), all in float64.  weight (per image, optional)
    multiplies each image's squared errors before the mean."""
    p = {k: torch.tensor(np.asarray(v, dtype=np.float64), requires_grad=True) for k, v in params.items()}
    xt = torch.as_tensor(np.asarray(x, dtype=np.float64))
    tt = torch.as_tensor(np.asarray(target, dtype=np.float64))
    y = forward(p, xt)
    sq = (y - tt) ** 2
    if weight is not None:
        sq = sq * torch.as_tensor(np.asarray(weight, dtype=np.float64)).reshape(-1, 1, 1, 1)
    loss = torch.mean(sq)
    loss.backward()
    return loss.item(), {k: v.grad.numpy().copy() for k, v in p.items()}, y.detach().numpy()


def conv3x3(x, w, b, relu):
    """One convolution layer (zero padding 1), float64 numpy in and out."""
    y = F.conv2d(torch.as_tensor(x), torch.as_tensor(w), torch.as_tensor(b), padding=1)
    return (F.relu(y) if relu else y).numpy()


def conv3x3_grads(x, w, dy):
    """Gradients of sum(dy * conv3x3(x, w, b)) with respect to x, w and b."""
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.zeros(w.shape[0], dtype=torch.float64, requires_grad=True)
    y = F.conv2d(xt, wt, bt, padding=1)
    (y * torch.as_tensor(dy)).sum().backward()
    return xt.grad.numpy(), wt.grad.numpy(), bt.grad.numpy()


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) in float64; returns the
    new (param, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v
