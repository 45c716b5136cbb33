"""Pins of the U-Net oracle (learned warm start) against definitions that do
not go through it: the convolution sum written out, central finite
differences of the loss, the adjoint pairs of pooling and up-sampling, and the
Adam recurrence evaluated by hand."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet as U


def _direct_conv(x, w, b):
    B, C, H, W = x.shape
    O = w.shape[0]
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((B, O, H, W))
    for o in range(O):
        for dy in range(3):
            for dx in range(3):
                y[:, o] += np.einsum("bchw,c->bhw", xp[:, :, dy:dy + H, dx:dx + W], w[o, :, dy, dx])
        y[:, o] += b[o]
    return y


def test_conv_is_the_written_out_sum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 7, 6))
    w = rng.standard_normal((4, 5, 3, 3))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(U.conv3x3(x, w, b, False), _direct_conv(x, w, b), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(U.conv3x3(x, w, b, True), np.maximum(_direct_conv(x, w, b), 0.0),
                               rtol=1e-12, atol=1e-12)


def test_conv_gradients_are_the_adjoint_sums():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 3, 6, 5))
    w = rng.standard_normal((2, 3, 3, 3))
    dy = rng.standard_normal((1, 2, 6, 5))
    gx, gw, gb = U.conv3x3_grads(x, w, dy)
    # d/dw[o,c,a,e] sum(dy * y) = sum_p dy[o,p] x_pad[c, p + (a, e)]
    xp = np.zeros((1, 3, 8, 7))
    xp[:, :, 1:-1, 1:-1] = x
    gw_ref = np.zeros_like(w)
    for o in range(2):
        for c in range(3):
            for a in range(3):
                for e in range(3):
                    gw_ref[o, c, a, e] = np.sum(dy[0, o] * xp[0, c, a:a + 6, e:e + 5])
    np.testing.assert_allclose(gw, gw_ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gb, dy.sum(axis=(0, 2, 3)), rtol=1e-12)
    # <dy, conv(x)> = <conv^T(dy), x>: the x gradient is the adjoint
    np.testing.assert_allclose(np.sum(dy * _direct_conv(x, w, np.zeros(2))), np.sum(gx * x), rtol=1e-12)


def test_pool_and_upsample_are_adjoint_up_to_a_factor():
    rng = np.random.default_rng(2)
    a = torch.as_tensor(rng.standard_normal((1, 2, 8, 6)))
    c = torch.as_tensor(rng.standard_normal((1, 2, 4, 3)))
    lhs = float(torch.sum(F.avg_pool2d(a, 2) * c))
    rhs = float(torch.sum(a * F.interpolate(c, scale_factor=2, mode="nearest"))) / 4.0
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_unet_shapes_and_parameter_count():
    p = U.init_params(0)
    x = torch.zeros((2, 3, 16, 24), dtype=torch.float64)
    y = U.forward(p, x)
    assert tuple(y.shape) == (2, 1, 16, 24)
    n = sum(v.size for v in p.values())
    w0, w1, w2, w3 = U.WIDTHS
    by_hand = 9 * (3 * w0 + w0 * w0 + w0 * w1 + w1 * w1 + w1 * w2 + w2 * w2 + w2 * w3 + w3 * w3
                   + (w3 + w2) * w2 + w2 * w2 + (w2 + w1) * w1 + w1 * w1 + (w1 + w0) * w0 + w0 * w0 + w0)
    by_hand += 2 * w0 + 2 * w1 + 2 * w2 + 2 * w3 + 2 * w2 + 2 * w1 + 2 * w0 + 1
    assert n == by_hand


@pytest.mark.parametrize("name", ["enc0a.w", "mid_b.w", "dec1a.w", "out.w", "dec0b.b"])
def test_unet_gradient_matches_central_differences(name):
    rng = np.random.default_rng(3)
    p = U.init_params(4, widths=(4, 4, 4, 4))
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    x = rng.standard_normal((1, 3, 8, 8))
    t = rng.standard_normal((1, 1, 8, 8))

    def loss(pp):
        y = U.forward(pp, torch.as_tensor(x))
        return float(torch.mean((y - torch.as_tensor(t)) ** 2))

    _, g, _ = U.loss_and_grads(p, x, t)   # narrow widths (4, 4, 4, 4): a fast check
    flat = p[name].reshape(-1)
    for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
        h = 1e-6
        pp = {k: v.copy() for k, v in p.items()}
        pp[name].reshape(-1)[idx] += h
        lp = loss(pp)
        pp[name].reshape(-1)[idx] -= 2 * h
        lm = loss(pp)
        fd = (lp - lm) / (2 * h)
        assert abs(g[name].reshape(-1)[idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (name, idx)


def test_adam_step_by_hand():
    p, g = np.array([1.0, -2.0]), np.array([0.5, 0.25])
    m, v = np.zeros(2), np.zeros(2)
    p1, m1, v1 = U.adam_step(p, g, m, v, 1, lr=0.1)
    # the first step moves each parameter by lr * sign(g) (up to eps)
    np.testing.assert_allclose(p1, p - 0.1 * np.sign(g), rtol=1e-7)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(v1, 0.001 * g * g)


def test_weighted_loss_is_the_per_image_weighted_mean():
    # weights (1, 0) keep only the first image: the batch mean over 2 images
    # is half the mean of that image alone, and so are its gradients
    rng = np.random.default_rng(9)
    p = U.init_params(9)
    x = rng.standard_normal((2, 3, 16, 16))
    t = rng.standard_normal((2, 1, 16, 16))
    lw, gw, _ = U.loss_and_grads(p, x, t, weight=(1.0, 0.0))
    l1, g1, _ = U.loss_and_grads(p, x[:1], t[:1])
    assert abs(lw - 0.5 * l1) <= 1e-12 * l1
    for k in g1:
        np.testing.assert_allclose(gw[k], 0.5 * g1[k], rtol=1e-10, atol=1e-14)
    lu, _, _ = U.loss_and_grads(p, x, t)
    lo, _, _ = U.loss_and_grads(p, x, t, weight=(1.0, 1.0))
    assert lu == lo

