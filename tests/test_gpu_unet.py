"""Parity of the warm-start network's BF16 matrix-core kernels with the float64
CPU oracle of the same network.

Tolerances.  The kernels round every operand of a convolution (input,
weights, upstream gradient) to bfloat16 and accumulate the exact products in
float32.  The single-layer tests feed the oracle the same bfloat16-rounded
operands, so the only difference is float32 summation of K products: the
standard bound |s - s_hat| <= gamma_K sum |a_i b_i| with gamma_K = K u / (1 - K u),
u = 2^-24 (taken twice over, since the matrix-core summation order is not
specified), with the absolute sums computed by the oracle on |operands|.

The whole-network tests also round every stored activation and activation
gradient to bfloat16 (unit roundoff 2^-8 each).  With 15 convolution layers
plus pooling, up-sampling and the loss gradient on the path, a first-order
bound of the relative error is about 20 roundings x 2^-8 = 8e-2 if all
rounding errors lined up; independent errors add in quadrature,
sqrt(20) x 2^-8 / sqrt(3) = 1e-2.  The tests use 3e-2 for the output and loss
and 8e-2 for each parameter gradient (the worst-case figure; gradients of
early layers pass through every rounding twice).
"""
import numpy as np
import pytest
import torch

from oracle import unet as OU

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bf(a):
    """Round to bfloat16 (nearest-even), returned as float64."""
    return torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _gamma(k):
    u = 2.0 ** -24
    return 2.0 * k * u / (1.0 - k * u)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32), device=DEV)


CONV_CASES = [  # n, h, w, cin, cout
    (1, 5, 8, 3, 1),       # smallest: padded input and output channels, one partial
    (2, 12, 24, 16, 16),
    (2, 7, 16, 48, 32),    # odd height, K = 432 (14 slices, ragged)
    (2, 24, 48, 32, 64),   # 2304 pixels: three gradient partials, the last ragged
    (1, 8, 64, 192, 16),   # widest input of the network (the LDS tile's limit)
    (1, 6, 16, 200, 24),   # wider than the LDS tile: the untiled kernel
]


@pytest.mark.parametrize("n,h,w,cin,cout", CONV_CASES)
def test_conv_forward_matches_oracle(n, h, w, cin, cout):
    _need_gpu()
    from paper_2402_17337_amd import unet as U
    rng = np.random.default_rng(100 + cin + cout)
    x = rng.standard_normal((n, cin, h, w))
    wt = rng.standard_normal((cout, cin, 3, 3)) / np.sqrt(9 * cin)
    b = rng.standard_normal(cout)
    out = U.conv3x3(U.CONV_FORWARD, x=_dev(x), w=_dev(wt), b=_dev(b)).cpu().numpy().astype(np.float64)
    xr, wr, br = _bf(x), _bf(wt), np.asarray(np.float32(b), np.float64)
    ref = OU.conv3x3(xr, wr, br, False)
    bound = _gamma(9 * cin + 1) * (OU.conv3x3(np.abs(xr), np.abs(wr), np.abs(br), False)) + 1e-30
    err = np.abs(out - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


@pytest.mark.parametrize("n,h,w,cin,cout", CONV_CASES)
def test_conv_input_gradient_matches_oracle(n, h, w, cin, cout):
    _need_gpu()
    from paper_2402_17337_amd import unet as U
    rng = np.random.default_rng(200 + cin + cout)
    x = rng.standard_normal((n, cin, h, w))
    wt = rng.standard_normal((cout, cin, 3, 3))
    gy = rng.standard_normal((n, cout, h, w))
    gx = U.conv3x3(U.CONV_DGRAD, w=_dev(wt), gy=_dev(gy), n=n, h=h, wd=w, cin=cin,
                   cout=cout).cpu().numpy().astype(np.float64)
    wr, gyr = _bf(wt), _bf(gy)
    ref = OU.conv3x3_grads(x, wr, gyr)[0]
    bound = _gamma(9 * cout) * OU.conv3x3_grads(x, np.abs(wr), np.abs(gyr))[0] + 1e-30
    err = np.abs(gx - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


@pytest.mark.parametrize("n,h,w,cin,cout", CONV_CASES)
def test_conv_weight_and_bias_gradients_match_oracle(n, h, w, cin, cout):
    _need_gpu()
    from paper_2402_17337_amd import unet as U
    rng = np.random.default_rng(300 + cin + cout)
    x = rng.standard_normal((n, cin, h, w))
    wt = rng.standard_normal((cout, cin, 3, 3))
    gy = rng.standard_normal((n, cout, h, w))
    g = U.conv3x3(U.CONV_WGRAD, x=_dev(x), w=_dev(wt), gy=_dev(gy)).cpu().numpy().astype(np.float64)
    gw, gb = g[:cout * cin * 9].reshape(cout, cin, 3, 3), g[cout * cin * 9:]
    xr, gyr = _bf(x), _bf(gy)
    _, ref_w, ref_b = OU.conv3x3_grads(xr, wt, gyr)
    _, abs_w, abs_b = OU.conv3x3_grads(np.abs(xr), wt, np.abs(gyr))
    npix = n * h * w
    assert np.all(np.abs(gw - ref_w) <= _gamma(npix) * abs_w + 1e-30)
    assert np.all(np.abs(gb - ref_b) <= _gamma(npix) * abs_b + 1e-30)


# ---------------------------------------------------------------------------
# whole network
# ---------------------------------------------------------------------------
def _problem(seed, B, H, W):
    rng = np.random.default_rng(seed)
    p = OU.init_params(seed)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)  # exercise the bias path
    x = rng.standard_normal((B, 3, H, W))
    t = rng.standard_normal((B, 1, H, W))
    return p, x, t


def _bf_params(p):
    return {k: (_bf(v) if k.endswith(".w") else np.asarray(np.float32(v), np.float64)) for k, v in p.items()}


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@pytest.mark.parametrize("B,H,W", [(2, 16, 64), (1, 24, 128)])
def test_network_forward_matches_oracle(B, H, W):
    _need_gpu()
    from paper_2402_17337_amd import unet as U
    p, x, _ = _problem(1, B, H, W)
    net = U.UNet(B, H, W)
    net.set_params(p)
    y = net.forward(_dev(x)).cpu().numpy().astype(np.float64)
    ref = OU.forward(_bf_params(p), torch.as_tensor(_bf(x))).numpy()
    assert _rel(y, ref) < 3e-2, _rel(y, ref)


def test_network_batch_subset_is_bitwise_the_same():
    _need_gpu()
    from paper_2402_17337_amd import unet as U
    p, x, _ = _problem(2, 3, 16, 64)
    net = U.UNet(3, 16, 64)
    net.set_params(p)
    y3 = net.forward(_dev(x)).cpu().numpy()
    y1 = net.forward(_dev(x[1:2])).cpu().numpy()
    assert np.array_equal(y1[0], y3[1])


@pytest.mark.parametrize("weight", [None, (0.25, 3.0)])
def test_network_loss_and_gradients_match_oracle(weight):
    _need_gpu()
    from paper_2402_17337_amd import unet as U
    B, H, W = 2, 16, 64
    p, x, t = _problem(3, B, H, W)
    net = U.UNet(B, H, W)
    net.set_params(p)
    loss = net.loss_grad(_dev(x), _dev(t), None if weight is None else _dev(np.array(weight)))
    g = U.unflatten_params(net.get_grads().astype(np.float64))
    ref_loss, ref_g, _ = OU.loss_and_grads(_bf_params(p), _bf(x), np.float32(t).astype(np.float64), weight)
    assert abs(loss - ref_loss) <= 3e-2 * ref_loss
    worst = max((_rel(g[k], ref_g[k]), k) for k in ref_g)
    assert worst[0] < 8e-2, worst


def test_gradients_are_deterministic():
    _need_gpu()
    from paper_2402_17337_amd import unet as U
    p, x, t = _problem(4, 2, 16, 64)
    net = U.UNet(2, 16, 64)
    net.set_params(p)
    net.loss_grad(_dev(x), _dev(t))
    g1 = net.get_grads()
    net.loss_grad(_dev(x), _dev(t))
    assert np.array_equal(g1, net.get_grads())


def test_adam_updates_match_the_oracle_recurrence():
    _need_gpu()
    from paper_2402_17337_amd import unet as U
    p, x, t = _problem(5, 2, 16, 64)
    net = U.UNet(2, 16, 64)
    net.set_params(p)
    w = U.flatten_params(p).astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for k in (1, 2, 3):
        net.loss_grad(_dev(x), _dev(t))
        g = net.get_grads().astype(np.float64)
        net.adam_step(1e-3)
        w, m, v = OU.adam_step(w, g, m, v, k, 1e-3)
        got = net.get_params().astype(np.float64)
        # float32 arithmetic of one update on values of size ~1: a few ulps of w
        # plus a few ulps of the lr-sized step
        assert np.max(np.abs(got - w)) < 1e-6, (k, np.max(np.abs(got - w)))
        w = got  # continue from the device's float32 weights


def test_training_reduces_the_loss():
    _need_gpu()
    from paper_2402_17337_amd import unet as U
    B, H, W = 4, 32, 64
    rng = np.random.default_rng(6)
    net = U.UNet(B, H, W)
    net.set_params(OU.init_params(6))
    # a smooth target the network can fit: a low-pass of channel 0
    x = rng.standard_normal((B, 3, H, W))
    k = np.ones(5) / 5
    t = np.apply_along_axis(lambda r: np.convolve(r, k, "same"), 3, x[:, :1])
    xd, td = _dev(x), _dev(t)
    first = net.train_step(xd, td, 2e-3)
    for _ in range(60):
        last = net.train_step(xd, td, 2e-3)
    assert np.isfinite(last) and last < 0.5 * first, (first, last)
