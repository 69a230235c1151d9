"""Pins of the oracle's learned-flagger arithmetic against things other than
itself: library convolutions (scipy, torch on the CPU), the adjoint identity of
a linear map, central finite differences of the whole network, closed forms of
the loss and of Adam's first steps, and invariances of the tile input."""
import numpy as np
import pytest

import oracle


def _rng(seed):
    return np.random.default_rng(seed)


def test_conv_single_channel_matches_scipy_correlate2d():
    from scipy.signal import correlate2d
    g = _rng(1)
    x = g.standard_normal((1, 1, 7, 11))
    w = g.standard_normal((1, 1, 3, 3))
    b = np.array([0.37])
    y = oracle.conv3x3(x, w, b)
    ref = correlate2d(x[0, 0], w[0, 0], mode="same", boundary="fill") + b[0]
    assert np.allclose(y[0, 0], ref, rtol=0, atol=1e-12)


def test_conv_multi_channel_matches_torch_conv2d():
    import torch
    g = _rng(2)
    for ci, co in [(1, 16), (16, 16), (16, 1), (3, 5)]:
        x = g.standard_normal((2, ci, 6, 9))
        w = g.standard_normal((co, ci, 3, 3))
        b = g.standard_normal(co)
        y = oracle.conv3x3(x, w, b)
        ref = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b),
                                         padding=1).numpy()
        assert np.allclose(y, ref, rtol=0, atol=1e-11), (ci, co)


def test_conv_delta_kernel_is_identity_plus_bias():
    g = _rng(3)
    x = g.standard_normal((1, 2, 5, 8))
    w = np.zeros((2, 2, 3, 3))
    w[0, 0, 1, 1] = 1.0
    w[1, 1, 1, 1] = 1.0
    y = oracle.conv3x3(x, w, np.array([1.0, -2.0]))
    assert np.array_equal(y[0, 0], x[0, 0] + 1.0) and np.array_equal(y[0, 1], x[0, 1] - 2.0)
    # a shift tap moves the image by one pixel and fills the edge with zeros
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, 1, 2] = 1.0  # y[r][c] = x[r][c+1]
    y = oracle.conv3x3(x[:, :1], w, np.zeros(1))
    assert np.array_equal(y[0, 0, :, :-1], x[0, 0, :, 1:]) and not y[0, 0, :, -1].any()


def test_conv_backward_is_the_adjoint():
    """The convolution is linear in x and in (w, b): for any direction d,
    <conv(x + d) - conv(x), dy> = <d, dx>, and the same for w and b."""
    g = _rng(4)
    x = g.standard_normal((2, 16, 6, 7))
    w = g.standard_normal((3, 16, 3, 3))
    b = g.standard_normal(3)
    dy = g.standard_normal((2, 3, 6, 7))
    dx, dw, db = oracle.conv3x3_bwd(x, w, dy)
    dxd = g.standard_normal(x.shape)
    lhs = np.sum((oracle.conv3x3(x + dxd, w, b) - oracle.conv3x3(x, w, b)) * dy)
    assert abs(lhs - np.sum(dxd * dx)) < 1e-9 * (1 + abs(lhs))
    dwd, dbd = g.standard_normal(w.shape), g.standard_normal(b.shape)
    lhs = np.sum((oracle.conv3x3(x, w + dwd, b + dbd) - oracle.conv3x3(x, w, b)) * dy)
    assert abs(lhs - (np.sum(dwd * dw) + np.sum(dbd * db))) < 1e-9 * (1 + abs(lhs))


def test_bce_closed_forms():
    z = np.array([-3.0, -0.5, 0.0, 0.7, 4.0])
    y = np.array([0.0, 1.0, 1.0, 0.0, 1.0])
    sig = 1 / (1 + np.exp(-z))
    direct = -(y * np.log(sig) + (1 - y) * np.log(1 - sig))
    assert abs(oracle.bce_with_logits(z, y) - direct.mean()) < 1e-14
    assert abs(oracle.bce_with_logits(np.zeros(4), np.array([0, 1, 0, 1.0])) - np.log(2)) < 1e-15
    # far from zero the stable form still gives the right limits
    assert oracle.bce_with_logits(np.array([800.0]), np.array([1.0])) == 0.0
    assert abs(oracle.bce_with_logits(np.array([-800.0]), np.array([1.0])) - 800.0) < 1e-12


def _params(seed, scale=0.4):
    return _rng(seed).standard_normal(oracle.cnn_param_count()) * scale


def test_param_layout_round_trip():
    assert oracle.cnn_param_count() == 16 * 9 + 16 + 16 * 16 * 9 + 16 + 16 * 9 + 1 == 2625
    p = np.arange(2625, dtype=np.float64)
    (w1, b1), (w2, b2), (w3, b3) = oracle.cnn_unpack(p)
    assert w1.shape == (16, 1, 3, 3) and w2.shape == (16, 16, 3, 3) and w3.shape == (1, 16, 3, 3)
    flat = np.concatenate([w1.ravel(), b1, w2.ravel(), b2, w3.ravel(), b3])
    assert np.array_equal(flat, p)


def test_network_gradient_matches_central_differences():
    g = _rng(5)
    B, H, W = 2, 5, 9
    x = g.standard_normal((B, 1, H, W))
    y = (g.random((B, 1, H, W)) < 0.3).astype(np.float64)
    # parameters whose pre-activations all stay away from the ReLU kink (a step
    # of h moves none of them by more than ~1e-5), so the difference is smooth
    for seed in range(6, 100):
        p = _params(seed)
        _, (_, z1, _, z2, _) = oracle.cnn_forward(p, x)
        if min(np.abs(z1).min(), np.abs(z2).min()) > 1e-4:
            break
    assert min(np.abs(z1).min(), np.abs(z2).min()) > 1e-4
    loss, grad = oracle.cnn_loss_and_grad(p, x, y)
    h = 1e-6
    idx = np.concatenate([np.arange(0, 160, 7), np.arange(160, 2480, 53), np.arange(2480, 2625, 5), [2624]])
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (oracle.cnn_loss_and_grad(p + e, x, y)[0] - oracle.cnn_loss_and_grad(p - e, x, y)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1e-3, abs(grad[i])) + 1e-9, (i, fd, grad[i])


def test_network_gradient_of_relu_layers_is_masked():
    """With every pre-activation of the two hidden layers negative, the network
    output is the constant b3: every gradient but that of b3 vanishes, and that
    one is the mean of sigmoid(b3) - y."""
    g = _rng(7)
    x = np.abs(g.standard_normal((1, 1, 4, 6)))
    p = _params(8)
    p[:144] = -np.abs(p[:144])
    p[144:160] = -1.0
    p[2464:2480] = -1.0  # b2
    y = (g.random((1, 1, 4, 6)) < 0.5).astype(np.float64)
    loss, grad = oracle.cnn_loss_and_grad(p, x, y)
    z3, _ = oracle.cnn_forward(p, x)
    assert np.all(z3 == p[2624])
    assert not grad[:2624].any()
    z3 = p[2624]
    assert abs(grad[2624] - np.mean(1 / (1 + np.exp(-z3)) - y)) < 1e-15


def test_adam_first_steps_move_by_lr_times_sign():
    """From zero moments, Adam's bias-corrected step is lr * g / (|g| + eps)
    at t = 1, and again at t = 2 for the same gradient."""
    g = np.array([0.3, -2.0, 1e-3, -5e-5])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    lr, eps = 0.01, 1e-8
    p1, m, v = oracle.adam_step(p0, np.zeros(4), np.zeros(4), g, 1, lr, eps=eps)
    assert np.allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    p2, m, v = oracle.adam_step(p1, m, v, g, 2, lr, eps=eps)
    assert np.allclose(p2, p1 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)


def test_adam_minimises_a_quadratic():
    target = np.array([0.5, -1.5, 2.0])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        p, m, v = oracle.adam_step(p, m, v, p - target, t, 0.01)
    assert np.abs(p - target).max() < 1e-3


def test_tile_input_invariances():
    g = _rng(9)
    assert np.allclose(oracle.cnn_tile_input(np.full((64, 256), 3.5)), np.log(2.0), rtol=0, atol=1e-15)
    P = g.exponential(5.0, (64, 256))
    a = oracle.cnn_tile_input(P)
    assert np.allclose(oracle.cnn_tile_input(P * 1000.0), a, rtol=1e-13, atol=0)
    # the reference level is the median of the 256 channel means
    m = np.sort(P.mean(axis=0))
    ref = 0.5 * (m[127] + m[128])
    assert np.allclose(a, np.log1p(P / ref), rtol=1e-14, atol=0)


def test_tile_input_of_an_empty_tile_is_zero():
    assert not oracle.cnn_tile_input(np.zeros((64, 256))).any()
