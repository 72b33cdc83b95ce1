"""Pins of the FP64 network oracle (oracle/net.py) to things other than
itself: a brute-force direct sum, closed forms of special kernels, central
finite differences, adjoint identities and Adam's closed-form first steps."""
import itertools

import numpy as np
import pytest

from oracle import net


def _brute_conv(x, W, b, stride):
    cin, n = x.shape[0], x.shape[1]
    cout = W.shape[0]
    m = n // stride
    y = np.zeros((cout, m, m, m))
    for o, i, j, k in itertools.product(range(cout), range(m), range(m), range(m)):
        acc = b[o]
        for c, a1, a2, a3 in itertools.product(range(cin), range(3), range(3), range(3)):
            acc += W[o, c, a1, a2, a3] * x[c, (stride * i + a1 - 1) % n, (stride * j + a2 - 1) % n,
                                           (stride * k + a3 - 1) % n]
        y[o, i, j, k] = acc
    return y


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_equals_brute_force_direct_sum(stride):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 4, 4))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    np.testing.assert_allclose(net.conv3d(x, W, b, stride), _brute_conv(x, W, b, stride), rtol=0, atol=1e-13)


def test_single_tap_kernels_are_periodic_shifts():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 6, 6, 6))
    for t in [(1, 1, 1), (0, 1, 2), (2, 2, 0)]:
        W = np.zeros((1, 1, 3, 3, 3))
        W[0, 0][t] = 1.0
        y = net.conv3d(x, W, np.zeros(1))
        # y[i] = x[i + t - 1]
        ref = np.roll(x, shift=tuple(1 - a for a in t), axis=(1, 2, 3))
        assert np.array_equal(y, ref)
    # stride 2 with the centre tap samples the even points
    W = np.zeros((1, 1, 3, 3, 3))
    W[0, 0, 1, 1, 1] = 1.0
    assert np.array_equal(net.conv3d(x, W, np.zeros(1), 2), x[:, ::2, ::2, ::2])


def _fd(f, arr, idx, eps=1e-6):
    old = arr[idx]
    arr[idx] = old + eps
    fp = f()
    arr[idx] = old - eps
    fm = f()
    arr[idx] = old
    return (fp - fm) / (2 * eps)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_backward_matches_finite_differences(stride):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 4, 4, 4))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    m = 4 // stride
    r = rng.standard_normal((3, m, m, m))

    def loss():
        return float(np.sum(r * net.conv3d(x, W, b, stride)))

    dx, dW, db = net.conv3d_backward(x, W, r, stride)
    for idx in [(0, 0, 0, 0), (1, 3, 2, 1), (0, 2, 3, 3)]:
        assert abs(_fd(loss, x, idx) - dx[idx]) <= 1e-7 * max(1.0, abs(dx[idx]))
    for idx in [(0, 0, 0, 0, 0), (2, 1, 1, 2, 0), (1, 1, 2, 2, 2)]:
        assert abs(_fd(loss, W, idx) - dW[idx]) <= 1e-7 * max(1.0, abs(dW[idx]))
    for o in range(3):
        assert abs(_fd(loss, b, (o,)) - db[o]) <= 1e-7 * max(1.0, abs(db[o]))


def test_up2_backward_is_the_adjoint():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, 4, 4, 4))
    y = rng.standard_normal((3, 8, 8, 8))
    assert abs(np.sum(net.up2(x) * y) - np.sum(x * net.up2_backward(y))) <= 1e-12 * np.sum(np.abs(x)) * 8
    assert net.up2(x)[1, 5, 2, 7] == x[1, 2, 1, 3]


def test_network_backward_matches_finite_differences():
    """Whole network (8^3 input: levels 8, 4, 2) against central FD of the
    MSE loss, for entries of every layer's weights and biases and the input."""
    rng = np.random.default_rng(5)
    params = [(W.copy(), b.copy()) for W, b in net.random_params(6)]
    x = rng.standard_normal((2, 8, 8, 8))
    target = rng.standard_normal((3, 8, 8, 8))

    def loss():
        v, _ = net.forward(params, x)
        return net.mse(v, target)[0]

    v, acts = net.forward(params, x)
    L, dv = net.mse(v, target)
    grads, dx = net.backward(params, acts, dv)
    worst = 0.0
    for i, ((W, b), (dW, db)) in enumerate(zip(params, grads)):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in W.shape)
            fd = _fd(loss, W, idx)
            worst = max(worst, abs(fd - dW[idx]) / max(1e-6, abs(dW[idx]) + abs(fd)))
        o = (int(rng.integers(0, b.shape[0])),)
        fd = _fd(loss, b, o)
        worst = max(worst, abs(fd - db[o]) / max(1e-6, abs(db[o]) + abs(fd)))
    for _ in range(4):
        idx = tuple(int(rng.integers(0, s)) for s in x.shape)
        fd = _fd(loss, x, idx)
        worst = max(worst, abs(fd - dx[idx]) / max(1e-6, abs(dx[idx]) + abs(fd)))
    assert worst <= 1e-6, worst


def test_mse_gradient():
    rng = np.random.default_rng(7)
    v = rng.standard_normal((3, 4, 4, 4))
    t = rng.standard_normal((3, 4, 4, 4))
    L, dv = net.mse(v, t)
    assert abs(L - np.sum((v - t) ** 2) / v.size) <= 1e-15
    idx = (2, 1, 0, 3)
    assert abs(_fd(lambda: net.mse(v, t)[0], v, idx) - dv[idx]) <= 1e-9


def test_adam_first_two_steps_closed_form():
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    W = np.array([[[[[0.5]]]]]) * np.ones((1, 1, 3, 3, 3))
    b = np.array([0.25])
    params = [(W, b)]
    g1 = [(np.full_like(W, 2.0), np.array([-3.0]))]
    m, s = net.zeros_like_params(params), net.zeros_like_params(params)
    net.adam_step(params, g1, m, s, 1, lr, b1, b2, eps)
    # step 1: m_hat = g, s_hat = g^2, so the move is -lr g / (|g| + eps)
    assert np.allclose(W, 0.5 - lr * 2.0 / (2.0 + eps), rtol=0, atol=1e-15)
    assert abs(b[0] - (0.25 + lr * 3.0 / (3.0 + eps))) <= 1e-15
    g2 = [(np.full_like(W, -1.0), np.array([1.0]))]
    w_before = W.copy()
    net.adam_step(params, g2, m, s, 2, lr, b1, b2, eps)
    m2 = b1 * (1 - b1) * 2.0 + (1 - b1) * -1.0
    s2 = b2 * (1 - b2) * 4.0 + (1 - b2) * 1.0
    step = lr * (m2 / (1 - b1 ** 2)) / (np.sqrt(s2 / (1 - b2 ** 2)) + eps)
    assert np.allclose(W, w_before - step, rtol=0, atol=1e-15)
