"""FP64 reference of the learned warm-start network.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the product package
never does, and this module imports nothing from it.

The network is not part of the paper (its Gauss-Newton-Krylov solver starts
from v = 0 or from the previous continuation level). It maps the template and
reference images, sampled on a 64^3 grid, to an initial velocity on the same
grid; the solver then refines that velocity. Plain numpy, float64, written
from the definitions:

* conv3d with 3x3x3 kernels and circular padding (the images are periodic,
  section III-B1 of the paper), cross-correlation convention
      y[o, p] = b[o] + sum_c sum_t W[o, c, t] x[c, (s*p + t - 1) mod n]
  per axis, t in {0, 1, 2}, stride s in {1, 2};
* ReLU, nearest-neighbour upsampling by 2, channel concatenation;
* the hand-written backward of each, the mean-squared-error loss and Adam.

Architecture (3 levels, 16/32/64 channels, skip concatenation):
    e1a = relu(conv(x, 2->16))            64^3
    e1  = relu(conv(e1a, 16->16))         64^3
    d2  = relu(conv_s2(e1, 16->32))       32^3
    e2  = relu(conv(d2, 32->32))          32^3
    d3  = relu(conv_s2(e2, 32->64))       16^3
    b1  = relu(conv(d3, 64->64))          16^3
    b2  = relu(conv(b1, 64->64))          16^3
    u2  = relu(conv(up2(b2), 64->32))     32^3
    m2  = relu(conv([u2, e2], 64->32))    32^3
    u1  = relu(conv(up2(m2), 32->16))     64^3
    m1  = relu(conv([u1, e1], 32->16))    64^3
    v   = conv(m1, 16->3)                 64^3
Parameters are the list of (W [cout, cin, 3, 3, 3], b [cout]) in that order.
"""
import numpy as np

# (cin, cout, stride) of the twelve convolutions, in order
LAYERS = [(2, 16, 1), (16, 16, 1), (16, 32, 2), (32, 32, 1), (32, 64, 2), (64, 64, 1), (64, 64, 1),
          (64, 32, 1), (64, 32, 1), (32, 16, 1), (32, 16, 1), (16, 3, 1)]


def _taps():
    for a in range(3):
        for b in range(3):
            for c in range(3):
                yield a, b, c


def _shifted(x, t, stride):
    """x[c, (stride*p + t - 1) mod n] on the output grid p."""
    s = np.roll(x, shift=(1 - t[0], 1 - t[1], 1 - t[2]), axis=(1, 2, 3))
    return s[:, ::stride, ::stride, ::stride]


def conv3d(x, W, b, stride=1):
    """Circular 3x3x3 convolution (cross-correlation) with bias."""
    cout = W.shape[0]
    m = [n // stride for n in x.shape[1:]]
    y = np.zeros((cout, *m))
    for t in _taps():
        y += np.einsum("oc,cijk->oijk", W[:, :, t[0], t[1], t[2]], _shifted(x, t, stride))
    return y + b[:, None, None, None]


def conv3d_backward(x, W, dy, stride=1):
    """Gradients of sum(dy * conv3d(x, W, b)) with respect to x, W and b."""
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t in _taps():
        dW[:, :, t[0], t[1], t[2]] = np.einsum("oijk,cijk->oc", dy, _shifted(x, t, stride))
        # scatter W^T dy back to the input points stride*p + t - 1
        z = np.zeros_like(x)
        z[:, ::stride, ::stride, ::stride] = np.einsum("oc,oijk->cijk", W[:, :, t[0], t[1], t[2]], dy)
        dx += np.roll(z, shift=(t[0] - 1, t[1] - 1, t[2] - 1), axis=(1, 2, 3))
    db = dy.sum(axis=(1, 2, 3))
    return dx, dW, db


def relu(z):
    return np.maximum(z, 0.0)


def relu_backward(y, dy):
    """Gradient through y = relu(z), from the output y."""
    return dy * (y > 0)


def up2(x):
    """Nearest-neighbour upsampling by 2 per axis: u[c, i] = x[c, i // 2]."""
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def up2_backward(du):
    """Adjoint of up2: each coarse point collects its 8 children."""
    c, n1, n2, n3 = du.shape
    return du.reshape(c, n1 // 2, 2, n2 // 2, 2, n3 // 2, 2).sum(axis=(2, 4, 6))


def forward(params, x):
    """v = net(x) for x [2, n, n, n] (n divisible by 4); returns v and the
    activations the backward pass needs."""
    P = params
    a = {"x": x}
    a["e1a"] = relu(conv3d(x, *P[0]))
    a["e1"] = relu(conv3d(a["e1a"], *P[1]))
    a["d2"] = relu(conv3d(a["e1"], *P[2], stride=2))
    a["e2"] = relu(conv3d(a["d2"], *P[3]))
    a["d3"] = relu(conv3d(a["e2"], *P[4], stride=2))
    a["b1"] = relu(conv3d(a["d3"], *P[5]))
    a["b2"] = relu(conv3d(a["b1"], *P[6]))
    a["up_b2"] = up2(a["b2"])
    a["u2"] = relu(conv3d(a["up_b2"], *P[7]))
    a["cat2"] = np.concatenate([a["u2"], a["e2"]])
    a["m2"] = relu(conv3d(a["cat2"], *P[8]))
    a["up_m2"] = up2(a["m2"])
    a["u1"] = relu(conv3d(a["up_m2"], *P[9]))
    a["cat1"] = np.concatenate([a["u1"], a["e1"]])
    a["m1"] = relu(conv3d(a["cat1"], *P[10]))
    v = conv3d(a["m1"], *P[11])
    return v, a


def backward(params, a, dv):
    """Gradients (dW, db) of every layer and dx, for the loss gradient dv."""
    P = params
    g = [None] * len(P)

    def layer(i, inp, dz, stride=1):
        dx, dW, db = conv3d_backward(inp, P[i][0], dz, stride)
        g[i] = (dW, db)
        return dx

    d = layer(11, a["m1"], dv)
    d = layer(10, a["cat1"], relu_backward(a["m1"], d))
    du1, de1_skip = d[:16], d[16:]
    d = layer(9, a["up_m2"], relu_backward(a["u1"], du1))
    d = up2_backward(d)
    d = layer(8, a["cat2"], relu_backward(a["m2"], d))
    du2, de2_skip = d[:32], d[32:]
    d = layer(7, a["up_b2"], relu_backward(a["u2"], du2))
    d = up2_backward(d)
    d = layer(6, a["b1"], relu_backward(a["b2"], d))
    d = layer(5, a["d3"], relu_backward(a["b1"], d))
    d = layer(4, a["e2"], relu_backward(a["d3"], d), stride=2)
    d = layer(3, a["d2"], relu_backward(a["e2"], d + de2_skip))
    d = layer(2, a["e1"], relu_backward(a["d2"], d), stride=2)
    d = layer(1, a["e1a"], relu_backward(a["e1"], d + de1_skip))
    dx = layer(0, a["x"], relu_backward(a["e1a"], d))
    return g, dx


def mse(v, target):
    """Mean squared error over all elements and its gradient."""
    r = v - target
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam_step(params, grads, m, s, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments) of every array, in place.
    step counts from 1; m and s are lists of first and second moments shaped
    like params."""
    for (W, b), (dW, db), mm, ss in zip(params, grads, m, s):
        for p, gr, mi, si in ((W, dW, mm[0], ss[0]), (b, db, mm[1], ss[1])):
            mi *= beta1
            mi += (1 - beta1) * gr
            si *= beta2
            si += (1 - beta2) * gr * gr
            mhat = mi / (1 - beta1 ** step)
            shat = si / (1 - beta2 ** step)
            p -= lr * mhat / (np.sqrt(shat) + eps)


def zeros_like_params(params):
    return [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]


def random_params(seed, scale=1.0):
    """Seeded He-normal weights and small biases (for tests)."""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout, _ in LAYERS:
        W = rng.standard_normal((cout, cin, 3, 3, 3)) * scale * np.sqrt(2.0 / (27 * cin))
        b = 0.01 * rng.standard_normal(cout)
        out.append((W, b))
    return out
