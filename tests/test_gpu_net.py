"""The warm-start network on the GPU (BF16 MFMA convolutions, FP32
accumulation) against the FP64 network oracle on the same weights and inputs:
every layer's forward output, the whole network, the loss and every
parameter gradient; Adam's first step against its closed form; training
reduces the loss; the warm start falls back to v = 0 when its proposal folds
the grid. Tolerances follow BF16's 8-bit mantissa (unit round-off 2^-9 =
2e-3 per rounding): a layer's output is rounded once (plus its BF16 inputs
and weights), so <= 1e-2 per layer; the whole forward compounds twelve such
layers (<= 3e-2); weight gradients sum BF16 products of BF16-rounded
backward activations (<= 5e-2)."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import rel_l2, say
from oracle import net as onet

pytestmark = pytest.mark.gpu

N = 16  # network grid in these tests: levels 16^3, 8^3, 4^3
# 32^3 levels take the kernels' four-point-block path (grids of 32^3 and more)
SIZES = [16, 32]


@pytest.fixture(scope="module")
def reg():
    from paper_1608_03630_amd import reg as r

    r.lib()
    assert torch.cuda.is_available()
    return r


def _bf16(x):
    return torch.from_numpy(np.asarray(x, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _flat(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers]).astype(np.float32)


def _layers(flat):
    out, o = [], 0
    for cin, cout, _ in onet.LAYERS:
        W = flat[o:o + cout * cin * 27].reshape(cout, cin, 3, 3, 3).astype(np.float64)
        o += cout * cin * 27
        b = flat[o:o + cout].astype(np.float64)
        o += cout
        out.append((W, b))
    return out


def _setup(reg, seed=11, n=N):
    layers = onet.random_params(seed)
    flat = _flat(layers)
    net = reg.Net(n)
    assert net.count == flat.size
    net.reg_net_set_params(torch.from_numpy(flat).cuda())
    T = synth.smooth_random_field((n, n, n), seed + 1, kmax=4).astype(np.float32)
    R = synth.smooth_random_field((n, n, n), seed + 2, kmax=4).astype(np.float32)
    return net, _layers(flat), T, R


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()


@pytest.mark.parametrize("n", SIZES)
def test_every_layer_forward_matches_oracle(reg, n):
    net, layers, T, R = _setup(reg, 11, n)
    net.reg_net_forward(_gpu(T), _gpu(R))
    torch.cuda.synchronize()
    act = [net.reg_net_activation(l).double().cpu().numpy() for l in range(12)]
    Wb = [(_bf16(W), b) for W, b in layers]
    x = _bf16(np.stack([T, R]))
    ins = [x, act[0], act[1], act[2], act[3], act[4], act[5], onet.up2(act[6]),
           np.concatenate([act[7], act[3]]), onet.up2(act[8]), np.concatenate([act[9], act[1]]), act[10]]
    for l, (cin, cout, stride) in enumerate(onet.LAYERS):
        z = onet.conv3d(ins[l], *Wb[l], stride=stride)
        ref = z if l == 11 else onet.relu(z)
        err = rel_l2(act[l], ref)
        say(f"  layer {l} ({cin}->{cout}, stride {stride}): rel-L2 {err:.2e}")
        assert err <= 1e-2


@pytest.mark.parametrize("n", [16, 32, 64])
def test_whole_forward_matches_oracle(reg, n):
    """Up to 64^3, the grid the warm start runs the network on (the oracle's
    direct sums take about half a minute there)."""
    net, layers, T, R = _setup(reg, 21, n)
    v = net.reg_net_forward(_gpu(T), _gpu(R)).double().cpu().numpy()
    ref, _ = onet.forward(layers, np.stack([T, R]).astype(np.float64))
    err = rel_l2(v, ref)
    say(f"  {n}^3 network output rel-L2 {err:.2e}")
    assert err <= 3e-2


@pytest.mark.parametrize("n", SIZES)
def test_loss_and_parameter_gradients_match_oracle(reg, n):
    net, layers, T, R = _setup(reg, 31, n)
    target = synth.smooth_random_field((n, n, n), 34, kmax=3, ncomp=3).astype(np.float32) * 0.1
    loss, g = net.reg_net_loss_grad(_gpu(T), _gpu(R), _gpu(target))
    g = _layers(g.cpu().numpy())
    Wb = [(_bf16(W), b) for W, b in layers]
    v, acts = onet.forward(Wb, _bf16(np.stack([T, R])))
    L, dv = onet.mse(v, target.astype(np.float64))
    grads, _ = onet.backward(Wb, acts, dv)
    say(f"  loss gpu {loss:.6e} oracle {L:.6e}")
    assert abs(loss - L) <= 1e-2 * L
    for l, ((dW, db), (gW, gb)) in enumerate(zip(grads, g)):
        ew, eb = rel_l2(gW, dW), rel_l2(gb, db)
        say(f"  layer {l}: dW rel-L2 {ew:.2e}, db rel-L2 {eb:.2e}")
        assert ew <= 5e-2 and eb <= 5e-2


def test_backward_and_step_compose_the_training_step(reg):
    """reg_net_backward with dv = d(MSE)/dv after reg_net_forward gives the
    gradient of reg_net_loss_grad (the same BF16 head gradient, the same
    kernels), and reg_net_step with it moves the parameters exactly as
    reg_net_train_step on that one sample; backward without a forward is
    refused."""
    n = N
    net, layers, T, R = _setup(reg, 41, n)
    target = synth.smooth_random_field((n, n, n), 44, kmax=3, ncomp=3).astype(np.float32) * 0.1
    with pytest.raises(reg.RegError):
        net.reg_net_backward(torch.zeros(3 * n ** 3, device="cuda"))
    _, g_ref = net.reg_net_loss_grad(_gpu(T), _gpu(R), _gpu(target))
    v = net.reg_net_forward(_gpu(T), _gpu(R))
    dv = (2.0 / (3 * n ** 3)) * (v - _gpu(target))
    g = net.reg_net_backward(dv)
    torch.cuda.synchronize()
    err = rel_l2(g.double().cpu().numpy(), g_ref.double().cpu().numpy())
    say(f"  backward against loss_grad: rel-L2 {err:.1e}")
    assert err <= 1e-6
    p0 = net.reg_net_get_params().clone()
    net.reg_net_train_step([_gpu(T)], [_gpu(R)], [_gpu(target)], lr=1e-3)
    p_train = net.reg_net_get_params().clone()
    net.reg_net_set_params(p0)
    _, g1 = net.reg_net_loss_grad(_gpu(T), _gpu(R), _gpu(target))
    net.reg_net_step(g1, lr=1e-3)
    p_step = net.reg_net_get_params()
    torch.cuda.synchronize()
    assert torch.equal(p_train, p_step)
    assert not torch.equal(p_step, p0)


def test_first_adam_step_is_the_closed_form(reg):
    net, layers, T, R = _setup(reg, 41)
    target = np.zeros((3, N, N, N), np.float32)
    p0 = net.reg_net_get_params().cpu().numpy().astype(np.float64)
    _, g = net.reg_net_loss_grad(_gpu(T), _gpu(R), _gpu(target))
    g = g.cpu().numpy().astype(np.float64)
    lr = 1e-3
    net.reg_net_train_step([_gpu(T)], [_gpu(R)], [_gpu(target)], lr)
    p1 = net.reg_net_get_params().cpu().numpy().astype(np.float64)
    # step 1 with bias correction: p -= lr g / (|g| + eps)
    ref = p0 - lr * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(p1 - ref)) <= 1e-6


def test_training_reduces_the_loss(reg):
    net, layers, _, _ = _setup(reg, 51)
    Ts, Rs, Vs = [], [], []
    for i in range(4):
        T = synth.smooth_random_field((N, N, N), 60 + i, kmax=3).astype(np.float32)
        R = synth.smooth_random_field((N, N, N), 70 + i, kmax=3).astype(np.float32)
        # a target the network can express: a smooth function of the images
        V = np.stack([0.1 * (R - T), 0.05 * (R + T), 0.02 * T * R]).astype(np.float32)
        Ts.append(_gpu(T))
        Rs.append(_gpu(R))
        Vs.append(_gpu(V))
    losses = [net.reg_net_train_step(Ts, Rs, Vs, 2e-3) for _ in range(40)]
    say(f"  loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert losses[-1] < 0.5 * losses[0]


def test_warmstart_accepts_a_smooth_proposal_and_rejects_a_folding_one(reg):
    net, layers, T, R = _setup(reg, 81)
    shape = (32, 32, 32)
    ctx = reg.Context(reg.reg_default_params(shape, nt=4, prec=0))
    rT = synth.smooth_random_field(shape, 82, kmax=3).astype(np.float32)
    rR = synth.smooth_random_field(shape, 83, kmax=3).astype(np.float32)
    ctx.reg_set_images(_gpu(rT), _gpu(rR))
    # zero weights, small head bias: a constant velocity (det = 1)
    flat = np.zeros(net.count, np.float32)
    flat[-3:] = [0.05, -0.02, 0.01]
    net.reg_net_set_params(torch.from_numpy(flat).cuda())
    v, fb, dmin = net.reg_warmstart(ctx)
    torch.cuda.synchronize()
    say(f"  constant proposal: fallback {fb}, det min {dmin:.6f}")
    assert not fb and abs(dmin - 1.0) <= 1e-5
    vh = v.cpu().numpy()
    assert np.allclose(vh[0], 0.05, atol=1e-6) and np.allclose(vh[1], -0.02, atol=1e-6)
    # random weights with a head scaled by 1e3: a rough, large velocity
    # (tens of radians) that folds the grid
    big = _flat(layers[:-1] + [(layers[-1][0] * 1e3, layers[-1][1])])
    net.reg_net_set_params(torch.from_numpy(big).cuda())
    v, fb, dmin = net.reg_warmstart(ctx)
    torch.cuda.synchronize()
    say(f"  large proposal: fallback {fb}, det min {dmin:.3e}")
    assert fb and not dmin > 0
    assert torch.count_nonzero(v).item() == 0
