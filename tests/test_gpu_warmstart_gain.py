"""What the trained warm-start network gains over the method without it.

The committed parameters (paper_1608_03630_amd/weights/warmstart_n64.npy,
trained on pairs the method itself registered; profiles/warmstart_blob256.md)
propose the initial velocity of held-out pairs of the training recipe. Cold
(v = 0) and warm starts run to the same stopping rule (||g|| <= gtol
||g(v = 0)||, forcing relative to the same reference): the warm start must
reach the same final mismatch with fewer Hessian matvecs in total, and its
proposals must pass the det(grad y1) > 0 check."""
import os

import numpy as np
import pytest
import torch

from gpu_util import say

pytestmark = pytest.mark.gpu

SEEDS = [53000, 53001, 53002, 53003]  # held out: training used 50000-51999
N = 128


@pytest.fixture(scope="module")
def ws():
    from paper_1608_03630_amd import reg, warmstart

    reg.lib()
    assert torch.cuda.is_available()
    assert os.path.exists(warmstart.WEIGHTS)
    return reg, warmstart


def test_trained_network_saves_matvecs_at_equal_accuracy(ws):
    reg, warmstart = ws
    net = reg.Net(warmstart.NET_N)
    net.reg_net_set_params(torch.from_numpy(np.load(warmstart.WEIGHTS)).cuda())
    cold_mv = warm_mv = 0
    for s in SEEDS:
        rhoT, v_true = warmstart.make_pair(N, s)
        ctx = reg.Context(warmstart.pair_params(N))
        rhoR = ctx.reg_transport_forward(v_true, rhoT)
        ctx.reg_set_images(rhoT, rhoR)
        zero = torch.zeros((3,) + ctx.shape, dtype=torch.float64, device="cuda")
        _, _, _, g0 = ctx.reg_gradient(zero)
        ctx.reg_set_solver(warmstart.pair_params(N, gnorm_ref=g0))
        _, rc = ctx.reg_solve(zero.clone())
        vw, fb, dmin = net.reg_warmstart(ctx)
        _, mis0 = ctx.reg_objective(vw)
        _, rw = ctx.reg_solve(vw)
        torch.cuda.synchronize()
        say(f"  pair {s}: cold {rc['n_iter']} GN / {rc['matvecs']} mv / mis {rc['final_mismatch']:.4f}; warm "
            f"{rw['n_iter']} GN / {rw['matvecs']} mv / mis {rw['final_mismatch']:.4f} (proposal mismatch "
            f"{mis0:.3f}, det min {dmin:.3f})")
        assert not fb and dmin > 0
        assert mis0 < 0.8  # the proposal already removes a large part of the mismatch
        assert rw["stop_reason"] == rc["stop_reason"] == 0
        assert abs(rw["final_mismatch"] - rc["final_mismatch"]) <= 0.01 * rc["final_mismatch"]
        cold_mv += rc["matvecs"]
        warm_mv += rw["matvecs"]
    say(f"  total matvecs: cold {cold_mv}, warm {warm_mv}")
    assert warm_mv <= 0.9 * cold_mv
