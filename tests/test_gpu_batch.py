"""Batches of independent problems of mixed sizes (reg_batch_*): every
problem's results through the batched persistent launches, the autotuned
launch shapes and the captured matvec graphs equal, bit for bit, those of the
single-problem entry points on a context of its own (same kernels, same
arguments), and the batched transport matches the FP64 oracle like the single
one. The mix holds grids in whole 4x8x64 tiles (canonical LDS boxes), a
ragged grid (generic box, in a batched launch of its own), different nt, both the
compressible and the isochoric case, small and multi-cell steps (canonical and
generic boxes side by side) and both precisions."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import TOL, rel_l2, say, to_dev, to_host, to_vel

pytestmark = pytest.mark.gpu

# shape, nt, isochoric
PROBLEMS = [
    ((64, 64, 64), 4, 0),
    ((32, 48, 64), 3, 1),
    ((24, 36, 54), 4, 0),
    ((16, 16, 128), 2, 0),
]
BETA = 1e-2


@pytest.fixture(scope="module")
def reg():
    from paper_1608_03630_amd import reg as r

    r.lib()
    assert torch.cuda.is_available()
    return r


def _params(reg, shape, nt, iso, **kw):
    kw.setdefault("prec", 0)
    return reg.reg_default_params(shape, nt=nt, beta=BETA, isochoric=iso, **kw)


@pytest.fixture(scope="module")
def cases():
    """Seeded blob images; rho_R from the FP64 oracle's transport."""
    out = []
    for i, (shape, nt, iso) in enumerate(PROBLEMS):
        case = synth.blob_case(shape, seed=2000 + i)
        rhoT = case["rhoT"].astype(np.float32).astype(np.float64)
        P = oracle.params(shape, nt, BETA, isochoric=bool(iso))
        rhoR = oracle.transport_forward(P, case["v_true"], rhoT).astype(np.float32).astype(np.float64)
        out.append({"rhoT": rhoT, "rhoR": rhoR, "v": 0.3 * case["v_true"], "P": P})
    return out


def _batch(reg, cases, **kw):
    say(f"  [batch] {PROBLEMS} {kw}")
    b = reg.Batch([_params(reg, s, nt, iso, **kw) for s, nt, iso in PROBLEMS])
    for i, c in enumerate(cases):
        ctx = b.contexts[i]
        b.reg_set_images(i, to_dev(c["rhoT"], ctx), to_dev(c["rhoR"], ctx))
    return b


def _singles(reg, cases, **kw):
    out = []
    for (s, nt, iso), c in zip(PROBLEMS, cases):
        ctx = reg.Context(_params(reg, s, nt, iso, **kw))
        ctx.reg_set_images(to_dev(c["rhoT"], ctx), to_dev(c["rhoR"], ctx))
        out.append(ctx)
    return out


# velocity scales: small steps (canonical boxes), and steps of several cells
# per step on the larger grids (generic boxes beside canonical ones)
@pytest.mark.parametrize("prec,scale", [(0, 0.3), (0, 4.0), (1, 0.3)])
def test_batch_transport_matches_single_and_oracle(reg, cases, prec, scale):
    b = _batch(reg, cases, prec=prec)
    vs = [to_vel(scale * c["v"], ctx) for c, ctx in zip(cases, b.contexts)]
    r0 = [to_dev(c["rhoT"], ctx) for c, ctx in zip(cases, b.contexts)]
    rb = b.reg_batch_transport_forward(vs, r0)
    torch.cuda.synchronize()
    st = b.reg_batch_stats()
    say(f"  stats {st}, interp launch (blocks, chunked, variant, tile, ms) {b.reg_batch_launch_info(0)}")
    # single precision always goes through the batched persistent launch;
    # double precision does where its boxes fit the LDS
    if prec == 0:
        assert st["batched_launches"] > 0
    singles = _singles(reg, cases, prec=prec)
    for i, (ctx, c) in enumerate(zip(singles, cases)):
        rs = ctx.reg_transport_forward(to_vel(scale * c["v"], ctx), to_dev(c["rhoT"], ctx))
        torch.cuda.synchronize()
        assert torch.equal(rb[i], rs), f"problem {i}"
        ref = oracle.transport_forward(c["P"], scale * c["v"], c["rhoT"])
        err = rel_l2(to_host(rb[i]), ref)
        say(f"  problem {i} {PROBLEMS[i]}: rel-L2 vs oracle {err:.2e}")
        assert err <= TOL[("transport", prec)]


@pytest.mark.parametrize("blocks,chunked", [(8, 0), (8, 1), (72, 1), (4096, 0)])
def test_batch_launch_shape_does_not_change_results(reg, cases, blocks, chunked):
    b = _batch(reg, cases)
    vs = [to_vel(c["v"], ctx) for c, ctx in zip(cases, b.contexts)]
    r0 = [to_dev(c["rhoT"], ctx) for c, ctx in zip(cases, b.contexts)]
    auto = b.reg_batch_transport_forward(vs, r0)
    b.reg_batch_set_launch(blocks, chunked)
    fixed = b.reg_batch_transport_forward(vs, r0)
    torch.cuda.synchronize()
    info = b.reg_batch_launch_info(0)
    say(f"  fixed launch (blocks, chunked, variant, tile, ms) {info}")
    assert info[0] == blocks and info[1] == chunked
    for i in range(len(PROBLEMS)):
        assert torch.equal(auto[i], fixed[i]), f"problem {i}"


@pytest.mark.parametrize("tile", [(2, 8), (8, 8), (4, 4), (8, 4), (4, 8)])
def test_batch_tile_shape_does_not_change_results(reg, cases, tile):
    """Every tile shape of the batched canonical kernels computes each point
    with the same arithmetic from the same box values: results equal the
    autotuned launch bit for bit, for the three step kinds (the problems in
    whole tiles of every shape, so that each launch is canonical and reports
    the shape it ran)."""
    idx = [i for i, (s, _, _) in enumerate(PROBLEMS) if s[0] % 8 == 0 and s[1] % 8 == 0 and s[2] % 64 == 0]
    b = reg.Batch([_params(reg, *PROBLEMS[i]) for i in idx])
    cs = [cases[i] for i in idx]
    for j, c in enumerate(cs):
        b.reg_set_images(j, to_dev(c["rhoT"], b.contexts[j]), to_dev(c["rhoR"], b.contexts[j]))
    vs = [to_vel(c["v"], ctx) for c, ctx in zip(cs, b.contexts)]
    r0 = [to_dev(c["rhoT"], ctx) for c, ctx in zip(cs, b.contexts)]
    auto = b.reg_batch_transport_forward(vs, r0)
    gauto = [g.clone() for g in b.reg_batch_gradient(vs)[0]]
    b.reg_batch_set_tile(*tile)
    fixed = b.reg_batch_transport_forward(vs, r0)
    info = b.reg_batch_launch_info(0)
    gfix = b.reg_batch_gradient(vs)[0]
    torch.cuda.synchronize()
    say(f"  tile {tile}: interp launch (blocks, chunked, variant, tile, ms) {info}")
    assert info[2] != 0 and info[3] == tile
    for i in range(len(idx)):
        assert torch.equal(auto[i], fixed[i]), f"transport of problem {idx[i]}"
        assert torch.equal(gauto[i], gfix[i]), f"gradient of problem {idx[i]}"


def test_batch_gradient_and_graph_matvec_match_single(reg, cases):
    b = _batch(reg, cases)
    singles = _singles(reg, cases)
    vs = [to_vel(c["v"], ctx) for c, ctx in zip(cases, b.contexts)]
    gb, Jb, mb, nb = b.reg_batch_gradient(vs)
    ref = []
    for i, (ctx, c) in enumerate(zip(singles, cases)):
        g, J, mis, gn = ctx.reg_gradient(to_vel(c["v"], ctx))
        torch.cuda.synchronize()
        assert torch.equal(gb[i], g), f"gradient of problem {i}"
        assert (Jb[i], mb[i], nb[i]) == (J, mis, gn), f"scalars of problem {i}"
        vt = to_vel(synth.smooth_random_field(ctx.shape, 300 + i, kmax=3, ncomp=3), ctx)
        H = ctx.reg_hessian_matvec(vt)
        torch.cuda.synchronize()
        ref.append((vt, H.clone()))
    vts = [vt for vt, _ in ref]
    outs = [torch.empty_like(vt) for vt in vts]
    # 1st call eager, 2nd captured, then replays; eager work in between
    for call in range(5):
        for o in outs:
            o.fill_(float("nan"))
        b.reg_batch_hessian_matvec(vts, outs)
        torch.cuda.synchronize()
        st = b.reg_batch_stats()
        say(f"  matvec call {call}: {st}")
        for i, (o, (_, H)) in enumerate(zip(outs, ref)):
            assert torch.equal(o, H), f"matvec call {call}, problem {i}"
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()
        singles[0].reg_hessian_matvec(vts[0])
        torch.cuda.synchronize()
    st = b.reg_batch_stats()
    assert st["graph_captures"] == 1 and st["graph_replays"] == 3
    # the same without graphs
    b.reg_batch_set_launch(0, 1, use_graph=False)
    eager = b.reg_batch_hessian_matvec(vts)
    torch.cuda.synchronize()
    for i, (_, H) in enumerate(ref):
        assert torch.equal(eager[i], H), f"eager matvec, problem {i}"


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_solve_matches_single(reg, cases, prec):
    kw = dict(max_newton=3, max_pcg=8, gtol=1e-3, prec=prec)
    b = _batch(reg, cases, **kw)
    vb, reps = b.reg_batch_solve()
    torch.cuda.synchronize()
    st = b.reg_batch_stats()
    say(f"  batch solve: {st}; " + ", ".join(f"{r['n_iter']} it/{r['matvecs']} mv" for r in reps))
    assert st["graph_replays"] > 0
    singles = _singles(reg, cases, **kw)
    for i, ctx in enumerate(singles):
        v, rep = ctx.reg_solve()
        torch.cuda.synchronize()
        assert torch.equal(vb[i], v), f"velocity of problem {i}"
        for k in ("status", "n_iter", "matvecs", "gradients", "objectives", "stop_reason", "final_J",
                  "final_mismatch", "J", "mismatch", "pcg_iters", "ls_trials", "interps"):
            assert reps[i][k] == rep[k], f"{k} of problem {i}"
        assert rep["final_mismatch"] < 1.0


def test_failing_problem_leaves_the_others_untouched(reg, cases):
    """A NaN in one problem's reference image: that problem stops with
    REG_ENONFINITE at its first gradient (v left at its initial value), the
    batch returns that status, and every other problem still solves exactly
    as it does alone."""
    kw = dict(max_newton=3, max_pcg=8, gtol=1e-3)
    bad = 1
    b = reg.Batch([_params(reg, s, nt, iso, **kw) for s, nt, iso in PROBLEMS])
    for i, c in enumerate(cases):
        ctx = b.contexts[i]
        rhoR = c["rhoR"].copy()
        if i == bad:
            rhoR[3, 5, 7] = np.nan
        b.reg_set_images(i, to_dev(c["rhoT"], ctx), to_dev(rhoR, ctx))
    with pytest.raises(reg.RegError) as e:
        b.reg_batch_solve()
    assert e.value.status == reg.REG_ENONFINITE
    vb, reps = b.reg_batch_solve(raise_on_error=False)
    torch.cuda.synchronize()
    say("  " + ", ".join(f"status {r['status']} {r['n_iter']} it" for r in reps))
    assert reps[bad]["status"] == reg.REG_ENONFINITE and reps[bad]["n_iter"] == 0
    assert torch.count_nonzero(vb[bad]).item() == 0
    singles = _singles(reg, cases, **kw)
    for i, ctx in enumerate(singles):
        if i == bad:
            continue
        v, rep = ctx.reg_solve()
        torch.cuda.synchronize()
        assert reps[i]["status"] == 0 and torch.equal(vb[i], v), f"problem {i}"
        assert reps[i]["pcg_iters"] == rep["pcg_iters"] and reps[i]["final_J"] == rep["final_J"]
