"""Training set, training and evaluation of the learned warm start.

The network (reg_net, BF16 MFMA convolutions) learns to map the template and
reference images, spectrally truncated to 64^3, to the velocity the
Gauss-Newton-Krylov solver finds for the pair, truncated likewise. Its
training pairs are registered by the method itself (reg_batch_solve); at use
the proposal is resampled to the problem's grid and checked by
reg_warmstart, and the solver then runs to the same stopping rule as a cold
start (an absolute gradient tolerance gtol * ||g(v = 0)||).

Pairs are blob images with a divergence-free |k| <= 4 velocity of max speed
0.5 (seeded; the reference is the template transported on the GPU), solved
with nt = 8, beta = 1e-3, isochoric, FP32 fields.

    python -m paper_1608_03630_amd.warmstart --train 2000 --val 100 --test 20 \\
        --epochs 20 --weights W.npy --report R.json

Everything runs on the GPU through the library; the host only shuffles,
schedules the learning rate and writes the results.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

from . import reg  # noqa: E402

NET_N = 64
TRAIN_SEED0, VAL_SEED0, TEST_SEED0 = 50000, 52000, 53000
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart_n64.npy")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pair_params(n, **kw):
    p = dict(nt=8, prec=0, beta=1e-3, isochoric=1, gtol=1e-2, max_newton=50, max_pcg=100, max_ls=20)
    p.update(kw)
    return reg.reg_default_params((n, n, n), **p)


def init_params(seed):
    """He-normal convolution weights (seeded), zero biases; the head starts
    small so that the first proposals are near zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, (cin, cout, _) in enumerate(reg.NET_LAYERS):
        W = rng.standard_normal((cout, cin, 3, 3, 3)) * math.sqrt(2.0 / (27 * cin))
        if i == len(reg.NET_LAYERS) - 1:
            W *= 0.1
        parts += [W.ravel(), np.zeros(cout)]
    return np.concatenate(parts).astype(np.float32)


def make_pair(n, seed):
    rhoT, v = synth.blob_case_device((n, n, n), seed, "cuda")
    return rhoT.float().contiguous(), v.contiguous()


def register_pairs(seeds, n, group, dst):
    """Registers the pairs with the batched solver; returns the truncations
    to the network grid (images and solved velocity, float32 on the GPU)."""
    out = []
    for g0 in range(0, len(seeds), group):
        chunk = seeds[g0:g0 + group]
        t0 = time.time()
        b = reg.Batch([pair_params(n) for _ in chunk])
        cases = [make_pair(n, s) for s in chunk]
        rhoR = b.reg_batch_transport_forward([v for _, v in cases], [r for r, _ in cases])
        for i, (rhoT, _) in enumerate(cases):
            b.reg_set_images(i, rhoT, rhoR[i])
        vs, reps = b.reg_batch_solve()
        for i, c in enumerate(b.contexts):
            rT = c.reg_resample(dst, cases[i][0])
            rR = c.reg_resample(dst, rhoR[i])
            v = c.reg_resample(dst, vs[i].float().contiguous())
            out.append((rT, rR, v))
        torch.cuda.synchronize()
        its = [r["n_iter"] for r in reps]
        mis = [r["final_mismatch"] for r in reps]
        log(f"[warmstart] registered pairs {chunk[0]}..{chunk[-1]} at {n}^3 in {time.time() - t0:.1f} s "
            f"(GN steps {np.mean(its):.1f}, mismatch {np.mean(mis):.3f})")
        b.close()
        del b, cases, rhoR, vs
        torch.cuda.empty_cache()
    return out


def mean_loss(net, data):
    return float(np.mean([net.reg_net_loss_grad(*d)[0] for d in data]))


def train(net, data, val, epochs, batch, lr, seed):
    rng = np.random.default_rng(seed)
    steps = epochs * max(1, len(data) // batch)
    hist = []
    k = 0
    for ep in range(epochs):
        t0 = time.time()
        order = rng.permutation(len(data))
        losses = []
        for s in range(0, len(order) - batch + 1, batch):
            idx = order[s:s + batch]
            lr_k = lr * (0.1 + 0.9 * 0.5 * (1 + math.cos(math.pi * k / steps)))
            losses.append(net.reg_net_train_step([data[i][0] for i in idx], [data[i][1] for i in idx],
                                                 [data[i][2] for i in idx], lr_k))
            k += 1
        vl = mean_loss(net, val) if val else None
        hist.append({"epoch": ep, "train_loss": float(np.mean(losses)), "val_loss": vl, "seconds": time.time() - t0})
        log(f"[warmstart] epoch {ep}: train {hist[-1]['train_loss']:.4e}, val {vl:.4e}, {hist[-1]['seconds']:.1f} s")
    return hist


def evaluate(net, seeds, n):
    """Cold (v = 0) against warm start on held-out pairs, both stopped at
    ||g|| <= gtol ||g(v = 0)||."""
    rows = []
    for s in seeds:
        rhoT, v_true = make_pair(n, s)
        p = pair_params(n)
        ctx = reg.Context(p)
        rhoR = ctx.reg_transport_forward(v_true, rhoT)
        ctx.reg_set_images(rhoT, rhoR)
        zero = torch.zeros((3,) + ctx.shape, dtype=torch.float64, device="cuda")
        _, _, _, g0 = ctx.reg_gradient(zero)
        ctx.reg_set_solver(pair_params(n, gnorm_ref=g0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v = zero.clone()
        _, rc = ctx.reg_solve(v)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        t0 = time.perf_counter()
        vw, fb, dmin = net.reg_warmstart(ctx)
        t_ws = time.perf_counter() - t0
        _, mis0 = ctx.reg_objective(vw)  # the proposal's mismatch (not timed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rw = ctx.reg_solve(vw)
        torch.cuda.synchronize()
        tw = t_ws + time.perf_counter() - t0
        row = {"seed": s, "cold": {"gn_steps": rc["n_iter"], "matvecs": rc["matvecs"], "seconds": tc,
                                   "mismatch": rc["final_mismatch"], "grel": rc["final_grel"]},
               "warm": {"gn_steps": rw["n_iter"], "matvecs": rw["matvecs"], "seconds": tw,
                        "warmstart_seconds": t_ws, "mismatch": rw["final_mismatch"], "fallback": fb,
                        "detmin": dmin, "initial_mismatch": mis0}}
        rows.append(row)
        log(f"[warmstart] test pair {s}: cold {rc['n_iter']} GN / {rc['matvecs']} mv / {tc:.2f} s / mis "
            f"{rc['final_mismatch']:.4f};  warm {rw['n_iter']} GN / {rw['matvecs']} mv / {tw:.2f} s / mis "
            f"{rw['final_mismatch']:.4f} (fallback {fb}, proposal mismatch {mis0:.3f})")
        ctx.close()
        del ctx, rhoT, rhoR, v_true
        torch.cuda.empty_cache()
    return rows


def summarize(rows):
    out = {}
    for k in ("cold", "warm"):
        out[k] = {m: float(np.mean([r[k][m] for r in rows])) for m in ("gn_steps", "matvecs", "seconds", "mismatch")}
    out["fallbacks"] = int(sum(r["warm"]["fallback"] for r in rows))
    out["speedup_seconds"] = out["cold"]["seconds"] / out["warm"]["seconds"]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train", type=int, default=2000, help="training pairs")
    ap.add_argument("--val", type=int, default=100, help="validation pairs")
    ap.add_argument("--test", type=int, default=20, help="held-out test pairs")
    ap.add_argument("--pair-n", type=int, default=128, help="registration grid of the training pairs")
    ap.add_argument("--test-n", type=int, default=256, help="grid of the test pairs")
    ap.add_argument("--group", type=int, default=64, help="pairs registered per batch")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--weights", type=str, default=WEIGHTS, help="where to write the trained parameters")
    ap.add_argument("--report", type=str, default=None, help="JSON report")
    ap.add_argument("--eval-only", action="store_true", help="load --weights and run only the test pairs")
    args = ap.parse_args(argv)

    reg.lib()
    torch.cuda.set_device(0)
    net = reg.Net(NET_N)
    report = {"config": vars(args).copy()}
    t_all = time.time()
    if args.eval_only:
        net.reg_net_set_params(torch.from_numpy(np.load(args.weights)).cuda())
    else:
        dst = reg.Context(reg.reg_default_params((NET_N,) * 3, nt=1, prec=0))
        t0 = time.time()
        data = register_pairs(list(range(TRAIN_SEED0, TRAIN_SEED0 + args.train)), args.pair_n, args.group, dst)
        val = register_pairs(list(range(VAL_SEED0, VAL_SEED0 + args.val)), args.pair_n, args.group, dst)
        report["registration_seconds"] = time.time() - t0
        net.reg_net_set_params(torch.from_numpy(init_params(args.seed)).cuda())
        report["val_loss_init"] = mean_loss(net, val)
        zero_loss = float(np.mean([float((v.double() ** 2).mean()) for _, _, v in val]))
        report["val_loss_of_zero"] = zero_loss
        t0 = time.time()
        report["history"] = train(net, data, val, args.epochs, args.batch, args.lr, args.seed)
        report["training_seconds"] = time.time() - t0
        w = net.reg_net_get_params().cpu().numpy()
        os.makedirs(os.path.dirname(os.path.abspath(args.weights)), exist_ok=True)
        np.save(args.weights, w)
        log(f"[warmstart] weights written to {args.weights}; val loss {report['history'][-1]['val_loss']:.4e} "
            f"(zero proposal {zero_loss:.4e})")
        del data, val
        torch.cuda.empty_cache()
    if args.test > 0:
        rows = evaluate(net, list(range(TEST_SEED0, TEST_SEED0 + args.test)), args.test_n)
        report["test"] = rows
        report["summary"] = summarize(rows)
        log(f"[warmstart] summary {json.dumps(report['summary'])}")
    report["seconds"] = time.time() - t_all
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    print(json.dumps({k: report[k] for k in report if k in ("summary", "val_loss_init", "val_loss_of_zero",
                                                             "registration_seconds", "training_seconds")}))


if __name__ == "__main__":
    main()
