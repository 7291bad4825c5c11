"""Training and evaluation of the learned preconditioner.

Pairs: from a plain GMRES(30)+BILU0 solve of each training system, the
iterate x_k after k steps is kept at every restart boundary and every 5th
step (and x_0 = 0); the pair is (r_k = b - A x_k, e_k = x_true - x_k), so
A e_k = r_k.  The network learns e ~ s N(r/s, ln k) with s = rms(r)
(user preconditioner hook of the Preconditioners section; the network
replaces the solve step of a user-defined preconditioner inside FGMRES).
Adam with a cosine-decayed learning rate, batch 8, FP32 master weights,
seeded batch order.  Every forward/backward/update runs in the library's
kernels; this module only moves tensors and picks batches.

    python -m paper_1602_05901_amd.train --workload C4 --seeds 1000-1031 \
        --steps 2000 --out net.bin --eval-seeds 2000-2007
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import inputs as I
from . import rsv


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class System:
    """One generated system on the GPU: grid, matrix, b = A x_true, ln k."""

    def __init__(self, ctx, cfg: I.GenConfig):
        import torch
        self.cfg = cfg
        lnk = I.lnk(cfg)
        self.g = rsv.Grid(ctx, cfg.nx, cfg.ny, cfg.nz)
        self.A = rsv.Matrix(self.g, _dev(I.blocks(cfg, lnk)))
        self.xt = _dev(I.x_true(cfg))
        self.b = torch.zeros_like(self.xt)
        self.A.spmv(self.xt, self.b)
        self.lnk = _dev(lnk.astype(np.float32))

    def close(self):
        self.A.close()
        self.g.close()


def harvest(ctx, sysm: System, every=5, restart=30, tol=1e-8, maxit=5000, mode=0):
    """(r_k, e_k) pairs of one system, stacked [P, 3*ncell] on the device.
    mode 1: the pairs the corrector of one BILU0 step learns from,
    (r_k - A t_k, e_k - t_k) with t_k = BILU0^-1 r_k."""
    import torch
    M = rsv.Precond(sysm.A, type=rsv.PC_BILU0)
    x = torch.zeros_like(sysm.b)
    st = rsv.solve(sysm.A, M, sysm.b, x, method=rsv.GMRES, restart=restart, tol=tol, maxit=maxit)
    K = st["its"]
    ks = sorted({0} | set(range(every, K, every)) | set(range(restart, K, restart)))
    rs, es = [], []
    for k in ks:
        x.zero_()
        if k > 0:
            rsv.solve(sysm.A, M, sysm.b, x, method=rsv.GMRES, restart=restart, tol=0.0, maxit=k)
        # r = b - A x and e = x_true - x with the library's product and vector
        # update (the clones only copy memory)
        r = sysm.b.clone()
        sysm.A.spmv(x, r, alpha=-1.0, beta=1.0)
        e = sysm.xt.clone()
        rsv.axpby(ctx, -1.0, x, 1.0, e)
        if mode == 1:
            t = torch.zeros_like(r)
            M.apply(r, t)
            sysm.A.spmv(t, r, alpha=-1.0, beta=1.0)
            rsv.axpby(ctx, -1.0, t, 1.0, e)
        rs.append(r)
        es.append(e)
    M.close()
    return torch.stack(rs), torch.stack(es), K


def cosine_lr(lr, t, steps):
    return lr * 0.5 * (1.0 + math.cos(math.pi * t / max(steps, 1)))


def train(ctx, net, data, steps, batch=8, lr=1e-3, seed=0, log=None):
    """data: list of (grid, R [P,3V], E [P,3V], lnk [V]) with one grid shape.
    Returns the per-step losses."""
    import torch
    rng = np.random.default_rng(seed)
    index = [(s, p) for s, d in enumerate(data) for p in range(d[1].shape[0])]
    g = data[0][0]
    losses = []
    for t in range(steps):
        pick = [index[i] for i in rng.integers(0, len(index), batch)]
        rb = torch.stack([data[s][1][p] for s, p in pick]).contiguous()
        eb = torch.stack([data[s][2][p] for s, p in pick]).contiguous()
        lb = torch.stack([data[s][3] for s, _ in pick]).contiguous()
        losses.append(net.train_step(g, batch, rb, eb, lb, cosine_lr(lr, t, steps)))
        if log and (t % 100 == 0 or t == steps - 1):
            log(f"step {t}: loss {losses[-1]:.4f}")
    return losses


def evaluate(ctx, sysm: System, net=None, restart=30, tol=1e-8, theta=0.99, none=False, maxit=10000, mode=0):
    """FGMRES(30)+net (BILU0 fallback when a column does not reduce the residual
    estimate by theta; theta = inf: the network alone) when net is given;
    GMRES(30) without a preconditioner when none; else GMRES(30)+BILU0."""
    import torch
    if none:
        M, method = None, rsv.GMRES
    elif net is None:
        M = rsv.Precond(sysm.A, type=rsv.PC_BILU0)
        method = rsv.GMRES
    else:
        M = rsv.Precond(sysm.A, type=rsv.PC_LEARNED, net=net, lnk=sysm.lnk, theta=theta, learned_mode=mode)
        method = rsv.FGMRES
    x = torch.zeros_like(sysm.b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = rsv.solve(sysm.A, M, sysm.b, x, method=method, restart=restart, tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    st["solve_s"] = time.perf_counter() - t0
    st["err_vs_xtrue"] = float(torch.linalg.norm(x - sysm.xt) / torch.linalg.norm(sysm.xt))
    if M is not None:
        M.close()
    return st


def _seeds(spec):
    a, b = (int(v) for v in spec.split("-"))
    return list(range(a, b + 1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="C4")
    ap.add_argument("--seeds", default="1000-1031")
    ap.add_argument("--eval-seeds", default="2000-2007")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--net-seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--load", default=None, help="evaluate a saved network instead of training one")
    ap.add_argument("--thetas", default="", help="extra fallback thresholds to evaluate, comma separated")
    ap.add_argument("--mode", type=int, default=0, help="0: the network maps the residual; 1: it corrects one BILU0 step")
    ap.add_argument("--eval-size", default="",
                    help="nx,ny,nz of the held-out systems (the workload's recipe at another size)")
    ap.add_argument("--theta", type=float, default=0.99, help="fallback threshold of the 'learned' runs")
    ap.add_argument("--maxit-alone", type=int, default=3000,
                    help="step limit for the network alone and for no preconditioner")
    args = ap.parse_args(argv)
    args.thetas = [float(t) for t in args.thetas.split(",") if t]

    import torch

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    ctx = rsv.Context(0)
    t0 = time.perf_counter()
    data, nits = [], []
    for s in ([] if args.load else _seeds(args.seeds)):
        sy = System(ctx, I.preset(args.workload, seed=s))
        R, E, K = harvest(ctx, sy, mode=args.mode)
        data.append((sy.g, R, E, sy.lnk))
        nits.append(K)
        sy._keep = sy
    t_h = time.perf_counter() - t0
    npairs = sum(d[1].shape[0] for d in data)
    net = rsv.Net(ctx, seed=args.net_seed)
    untrained = rsv.Net(ctx, seed=args.net_seed)
    if args.load:
        net.load(args.load)
        losses, t_train = [float("nan")], 0.0
    else:
        log(f"harvested {npairs} pairs from {len(data)} systems in {t_h:.1f}s (plain its {np.mean(nits):.1f})")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = train(ctx, net, data, args.steps, args.batch, args.lr, seed=args.net_seed, log=log)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
    if args.out:
        net.save(args.out)
    rows = []
    for s in _seeds(args.eval_seeds):
        cfg = I.preset(args.workload, seed=s)
        if args.eval_size:
            nx, ny, nz = (int(v) for v in args.eval_size.split(","))
            cfg = cfg.replace(nx=nx, ny=ny, nz=nz)
        sy = System(ctx, cfg)
        row = {"seed": s, "grid": [cfg.nx, cfg.ny, cfg.nz]}
        md = args.mode
        th = args.theta
        runs = [("plain", dict()), ("learned", dict(net=net, mode=md, theta=th)),
                ("untrained", dict(net=untrained, mode=md, theta=th)),
                ("learned_only", dict(net=net, theta=float("inf"), maxit=args.maxit_alone, mode=md)),
                ("no_preconditioner", dict(none=True, maxit=args.maxit_alone))]
        runs += [(f"learned_theta_{t}", dict(net=net, theta=t, mode=md)) for t in args.thetas]
        for name, kw in runs:
            st = evaluate(ctx, sy, **kw)
            row[name] = {k: st[k] for k in ("its", "fallbacks", "solve_s", "final_relres", "err_vs_xtrue", "status")}
        rows.append(row)
        log(json.dumps(row))
        sy.close()
    out = {"workload": args.workload, "mode": args.mode, "train_seeds": args.seeds, "pairs": npairs, "harvest_s": t_h,
           "steps": args.steps, "batch": args.batch, "train_s": t_train, "loss_first": losses[0],
           "loss_last": float(np.mean(losses[-20:])), "eval": rows}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
