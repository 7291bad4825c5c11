"""What the trained network gains over the method without it.

The network is trained on the GPU by the library's own kernels (forward,
backward, Adam) on (residual, error) pairs from plain GMRES(30)+BILU0 runs
of eight 64x64x32 systems (ln k ~ N(0,2), seeds 1000-1007), then used as the
FGMRES(30) preconditioner with the BILU0 fallback on held-out systems of the
same recipe (seeds 2000-2003 at 64x64x32, seed 2000 at 128x128x64).  Beside
it, on the same systems: GMRES(30)+BILU0 (the method without the network),
FGMRES(30) with an untrained network, and GMRES(30) without a
preconditioner.  Every preconditioned solve must reach 1e-8 by a residual
the oracle's SpMV recomputes; the steps and times are printed as a table
(the gain may be a loss: the test records it, it does not require a sign).
"""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1602_05901_amd import inputs as I  # noqa: E402
import oracle as O  # noqa: E402

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05901_amd import rsv as R
    R.lib()
    return R


def test_trained_network_against_the_method_without_it(rsv):
    from paper_1602_05901_amd import train as T
    ctx = rsv.Context(0)
    t0 = time.time()
    data, keep = [], []
    for sd in range(1000, 1008):
        sy = T.System(ctx, I.preset("C4", seed=sd))
        R, E, _ = T.harvest(ctx, sy)
        data.append((sy.g, R, E, sy.lnk))
        keep.append(sy)
    net = rsv.Net(ctx, seed=0)
    losses = T.train(ctx, net, data, 600, batch=8, lr=1e-3, seed=0)
    untrained = rsv.Net(ctx, seed=0)
    log(f"trained on {sum(d[1].shape[0] for d in data)} pairs, loss {losses[0]:.3f} -> "
        f"{np.mean(losses[-20:]):.3f} ({time.time() - t0:.1f}s)")
    for sy in keep:
        sy.close()
    held = [I.preset("C4", seed=s) for s in range(2000, 2004)]
    held.append(I.preset("C4", seed=2000).replace(nx=128, ny=128, nz=64))
    runs = [("GMRES(30)+BILU0", dict()),
            ("FGMRES(30)+trained, theta 0.99", dict(net=net, theta=0.99)),
            ("FGMRES(30)+trained, theta 0.9", dict(net=net, theta=0.9)),
            ("FGMRES(30)+untrained, theta 0.99", dict(net=untrained, theta=0.99)),
            ("GMRES(30), no preconditioner", dict(none=True, maxit=500))]
    table = {name: [] for name, _ in runs}
    for cfg in held:
        sy = T.System(ctx, cfg)
        Ao = O.BCSR.from_stencil(cfg.nx, cfg.ny, cfg.nz, I.blocks(cfg))
        bo = sy.b.cpu().numpy()
        for name, kw in runs:
            M = None
            x = torch.zeros_like(sy.b)
            if kw.get("none"):
                st = rsv.solve(sy.A, None, sy.b, x, method=rsv.GMRES, restart=30, tol=1e-8, maxit=kw["maxit"])
            elif "net" in kw:
                M = rsv.Precond(sy.A, type=rsv.PC_LEARNED, net=kw["net"], lnk=sy.lnk, theta=kw["theta"])
                st = rsv.solve(sy.A, M, sy.b, x, method=rsv.FGMRES, restart=30, tol=1e-8, maxit=5000)
            else:
                M = rsv.Precond(sy.A, type=rsv.PC_BILU0)
                st = rsv.solve(sy.A, M, sy.b, x, method=rsv.GMRES, restart=30, tol=1e-8, maxit=5000)
            torch.cuda.synchronize()
            rr = float(np.linalg.norm(bo - Ao.spmv(x.cpu().numpy())) / np.linalg.norm(bo))
            table[name].append((cfg.nx, cfg.seed, st["its"], st["fallbacks"], st["solve_ms"], rr))
            if not kw.get("none"):
                assert st["status"] == rsv.OK and rr <= 1e-8, (name, cfg.seed, st, rr)
            if M is not None:
                M.close()
        sy.close()
    log("| solver | 64x64x32 steps (seeds 2000-2003) | fallbacks | solve ms | 128x128x64 steps | fallbacks | solve ms |")
    log("|---|---|---|---|---|---|---|")
    for name, rows in table.items():
        small = [r for r in rows if r[0] == 64]
        big = [r for r in rows if r[0] == 128][0]
        log(f"| {name} | {' '.join(str(r[2]) for r in small)} | {' '.join(str(r[3]) for r in small)} | "
            f"{np.mean([r[4] for r in small]):.1f} | {big[2]} | {big[3]} | {big[4]:.1f} |")
    net.close(); untrained.close(); ctx.close()
