"""GPU parity of the learned preconditioner's network (BF16 MFMA kernels,
called through the C ABI) against the FP64 U-Net oracle.

Inputs are BF16-exact (activations, weights) so both sides start from the
same values; what remains is FP32 accumulation on the GPU against FP64 in
the oracle.  Bars:
  * one conv layer: |gpu - oracle| <= 2e-5 * (the same sum over |terms|),
    a bound on FP32 summation error at these lengths;
  * whole network vs the oracle with BF16 emulation: relative 2-norm
    <= 2e-3 (a BF16 rounding of an intermediate can flip when FP32 and FP64
    sums straddle a rounding boundary);
  * loss <= 1e-3 relative, gradient <= 3e-2 relative 2-norm (the GPU keeps
    back-propagated activation gradients in BF16, the oracle in FP64);
  * Adam: the GPU update equals the oracle's update of the GPU's own
    gradient to FP32 rounding.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1602_05901_amd import inputs as I  # noqa: E402
import oracle as O  # noqa: E402
from oracle import unet as U  # noqa: E402

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


@pytest.fixture(scope="module")
def ctx(rsv):
    c = rsv.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def bf16_values(seed, stream, n, lo=-1.0, hi=1.0):
    return U.bf16_array(I.uniform(seed, stream, n, lo, hi))


def bf16_bits(v):
    """BF16-exact float64 values -> device int16 tensor of their bit patterns."""
    f = np.asarray(v, np.float32)
    bits = (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return dev(bits.copy())


def layer_layout(c0, c1, c2):
    cin = [4, c0, c0, c1, c1, c2, c2, c1, c1, c0, c0]
    cout = [c0, c0, c1, c1, c2, c2, c1, c1, c0, c0, 3]
    out, off = [], 0
    for l in range(11):
        nw = (27 if l < 10 else 1) * cin[l] * cout[l]
        out.append((off, nw, cout[l], cin[l] * (27 if l < 10 else 1)))
        off += nw + cout[l]
    return out, off


def net_params(seed, ch=(16, 32, 64), bias=0.05):
    """BF16-exact He-uniform weights, small BF16-exact biases."""
    lay, n = layer_layout(*ch)
    p = np.zeros(n)
    for l, (off, nw, co, fan) in enumerate(lay):
        a = np.sqrt(6.0 / fan)
        p[off:off + nw] = U.bf16_array(I.uniform(seed + l, 5, nw, -a, a))
        p[off + nw:off + nw + co] = U.bf16_array(I.uniform(seed + 100 + l, 5, co, -bias, bias))
    return p


# ---------------------------------------------------------------- one layer

# small levels (one voxel block per wave), ragged ones, and two large levels
# (four voxel blocks per wave; the second with a partial last block)
CONV_CASES = [((8, 8, 4), 4, 16), ((8, 8, 4), 16, 16), ((6, 5, 3), 16, 32), ((4, 4, 4), 32, 64),
              ((4, 4, 2), 64, 32), ((5, 3, 7), 64, 64), ((16, 16, 8), 16, 16), ((3, 1, 1), 4, 32),
              ((64, 64, 32), 4, 16), ((65, 45, 45), 16, 32),
              # 8 and 24 input channels (8 per lane of a 16x16x32 MFMA), 12 (4 per lane of a
              # 16x16x16 MFMA), 32 on a grid large enough for the LDS-staged kernel
              ((9, 7, 5), 8, 16), ((10, 9, 8), 24, 64), ((7, 6, 5), 12, 32), ((20, 18, 16), 32, 16)]


@pytest.mark.parametrize("dims,cin,cout", CONV_CASES)
def test_conv3d_forward_parity(rsv, ctx, dims, cin, cout):
    log("conv3d fwd", dims, cin, cout)
    V = dims[0] * dims[1] * dims[2]
    x = bf16_values(1, 5, V * cin)
    w = bf16_values(2, 5, 27 * cin * cout, -0.2, 0.2)
    b = I.uniform(3, 5, cout, -0.5, 0.5).astype(np.float32).astype(np.float64)
    y = torch.zeros(V * cout, dtype=torch.float32, device="cuda")
    rsv.conv3d(ctx, dims, cin, cout, bf16_bits(x), dev(w.astype(np.float32)), dev(b.astype(np.float32)), y)
    ref = U.conv3d(dims, cin, cout, x, w, b)
    bound = U.conv3d(dims, cin, cout, np.abs(x), np.abs(w), np.abs(b))
    err = np.abs(y.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= 2e-5 * bound + 1e-30), float(np.max(err / (bound + 1e-30)))


@pytest.mark.parametrize("dims,cin,cout", CONV_CASES)
def test_conv3d_backward_parity(rsv, ctx, dims, cin, cout):
    log("conv3d bwd", dims, cin, cout)
    V = dims[0] * dims[1] * dims[2]
    x = bf16_values(4, 5, V * cin)
    w = bf16_values(5, 5, 27 * cin * cout, -0.2, 0.2)
    dy = bf16_values(6, 5, V * cout)
    dw = torch.zeros(27 * cin * cout, dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    dx = torch.zeros(V * cin, dtype=torch.float32, device="cuda") if cin % 16 == 0 else None
    rsv.conv3d_bwd(ctx, dims, cin, cout, bf16_bits(x), dev(w.astype(np.float32)), bf16_bits(dy), dx, dw, db)
    rdx, rdw, rdb = U.conv3d_bwd(dims, cin, cout, x, w, dy)
    bdx, bdw, bdb = U.conv3d_bwd(dims, cin, cout, np.abs(x), np.abs(w), np.abs(dy))
    for got, ref, bound in ((dx, rdx, bdx), (dw, rdw, bdw), (db, rdb, bdb)):
        if got is None:
            continue
        err = np.abs(got.cpu().numpy().astype(np.float64) - ref)
        assert np.all(err <= 2e-5 * bound + 1e-30), float(np.max(err / (bound + 1e-30)))


def test_conv3d_rejects_unsupported_channels(rsv, ctx):
    x = torch.zeros(64 * 3, dtype=torch.int16, device="cuda")
    w = torch.zeros(27 * 3 * 16, dtype=torch.float32, device="cuda")
    y = torch.zeros(64 * 16, dtype=torch.float32, device="cuda")
    with pytest.raises(rsv.RsvError):
        rsv.conv3d(ctx, (4, 4, 4), 3, 16, x, w, None, y)
    with pytest.raises(rsv.RsvError):
        rsv.conv3d(ctx, (4, 4, 4), 16, 24, x, w, None, y)


# ---------------------------------------------------------------- whole network

def net_inputs(dims, seed):
    nx, ny, nz = dims
    V = nx * ny * nz
    r = I.uniform(seed, 6, 3 * V, -1.0, 1.0) * 1e-3
    lnk = I.normal(seed, 5, V).astype(np.float32).astype(np.float64) * 2.0
    return r, lnk


@pytest.mark.parametrize("dims", [(8, 8, 4), (16, 16, 8), (12, 8, 4), (4, 4, 4), (32, 32, 8), (36, 20, 12)])
def test_net_forward_parity(rsv, ctx, dims):
    log("net forward", dims)
    ch = (16, 32, 64)
    p = net_params(10)
    r, lnk = net_inputs(dims, 11)
    net = rsv.Net(ctx, *ch)
    net.set_params(p.astype(np.float32))
    g = rsv.Grid(ctx, *dims)
    z = torch.zeros(len(r), dtype=torch.float64, device="cuda")
    net.forward(g, dev(r), dev(lnk.astype(np.float32)), z)
    zg = z.cpu().numpy()
    ze = U.apply(p, r, lnk, dims, ch, emulate=True)
    zx = U.apply(p, r, lnk, dims, ch, emulate=False)
    log("  rel vs emulated", rel(zg, ze), "vs fp64", rel(zg, zx))
    assert rel(zg, ze) <= 2e-3
    assert rel(zg, zx) <= 5e-2
    # the preconditioner object applies the same map (tile-lane path)
    B = I.blocks(I.GenConfig(*dims, I.LNK_IID, 1.0, 0.0, 2.0, 0, 1e3, 1.0, 1))
    A = rsv.Matrix(g, dev(B))
    M = rsv.Precond(A, type=rsv.PC_LEARNED, net=net, lnk=dev(lnk.astype(np.float32)))
    z2 = torch.zeros_like(z)
    M.apply(dev(r), z2)
    assert rel(z2.cpu().numpy(), zg) <= 1e-6
    M.close(); A.close(); g.close(); net.close()


def test_net_rejects_bad_grid(rsv, ctx):
    net = rsv.Net(ctx)
    g = rsv.Grid(ctx, 6, 8, 4)
    r = torch.zeros(3 * 6 * 8 * 4, dtype=torch.float64, device="cuda")
    lnk = torch.zeros(6 * 8 * 4, dtype=torch.float32, device="cuda")
    with pytest.raises(rsv.RsvError):
        net.forward(g, r, lnk, torch.zeros_like(r))
    g.close(); net.close()


@pytest.mark.parametrize("dims", [(8, 8, 4), (32, 16, 8)])
def test_net_loss_grad_parity(rsv, ctx, dims):
    ch, nb = (16, 32, 64), 2
    log("net loss/grad", dims, nb)
    p = net_params(20)
    V = dims[0] * dims[1] * dims[2]
    rs, es, ls = [], [], []
    for b in range(nb):
        r, lnk = net_inputs(dims, 30 + b)
        rs.append(r)
        es.append(I.uniform(40 + b, 6, 3 * V, -1.0, 1.0) * 1e-2)
        ls.append(lnk)
    net = rsv.Net(ctx, *ch)
    net.set_params(p.astype(np.float32))
    g = rsv.Grid(ctx, *dims)
    loss, grad = net.loss_grad(g, nb, dev(np.concatenate(rs)), dev(np.concatenate(es)),
                               dev(np.concatenate(ls).astype(np.float32)))
    lo, go = 0.0, np.zeros(len(p))
    for b in range(nb):
        x0, s = U.prepare(rs[b], ls[b], dims)
        lb, gb = U.loss_grad(p, x0, es[b] / s, dims, ch, emulate=True)
        lo += lb / nb
        go += gb / nb
    log("  loss", loss, lo, "grad rel", rel(grad.astype(np.float64), go))
    assert abs(loss - lo) <= 1e-3 * lo
    assert rel(grad.astype(np.float64), go) <= 3e-2
    # every layer's gradient block, not only the large ones
    lay, _ = layer_layout(*ch)
    for l, (off, nw, co, _) in enumerate(lay):
        blk = slice(off, off + nw + co)
        assert rel(grad[blk].astype(np.float64), go[blk]) <= 5e-2, l
    g.close(); net.close()


def test_adam_steps_match_oracle(rsv, ctx):
    dims, ch, lr = (8, 8, 4), (16, 32, 64), 1e-3
    p0 = net_params(50).astype(np.float32)
    r, lnk = net_inputs(dims, 51)
    e = I.uniform(52, 6, len(r), -1.0, 1.0)
    net = rsv.Net(ctx, *ch)
    net.set_params(p0)
    g = rsv.Grid(ctx, *dims)
    args = (g, 1, dev(r), dev(e), dev(lnk.astype(np.float32)))
    _, g0 = net.loss_grad(*args)
    net.train_step(*args, lr)
    p1 = net.get_params()
    _, g1 = net.loss_grad(*args)
    net.train_step(*args, lr)
    p2 = net.get_params()
    pa, m, v = U.adam(p0.astype(np.float64), g0.astype(np.float64), np.zeros(len(p0)), np.zeros(len(p0)), 1, lr)
    pb, m, v = U.adam(p1.astype(np.float64), g1.astype(np.float64), m, v, 2, lr)
    assert np.max(np.abs(p1 - pa)) <= 2e-6
    assert np.max(np.abs(p2 - pb)) <= 2e-6
    assert np.max(np.abs(p1 - p0)) > 0.5 * lr
    g.close(); net.close()


def test_net_save_load_roundtrip(rsv, ctx, tmp_path):
    net = rsv.Net(ctx, seed=7)
    p = net.get_params()
    assert p.size == U.nparams(16, 32, 64)
    assert np.std(p) > 0
    path = str(tmp_path / "net.bin")
    net.save(path)
    net2 = rsv.Net(ctx, seed=8)
    assert not np.array_equal(net2.get_params(), p)
    net2.load(path)
    assert np.array_equal(net2.get_params(), p)
    small = rsv.Net(ctx, 16, 16, 16)
    with pytest.raises(rsv.RsvError):
        small.load(path)
    net.close(); net2.close(); small.close()


def test_training_reduces_loss(rsv, ctx):
    """A few Adam steps on a fixed batch of (r, e) pairs with A e = r."""
    dims = (16, 16, 8)
    cfg = I.GenConfig(*dims, I.LNK_IID, 2.0, 0.0, 2.0, 0, 1e3, 1.0, 3)
    lnk = I.lnk(cfg)
    B = I.blocks(cfg, lnk)
    g = rsv.Grid(ctx, *dims)
    A = rsv.Matrix(g, dev(B))
    nb, n = 4, 3 * cfg.ncell
    e = torch.stack([dev(I.test_vector(9, n, k)) for k in range(nb)])
    r = torch.zeros_like(e)
    for k in range(nb):
        A.spmv(e[k], r[k])
    lk = dev(np.tile(lnk.astype(np.float32), nb))
    net = rsv.Net(ctx, seed=1)
    losses = [net.train_step(g, nb, r, e, lk, 2e-3) for _ in range(40)]
    log("  losses", losses[0], losses[-1])
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.7 * losses[0]
    A.close(); g.close(); net.close()


# ---------------------------------------------------------------- FGMRES with the learned preconditioner

def test_fgmres_learned_converges_with_fallback(rsv, ctx):
    dims = (16, 16, 8)
    cfg = I.GenConfig(*dims, I.LNK_IID, 1.0, 0.0, 2.0, 0, 1e3, 1.0, 5)
    lnk = I.lnk(cfg)
    B = I.blocks(cfg, lnk)
    Ao = O.BCSR.from_stencil(*dims, B)
    xt = I.x_true(cfg)
    b = Ao.spmv(xt)
    ref = O.gmres(Ao, b, pc=O.ILU(Ao), m=30, tol=1e-8, maxit=1000)
    g = rsv.Grid(ctx, *dims)
    A = rsv.Matrix(g, dev(B))
    for seed, scale in ((1, 1.0), (2, 0.0), (3, np.nan)):
        net = rsv.Net(ctx, seed=seed)
        if scale != 1.0:            # zeroed or NaN weights: every column of a cycle falls back
            net.set_params(np.full(net.num_params, scale, np.float32))
        M = rsv.Precond(A, type=rsv.PC_LEARNED, net=net, lnk=dev(lnk.astype(np.float32)))
        x = torch.zeros(3 * cfg.ncell, dtype=torch.float64, device="cuda")
        st = rsv.solve(A, M, dev(b), x, method=rsv.FGMRES, restart=30, tol=1e-8, maxit=2000)
        log("  fgmres learned", seed, st)
        assert st["status"] == rsv.OK and st["final_relres"] <= 1e-8
        assert rel(x.cpu().numpy(), ref["x"]) <= 1e-6
        if scale != 1.0:
            # same decisions as the oracle's FGMRES with that map and the ILU(0) fallback
            ref0 = O.fgmres(Ao, b, pc=lambda r, v=scale: np.full_like(r, 0.0) * v, fallback=O.ILU(Ao),
                            theta=0.99, m=30, tol=1e-8, maxit=2000)
            assert st["fallbacks"] == ref0["fallbacks"] >= 3
            assert st["its"] == ref0["its"]
        M.close(); net.close()
    A.close(); g.close()


def test_learned_mode1_is_bilu0_step_plus_network_correction(rsv, ctx):
    """learned_mode 1: z = t + s N((r - A t)/s) with t = BILU0^-1 r, checked
    against the same composition through separate calls (BILU0 apply, SpMV,
    network forward)."""
    dims = (16, 16, 8)
    cfg = I.GenConfig(*dims, I.LNK_IID, 1.0, 0.0, 2.0, 0, 1e3, 1.0, 7)
    lnk = I.lnk(cfg)
    g = rsv.Grid(ctx, *dims)
    A = rsv.Matrix(g, dev(I.blocks(cfg, lnk)))
    net = rsv.Net(ctx, seed=4)
    l32 = dev(lnk.astype(np.float32))
    n = 3 * cfg.ncell
    r = dev(I.test_vector(8, n))
    M1 = rsv.Precond(A, type=rsv.PC_LEARNED, net=net, lnk=l32, learned_mode=1)
    z = torch.zeros_like(r)
    M1.apply(r, z)
    B = rsv.Precond(A, type=rsv.PC_BILU0)
    t = torch.zeros_like(r)
    B.apply(r, t)
    r1 = r.clone()
    A.spmv(t, r1, alpha=-1.0, beta=1.0)
    z1 = torch.zeros_like(r)
    net.forward(g, r1, l32, z1)
    corr = (z - t).cpu().numpy()
    assert rel(corr, z1.cpu().numpy()) <= 1e-2
    assert rel(z.cpu().numpy(), (t + z1).cpu().numpy()) <= 1e-3
    with pytest.raises(rsv.RsvError):
        rsv.Precond(A, type=rsv.PC_LEARNED, net=net, lnk=l32, learned_mode=2)
    M1.close(); B.close(); A.close(); g.close(); net.close()


# ---------------------------------------------------------------- FGMRES decisions with accepted and rejected columns

def _robust_decisions(Ao, b, pc_of, F, theta, m=30, tol=1e-8, maxit=500):
    """The oracle's FGMRES decisions (its, fallbacks) with the network map
    pc_of(pert, seed), and whether they survive +-1% per-entry perturbations
    of the network's output (five times the GPU/oracle network difference the
    forward parity test allows): only then can the GPU's be required to be
    equal."""
    outs = [O.fgmres(Ao, b, pc=pc_of(pert, seed), fallback=F, theta=theta, m=m, tol=tol, maxit=maxit)
            for pert, seed in ((0.0, 0), (1e-2, 1), (1e-2, 2), (-1e-2, 3))]
    keys = {(o["its"], o["fallbacks"]) for o in outs}
    return outs[0], len(keys) == 1


def _perturbed(f, pert, seed):
    rng = np.random.default_rng(seed)

    def g(v):
        z = f(v)
        return z * (1.0 + pert * rng.choice([-1.0, 1.0], len(z))) if pert else z
    return g


@pytest.mark.parametrize("mode,thetas", [(0, (0.75, 0.8)), (1, (0.9,))])
def test_fgmres_mixed_decisions_match_oracle(rsv, ctx, mode, thetas):
    """A network that is accepted on some FGMRES columns and rejected on
    others: the identity-weight network (z = v up to BF16 rounding, an
    unpreconditioned column) in mode 0, and the same weights as the
    correction of one BILU0 step in mode 1 (z = t + s N((v - A t)/s),
    t = BILU0^-1 v), whose oracle counterpart is composed here from the
    oracle's ILU(0), SpMV and U-Net.  The oracle's decisions are first shown
    to be stable under +-1% output perturbations; then the GPU's iteration
    and fallback counts must equal them and its solution the oracle's."""
    from cases import identity_unet
    dims = (12, 12, 8)
    cfg = I.GenConfig(*dims, I.LNK_IID, 1.0, 0.0, 2.0, 0, 1e3, 1.0, 5)
    lnk = I.lnk(cfg)
    B = I.blocks(cfg, lnk)
    Ao = O.BCSR.from_stencil(*dims, B)
    b = Ao.spmv(I.x_true(cfg))
    F = O.ILU(Ao)
    p = identity_unet()

    def net_map(v):
        if mode == 0:
            return U.apply(p, v, lnk, dims, emulate=True)
        t = F.apply(v)
        return t + U.apply(p, v - Ao.spmv(t), lnk, dims, emulate=True)

    g = rsv.Grid(ctx, *dims)
    A = rsv.Matrix(g, dev(B))
    net = rsv.Net(ctx)
    net.set_params(p.astype(np.float32))
    checked = 0
    for theta in thetas:
        ref, stable = _robust_decisions(Ao, b, lambda pert, seed: _perturbed(net_map, pert, seed), F, theta)
        log("  mode", mode, "theta", theta, "oracle its", ref["its"], "fallbacks", ref["fallbacks"], "stable", stable)
        if not stable:
            continue
        assert ref["rc"] == O.OK and 0 < ref["fallbacks"] < ref["its"]     # both decisions occur
        M = rsv.Precond(A, type=rsv.PC_LEARNED, net=net, lnk=dev(lnk.astype(np.float32)), theta=theta,
                        learned_mode=mode)
        x = torch.zeros(3 * cfg.ncell, dtype=torch.float64, device="cuda")
        st = rsv.solve(A, M, dev(b), x, method=rsv.FGMRES, restart=30, tol=1e-8, maxit=500)
        log("  gpu its", st["its"], "fallbacks", st["fallbacks"])
        assert st["status"] == rsv.OK
        assert (st["its"], st["fallbacks"]) == (ref["its"], ref["fallbacks"])
        xg = x.cpu().numpy()
        assert np.linalg.norm(b - Ao.spmv(xg)) / np.linalg.norm(b) <= 1e-8
        assert rel(xg, ref["x"]) <= 1e-6
        M.close()
        checked += 1
    assert checked >= 1
    A.close(); g.close(); net.close()
